"""bench.py contract checks that need no GPU: the one-GPU refusal and the
algorithmic byte model of the series passes."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_series_byte_model():
    """Per launch: landmark pass (4 + 2s) n_obs + (6s + 48) n_l + 21s n_p,
    camera pass (4 + 2s) n_obs + 6s n_l + (1344 + 21s) n_p, s = 4 or 8."""
    sys.path.insert(0, ROOT)
    import bench
    for fp32, s in ((True, 4), (False, 8)):
        lp, cp = bench.series_bytes(1000, 200, 10, fp32)
        assert lp == (4 + 2 * s) * 1000 + (6 * s + 48) * 200 + 21 * s * 10
        assert cp == (4 + 2 * s) * 1000 + 6 * s * 200 + (1344 + 21 * s) * 10
