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


def test_series_byte_models_against_the_built_layout():
    """The per-order algorithmic bytes and the per-launch model bench.py
    reports, against what the host-built device layout of the 250-camera
    workload actually holds (povar_debug_layout_check, no device needed):
    the landmark pass streams 12 bytes per packet entry (packets pad each
    64-lane slot with whole landmarks only), the camera pass 12 bytes per
    camera-major observation (chunked layout: exactly n_obs)."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2405_05079_amd import povar, synth
    prob = synth.workload(2)
    lay = povar.layout_check(prob.cam_idx, prob.pt_idx, prob.meas, prob.n_cams, prob.n_pts, "fp32_bulk")
    assert not lay["blocked"]
    entries = 64 * lay["n_packets"]
    assert prob.n_obs <= entries <= 1.1 * prob.n_obs        # padding of the packet slots
    lp, cp = bench.series_bytes(prob.n_obs, prob.n_pts, prob.n_cams, True)
    # the model's per-observation part is the compulsory stream; the layout's
    # padded entries make the kernel stream at most 10% more
    stream_model = 12 * prob.n_obs
    assert stream_model <= 12 * entries <= 1.1 * stream_model
    assert lp > stream_model and cp > stream_model
    alg = bench.alg_bytes_per_order(prob.n_obs, prob.n_pts, prob.n_cams)
    # one stream of the observations per order, below the two passes' model
    assert 12 * prob.n_obs < alg < lp + cp
    # and below the device arrays the two passes read (entries and camera-major
    # observations, 12 bytes each in FP32-bulk)
    assert alg < 12 * entries + 12 * prob.n_obs + 36 * prob.n_pts + 800 * prob.n_cams + 1
