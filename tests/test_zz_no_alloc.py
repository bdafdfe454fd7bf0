"""povar_metric_upgrade_noalloc, the metric upgrade for callers that cannot
allocate device memory: it must give what povar_metric_upgrade gives (the
same kernels on the same inputs: bitwise), also on a second call in a row
with a smaller input, whose buffers sit where the first call's were; and it
must refuse a call larger than its scratch with a clear error."""
import numpy as np
import pytest

from paper_2405_05079_amd import povar, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


def projective_input(n_cams, seed, noise=1e-3):
    G, K = synth.calibrated_cameras(n_cams, seed)
    rng = np.random.default_rng(seed + 100)
    Hp = np.eye(4) + 0.3 * rng.standard_normal((4, 4))
    s = rng.uniform(0.5, 2.0, n_cams) * rng.choice([-1.0, 1.0], n_cams)
    return s[:, None, None] * (G @ Hp) * (1.0 + noise * rng.standard_normal((n_cams, 3, 4))), K


KEYS = ("H", "c", "alpha", "R", "t", "trace_cost", "trace_accept", "iters", "cost_initial", "cost_final",
        "lambda_", "stop")


def test_noalloc_metric_upgrade_equals_the_allocating_call():
    with povar.Context(0) as ctx:
        for n, seed in ((13700, 71), (300, 72), (7, 73)):   # each call smaller than the one before
            say("no-alloc metric upgrade", n)
            P, K = projective_input(n, seed)
            ref = povar.metric_upgrade(ctx, P, K, max_iters=60, ftol=1e-12)
            got = povar.metric_upgrade(ctx, P, K, max_iters=60, ftol=1e-12, noalloc=True)
            for k in KEYS:
                np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
            assert got["iters"] > 0
        # beyond the scratch: refused, and the next call still works
        P, K = projective_input(30000, 74)
        with pytest.raises(povar.PovarError) as e:
            povar.metric_upgrade(ctx, P, K, max_iters=10, noalloc=True)
        assert e.value.status == povar.EINVAL and "scratch" in str(e.value)
        P, K = projective_input(50, 75)
        ref = povar.metric_upgrade(ctx, P, K, max_iters=20)
        got = povar.metric_upgrade(ctx, P, K, max_iters=20, noalloc=True)
        for k in KEYS:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
