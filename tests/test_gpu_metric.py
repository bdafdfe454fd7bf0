"""Parity of the metric upgrade on the GPU (``povar_metric_upgrade``, App. D)
with its FP64 oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

from oracle import metric_oracle as MO
from paper_2405_05079_amd import povar, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = povar.Context(0)
    yield c
    c.close()


def say(*a):
    print("[case]", *a, flush=True)


def projective_input(n_cams, seed, noise=0.0):
    """Calibrated cameras through a random projective frame, each with a
    random scale and sign, optionally with relative noise on every entry."""
    G, K = synth.calibrated_cameras(n_cams, seed)
    rng = np.random.default_rng(seed + 100)
    Hp = np.eye(4) + 0.3 * rng.standard_normal((4, 4))
    s = rng.uniform(0.5, 2.0, n_cams) * rng.choice([-1.0, 1.0], n_cams)
    P = s[:, None, None] * (G @ Hp)
    if noise:
        P = P * (1.0 + noise * rng.standard_normal(P.shape))
    return P, K, G


def rel(a, b):
    return np.abs(np.asarray(a) - b).max() / np.abs(b).max()


SIZES = [2, 7, 300, 13700]


@pytest.mark.parametrize("n", SIZES)
def test_reduced_problem_matches_oracle(ctx, n):
    P, K, _ = projective_input(n, 40 + n, noise=1e-3)
    Q, _ = MO.normalized_cameras(P, K)
    for c in (np.zeros(3), np.array([0.3, -0.7, 0.2])):
        say("metric reduced", n, c)
        d = povar.metric_debug_reduced(ctx, P, K, c)
        red = MO.reduced(c, Q, K[0])
        Jm = red.J.reshape(-1, 3)
        assert rel(d["alpha"], red.alpha) < 1e-11
        assert rel(d["JtJ"], Jm.T @ Jm) < 1e-10
        assert rel(d["Jtr"], Jm.T @ red.r.reshape(-1)) < 1e-10
        assert abs(d["cost"] - red.cost) <= 1e-11 * red.cost


@pytest.mark.parametrize("n", SIZES[1:])
def test_upgrade_matches_oracle(ctx, n):
    """Noisy input: the same LM decisions and costs, c, H, the scales and the
    Euclidean cameras.  ftol 1e-8 ends these runs (checked with the oracle:
    every trial cost differs from the current one by more than 1e-12
    relative) before the cost changes at rounding level, where accept/reject
    would be a tie."""
    P, K, _ = projective_input(n, 60 + n, noise=1e-3)
    say("metric upgrade", n)
    g = povar.metric_upgrade(ctx, P, K, max_iters=60, ftol=1e-8)
    ref = MO.lm_solve(P, K, MO.Options(max_iters=60, ftol=1e-8))
    assert list(g["trace_accept"]) == ref.trace_accept
    np.testing.assert_allclose(g["trace_cost"], ref.trace_cost, rtol=1e-9)
    assert abs(g["cost_initial"] - ref.cost0) <= 1e-11 * ref.cost0
    assert abs(g["cost_final"] - ref.cost) <= 1e-9 * ref.cost
    assert g["stop"] in (1, 2)
    np.testing.assert_allclose(g["c"], ref.c, rtol=1e-8, atol=1e-10)
    assert rel(g["H"], ref.H) < 1e-8
    assert rel(g["alpha"], ref.alpha) < 1e-8
    R, t, _ = MO.euclidean_cameras(P, K, ref)
    np.testing.assert_allclose(g["R"], R, rtol=0, atol=1e-8)
    assert rel(g["t"], t) < 1e-8


def test_exact_scene_is_recovered(ctx):
    P, K, G = projective_input(50, 7)
    say("metric exact")
    g = povar.metric_upgrade(ctx, P, K)
    assert g["cost_final"] < 1e-24 * g["cost_initial"]
    B = np.linalg.solve(K, G)
    s = np.cbrt(np.linalg.det(B[:, :, :3]))
    Rg = B[:, :, :3] / s[:, None, None]
    np.testing.assert_allclose(g["R"], Rg @ Rg[0].T, atol=1e-9)
    np.testing.assert_allclose(np.einsum("nab,ncb->nac", g["R"], g["R"]), np.broadcast_to(np.eye(3), g["R"].shape),
                               atol=1e-12)


def test_stratified_pipeline_on_the_gpu(ctx):
    """PoVar, the projective refinement and the metric upgrade, all through the
    library, on a noisy calibrated scene: rotations within 2 degrees."""
    prob = synth.make_problem(8, 150, seed=21, calibrated=True, track=("uniform", 3, 5))
    say("metric pipeline")
    s1 = povar.Problem.from_synth(ctx, prob, precision="fp64", max_iters=60, ftol=1e-10)
    s1.solve()
    P1, X1 = s1.cameras(), s1.points()
    s1.close()
    unit = lambda a: a / np.linalg.norm(a, axis=1, keepdims=True)
    s2 = povar.Problem.refine(ctx, prob.n_cams, prob.n_pts, prob.cam_idx, prob.pt_idx, prob.meas, unit(P1),
                              unit(np.c_[X1, np.ones(len(X1))]), max_iters=30, ftol=1e-12)
    s2.solve()
    P2 = s2.cameras()
    s2.close()
    g = povar.metric_upgrade(ctx, P2, prob.K_gt)
    B = np.linalg.solve(prob.K_gt, prob.cams_gt.reshape(-1, 3, 4))
    Rg = B[:, :, :3] / np.cbrt(np.linalg.det(B[:, :, :3]))[:, None, None]
    cosang = (np.einsum("nab,nab->n", g["R"], Rg @ Rg[0].T) - 1.0) / 2.0
    assert np.degrees(np.arccos(np.clip(cosang, -1.0, 1.0))).max() < 2.0


def test_no_iteration_and_invalid_input(ctx):
    P, K, _ = projective_input(7, 3, noise=1e-3)
    say("metric edge cases")
    g = povar.metric_upgrade(ctx, P, K, max_iters=0)
    Q, _ = MO.normalized_cameras(P, K)
    f0 = MO.reduced(np.zeros(3), Q, K[0]).cost
    assert g["iters"] == 0 and g["stop"] == 0
    assert abs(g["cost_final"] - f0) <= 1e-12 * f0 and g["cost_initial"] == g["cost_final"]
    np.testing.assert_array_equal(g["c"], 0.0)
    bad = []
    bad.append((P[:1], K[:1]))                          # a single camera
    Kl = K.copy()
    Kl[2, 1, 0] = 0.1                                   # not upper triangular
    bad.append((P, Kl))
    Kz = K.copy()
    Kz[1, 1, 1] = 0.0                                   # zero on the diagonal
    bad.append((P, Kz))
    Pn = P.copy()
    Pn[3, 1, 2] = np.nan
    bad.append((Pn, K))
    Ps = P.copy()
    Ps[0, :, :3] = np.outer([1.0, 2.0, 3.0], [1.0, 0.5, 0.25])   # reference camera singular
    bad.append((Ps, K))
    for Pb, Kb in bad:
        with pytest.raises(povar.PovarError) as e:
            povar.metric_upgrade(ctx, Pb, Kb)
        assert e.value.status == povar.EINVAL
    for kw in (dict(max_iters=-1), dict(ftol=1.0)):
        with pytest.raises(povar.PovarError):
            povar.metric_upgrade(ctx, P, K, **kw)
