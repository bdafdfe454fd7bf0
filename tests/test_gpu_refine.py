"""Parity of the second-stage HIP path (projective refinement with RiPoBA,
objective (7) and Sec. 4.3) with its FP64 oracle (needs an MI355X).

Every comparison goes through the C ABI.  FP64 throughout: rounding-level
agreement (1e-10 relative on the blocks, 1e-8 on steps through a 12x12
inverse and up to 20 series terms)."""
import numpy as np
import pytest

from oracle import ripoba_oracle as R
from paper_2405_05079_amd import povar, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = povar.Context(0)
    yield c
    c.close()


def say(*a):
    print("[case]", *a, flush=True)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def start(prob, seed, noise=0.05):
    """Ground truth perturbed, cameras and homogeneous landmarks on their spheres."""
    rng = np.random.default_rng(seed)
    P, X = R.from_first_stage(prob.cams_gt.reshape(prob.n_cams, 12), prob.pts_gt)
    P = P + noise * rng.standard_normal(P.shape)
    X = X + noise * rng.standard_normal(X.shape)
    return P / np.linalg.norm(P, axis=1, keepdims=True), X / np.linalg.norm(X, axis=1, keepdims=True)


def refine(ctx, prob, P, X, **opts):
    return povar.Problem.refine(ctx, prob.n_cams, prob.n_pts, prob.cam_idx, prob.pt_idx, prob.meas, P, X, **opts)


# ragged packets, cameras over several 2048-observation chunks, landmarks with
# more than 64 observations (their own packet slots)
CASES = [
    dict(n_cams=6, n_pts=60, seed=3, track=("uniform", 3, 5)),
    dict(n_cams=7, n_pts=1000, seed=6, track=("uniform", 3, 6)),
    dict(n_cams=30, n_pts=129, seed=7, track=("geom", 0.25)),
    dict(n_cams=100, n_pts=50, seed=21, track=("uniform", 60, 90)),
    dict(n_cams=2, n_pts=5000, seed=22, track=("uniform", 2, 2)),
    # 70,000 landmarks: 64-byte (z, X) records above 4 MB, so the camera pass
    # runs over landmark-blocked camera slots and adds each camera's runs
    dict(n_cams=40, n_pts=70000, seed=23, track=("uniform", 2, 3)),
    # blocked, with heavy-tailed views per camera (Zipf): cameras with many runs
    dict(n_cams=300, n_pts=70000, seed=24, track=("uniform", 2, 3), cam_choice="zipf"),
    # cameras of up to 11 chunks (Zipf views, 100k observations): each
    # camera's linearisation partials added by one wave per camera
    dict(n_cams=12, n_pts=40000, seed=36, track=("uniform", 2, 3), cam_choice="zipf"),
]
IDS = ["small", "7-cameras", "ragged", "long-tracks", "3-chunk-cameras", "blocked", "blocked-zipf", "wave-sums"]


@pytest.mark.parametrize("lam", [1e-3, 1.0])
@pytest.mark.parametrize("kw", CASES, ids=IDS)
def test_refine_blocks(ctx, kw, lam):
    prob = synth.make_problem(**kw)
    P, X = start(prob, 5)
    say("refine blocks", kw, lam)
    gp = refine(ctx, prob, P, X)
    try:
        assert gp.layout()["blocked"] == (prob.n_pts >= 70000)
        d = gp.refine_blocks(lam)
        lin = R.linearize(P, X, prob)
        rs = R.riemannian_system(P, X, lin, lam)
        G = np.einsum("nai,nij,nbj->nab", rs.Bl, np.linalg.inv(rs.Vt), rs.Bl)
        assert rel(d["U"], lin.U) < 1e-10
        assert rel(d["bp"], lin.bp) < 1e-10
        assert rel(d["bl"], lin.bl) < 1e-10
        assert rel(d["G"], G) < 1e-9
        assert abs(d["cost"] - lin.cost) / lin.cost < 1e-12
        np.testing.assert_allclose(gp.points_h(), X, rtol=0, atol=1e-15)
    finally:
        gp.close()


@pytest.mark.parametrize("lam,order", [(1e-3, 0), (1e-2, 10), (1.0, 20)])
@pytest.mark.parametrize("kw", CASES, ids=IDS)
def test_refine_step(ctx, kw, lam, order):
    prob = synth.make_problem(**kw)
    P, X = start(prob, 8)
    say("refine step", kw, lam, order)
    gp = refine(ctx, prob, P, X)
    try:
        dp, pt, xt, ct = gp.refine_step(lam, order)
        lin = R.linearize(P, X, prob)
        dP, dX = R.step(P, X, lin, lam, order)
        Pn, Xn = R.retract(P, dP), R.retract(X, dX)
        assert rel(dp, dP) < 1e-8
        assert rel(pt, Pn) < 1e-9
        assert rel(xt, Xn) < 1e-9
        assert abs(ct - R.cost(Pn, Xn, prob)) / R.cost(Pn, Xn, prob) < 1e-8
    finally:
        gp.close()


@pytest.mark.parametrize("lam", [10.0, 1.0, 1e-2])
def test_refine_series_early_stop(ctx, lam):
    """series_rtol = 0.01 on the second stage: the oracle stops after 2, 4 and
    all 20 terms at these dampings, each decision at least 30% away from the
    threshold (ratios 0.0149 -> 0.0005, 0.0151 -> 0.0067, >= 0.0134 to the
    end), so rounding cannot flip one; the step taken must be the same."""
    prob = synth.make_problem(**CASES[4])
    P, X = start(prob, 8)
    say("refine early stop", lam)
    gp = refine(ctx, prob, P, X, series_rtol=0.01)
    try:
        dp, pt, xt, ct = gp.refine_step(lam, 20)
        lin = R.linearize(P, X, prob)
        info = {}
        dP, dX = R.step(P, X, lin, lam, 20, 0.01, info)
        assert info["terms"] == {10.0: 2, 1.0: 4, 1e-2: 20}[lam]
        assert rel(dp, dP) < 1e-8
        assert rel(xt, R.retract(X, dX)) < 1e-9
    finally:
        gp.close()


def test_refine_landmarks_at_infinity(ctx):
    """Homogeneous landmarks with w = 0 (points at infinity, which the unit
    sphere of R^4 represents like any other point): blocks and a step as the
    oracle computes them; nothing on the path divides by w."""
    prob = synth.make_problem(**CASES[2])
    P, X = start(prob, 11)
    X = X.copy()
    X[:10, 3] = 0.0
    X[:10] /= np.linalg.norm(X[:10], axis=1, keepdims=True)
    say("refine landmarks at infinity")
    gp = refine(ctx, prob, P, X)
    try:
        d = gp.refine_blocks(1e-2)
        lin = R.linearize(P, X, prob)
        assert rel(d["U"], lin.U) < 1e-10
        assert rel(d["bl"], lin.bl) < 1e-10
        dp, pt, xt, ct = gp.refine_step(1e-2, 10)
        dP, dX = R.step(P, X, lin, 1e-2, 10)
        assert rel(dp, dP) < 1e-8
        # the landmark update is -G_j (b_l + sum W^T dp): the camera step's
        # rounding (<= 1e-8) comes through G_j, which is badly conditioned for
        # these landmarks (measured 1.0e-8)
        assert rel(xt, R.retract(X, dX)) < 1e-7
        np.testing.assert_allclose(gp.points_h()[:10, 3], 0.0, atol=0)
    finally:
        gp.close()


def test_refine_trajectory_matches_oracle(ctx):
    prob = synth.make_problem(**CASES[2])
    P, X = start(prob, 9)
    say("refine trajectory")
    gp = refine(ctx, prob, P, X, order=20, max_iters=15, ftol=0.0)
    try:
        rep = gp.solve()
        cost, lam, acc = gp.trace()
        ref = R.lm_solve(prob, P, X, R.Options(order=20, max_iters=15, ftol=0.0))
        # identical decisions; costs to rounding of the trajectory (they fall
        # 300x from the start, and differences of 1e-11 absolute are 4e-8 there)
        assert list(acc) == ref.trace_accept
        np.testing.assert_allclose(cost, ref.trace_cost, rtol=1e-6)
        assert abs(rep["cost_final"] - ref.cost) <= 1e-6 * ref.cost
        # cameras and landmarks are fixed only up to the projective gauge (a 4x4
        # H moves both without changing the cost), so compare what the gauge
        # leaves alone: every predicted image point pi(P_i X_j)
        zero = np.zeros_like(prob.meas)
        y_gpu = R.residual(gp.cameras(), gp.points_h(), prob.cam_idx, prob.pt_idx, zero)
        y_ref = R.residual(ref.P, ref.Xh, prob.cam_idx, prob.pt_idx, zero)
        np.testing.assert_allclose(y_gpu, y_ref, rtol=0, atol=1e-8)
    finally:
        gp.close()


def test_first_stage_then_refinement_and_graph_replay(ctx):
    """The stratified pipeline on the GPU: PoVar from random cameras, then the
    refinement from its solution reaches the noise floor of the measurements;
    graph replays of the refinement equal direct launches bitwise."""
    prob = synth.make_problem(8, 150, track=("uniform", 3, 5), seed=21)
    say("pipeline")
    s1 = povar.Problem.from_synth(ctx, prob, precision="fp64", max_iters=60, ftol=1e-10)
    s1.solve()
    P1, X1 = s1.cameras(), s1.points()
    s1.close()
    P, X = R.from_first_stage(P1, X1)
    a = refine(ctx, prob, P, X, max_iters=30, ftol=1e-12)
    b = refine(ctx, prob, P, X, max_iters=30, ftol=1e-12, use_graph=False)
    try:
        for _ in range(3):
            a.step(5)
            b.step(5)
            np.testing.assert_array_equal(a.cameras(), b.cameras())
            np.testing.assert_array_equal(a.points_h(), b.points_h())
        rep = a.solve()
        assert rep["cost_final"] <= rep["cost_initial"]
        assert rep["cost_final"] < 3.0 * synth.SIGMA ** 2 * 2 * prob.n_obs
        Xe = a.points()
        Xh = a.points_h()
        np.testing.assert_allclose(Xe, Xh[:, :3] / Xh[:, 3:], rtol=1e-12)
    finally:
        a.close()
        b.close()


def test_refine_rejects_invalid_use(ctx):
    prob = synth.make_problem(**CASES[0])
    P, X = start(prob, 10)
    say("refine invalid")
    for opts in (dict(precision="fp32_bulk"), dict(manifold="euclidean"), dict(series_rtol=1.5)):
        with pytest.raises(povar.PovarError) as e:
            refine(ctx, prob, P, X, **opts)
        assert e.value.status == povar.EINVAL
    bad = X.copy()
    bad[3, 1] = np.nan
    with pytest.raises(povar.PovarError):
        refine(ctx, prob, P, bad)
    gp = refine(ctx, prob, P, X)
    try:
        with pytest.raises(povar.PovarError) as e:
            gp.debug_step(1e-3, 5)
        assert e.value.status == povar.ESTATE
    finally:
        gp.close()
    s1 = povar.Problem.from_synth(ctx, prob)
    try:
        with pytest.raises(povar.PovarError) as e:
            s1.refine_step(1e-3, 5)
        assert e.value.status == povar.ESTATE
        np.testing.assert_allclose(s1.points_h()[:, 3], 1.0)
    finally:
        s1.close()


def rel_rows(a, b):
    a, b = np.asarray(a).reshape(len(a), -1), np.asarray(b).reshape(len(b), -1)
    return (np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)).max()


@pytest.mark.parametrize("lam", [1e-8, 1e-10, 1e-12])
@pytest.mark.parametrize("kw", [CASES[0], CASES[1], CASES[5]], ids=["small", "7-cameras", "blocked"])
def test_refine_blocks_and_steps_at_small_damping(ctx, kw, lam):
    """The damped landmark and camera blocks are singular along their own
    point up to lambda; their tangent-space inverses, formed in an explicit
    basis, must keep rounding-level agreement with the oracle's (which inverts
    B^T V B in an explicit basis too) down to the smallest damping: every
    landmark's G_j and every camera's step."""
    prob = synth.make_problem(**kw)
    P, X = start(prob, 9)
    say("refine small damping", kw, lam)
    gp = refine(ctx, prob, P, X)
    try:
        d = gp.refine_blocks(lam)
        lin = R.linearize(P, X, prob)
        rs = R.riemannian_system(P, X, lin, lam)
        G = np.einsum("nai,nij,nbj->nab", rs.Bl, np.linalg.inv(rs.Vt), rs.Bl)
        assert rel_rows(d["G"], G) < 1e-9, rel_rows(d["G"], G)
        for order in (0, 10):
            dp, pt, xt, ct = gp.refine_step(lam, order)
            dP, dX = R.step(P, X, lin, lam, order)
            Pn, Xn = R.retract(P, dP), R.retract(X, dX)
            assert rel(dp, dP) < 1e-8, (order, rel(dp, dP))
            assert rel(xt, Xn) < 1e-9
            assert abs(ct - R.cost(Pn, Xn, prob)) / R.cost(Pn, Xn, prob) < 1e-8
    finally:
        gp.close()
