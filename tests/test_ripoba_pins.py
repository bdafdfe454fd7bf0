"""Pins of the second-stage oracle (projective refinement, RiPoBA) against
what the paper and the mathematics fix, independently of the oracle's own
code paths (CPU only)."""
import numpy as np
import pytest

from oracle import ripoba_oracle as R
from paper_2405_05079_amd import synth


def problem(n_cams=6, n_pts=60, seed=3, sigma=synth.SIGMA, track=("uniform", 3, 5)):
    return synth.make_problem(n_cams, n_pts, track=track, seed=seed, sigma=sigma)


def gt_state(prob):
    """Ground-truth cameras and homogeneous landmarks, each on its sphere."""
    return R.from_first_stage(prob.cams_gt.reshape(prob.n_cams, 12), prob.pts_gt)


def random_state(prob, seed):
    rng = np.random.default_rng(seed)
    P, Xh = gt_state(prob)
    P = P + 0.05 * rng.standard_normal(P.shape)
    Xh = Xh + 0.05 * rng.standard_normal(Xh.shape)
    return P / np.linalg.norm(P, axis=1, keepdims=True), Xh / np.linalg.norm(Xh, axis=1, keepdims=True)


def test_residual_worked_example():
    """(7) by hand: P = [[2,0,0,1],[0,2,0,0],[0,0,1,3]], X = (1,2,1,1):
    P X = (3, 4, 4), pi = (0.75, 1.0); with m = (0.5, 1.25), r = (0.25, -0.25).
    Scaling P and X (both are then put on their unit spheres) leaves r alone."""
    P = np.array([[2, 0, 0, 1, 0, 2, 0, 0, 0, 0, 1, 3]], float)
    X = np.array([[1, 2, 1, 1]], float)
    m = np.array([[0.5, 1.25]])
    idx = np.array([0])
    np.testing.assert_allclose(R.residual(P, X, idx, idx, m), [[0.25, -0.25]], rtol=0, atol=1e-15)
    Pn, Xn = P / np.linalg.norm(P), -3.0 * X / np.linalg.norm(X)
    np.testing.assert_allclose(R.residual(Pn, Xn, idx, idx, m), [[0.25, -0.25]], rtol=0, atol=1e-14)


def test_jacobians_match_central_differences():
    prob = problem(n_cams=3, n_pts=8, seed=5)
    P, Xh = random_state(prob, 6)
    cam, pt, m = prob.cam_idx, prob.pt_idx, prob.meas
    Jp, Jl = R.jacobians(P, Xh, cam, pt)
    h = 1e-6
    for k in range(12):
        E = np.zeros_like(P)
        E[:, k] = h
        fd = (R.residual(P + E, Xh, cam, pt, m) - R.residual(P - E, Xh, cam, pt, m)) / (2 * h)
        np.testing.assert_allclose(Jp[:, :, k], fd, rtol=1e-6, atol=1e-7 * np.abs(Jp).max())
    for k in range(4):
        E = np.zeros_like(Xh)
        E[:, k] = h
        fd = (R.residual(P, Xh + E, cam, pt, m) - R.residual(P, Xh - E, cam, pt, m)) / (2 * h)
        np.testing.assert_allclose(Jl[:, :, k], fd, rtol=1e-6, atol=1e-7 * np.abs(Jl).max())


def test_residual_is_homogeneous_of_degree_zero():
    """pi(a P X) = pi(P X) for any scale a, so each Jacobian block annihilates
    its own variable (Euler): the scale directions are the rank deficiency
    that the tangent spaces of Sec. 4.3 remove."""
    prob = problem(seed=7)
    P, Xh = random_state(prob, 8)
    Jp, Jl = R.jacobians(P, Xh, prob.cam_idx, prob.pt_idx)
    assert np.abs(np.einsum("nri,ni->nr", Jp, P[prob.cam_idx])).max() < 1e-12 * np.abs(Jp).max()
    assert np.abs(np.einsum("nri,ni->nr", Jl, Xh[prob.pt_idx])).max() < 1e-12 * np.abs(Jl).max()
    lin = R.linearize(P, Xh, prob)
    assert np.abs(np.einsum("nij,nj->ni", lin.U, P)).max() < 1e-10 * np.abs(lin.U).max()
    assert np.abs(np.einsum("nij,nj->ni", lin.V, Xh)).max() < 1e-10 * np.abs(lin.V).max()


def dense_tangent_system(prob, P, Xh, lam):
    """The damped Riemannian normal equations built densely from the stacked
    Jacobian (rows of every observation) and explicit tangent bases."""
    n, n_p, n_l = prob.n_obs, prob.n_cams, prob.n_pts
    Jp, Jl = R.jacobians(P, Xh, prob.cam_idx, prob.pt_idx)
    r = R.residual(P, Xh, prob.cam_idx, prob.pt_idx, prob.meas).reshape(-1)
    J = np.zeros((2 * n, 12 * n_p + 4 * n_l))
    for o in range(n):
        i, j = prob.cam_idx[o], prob.pt_idx[o]
        J[2 * o:2 * o + 2, 12 * i:12 * i + 12] = Jp[o]
        J[2 * o:2 * o + 2, 12 * n_p + 4 * j:12 * n_p + 4 * j + 4] = Jl[o]
    Bp, Bl = R.tangent_basis(P), R.tangent_basis(Xh)
    B = np.zeros((12 * n_p + 4 * n_l, 11 * n_p + 3 * n_l))
    for i in range(n_p):
        B[12 * i:12 * i + 12, 11 * i:11 * i + 11] = Bp[i]
    for j in range(n_l):
        B[12 * n_p + 4 * j:12 * n_p + 4 * j + 4, 11 * n_p + 3 * j:11 * n_p + 3 * j + 3] = Bl[j]
    H = J.T @ J
    # Marquardt damping on each camera and landmark block's own diagonal,
    # floored relative to that block, applied in ambient coordinates
    d = np.diag(H).copy()
    for a, b in [(12 * i, 12 * i + 12) for i in range(n_p)] + \
                [(12 * n_p + 4 * j, 12 * n_p + 4 * j + 4) for j in range(n_l)]:
        d[a:b] = np.maximum(d[a:b], 1e-12 * d[a:b].max())
    A = B.T @ (H + lam * np.diag(d)) @ B
    rhs = -B.T @ (J.T @ r)
    return A, rhs, B


@pytest.mark.parametrize("lam", [1e-4, 1e-1, 1.0])
def test_series_and_back_substitution_on_the_joint_riemannian_system(lam):
    """(20)-(29) against the joint damped tangent system built densely from the
    stacked Jacobian: with U~, W~, V~ its blocks, M = U~^-1 W~ V~^-1 W~^T and
    g = b~_p - W~ V~^-1 b~_l, the order-m camera update is the Neumann partial
    sum -(I - M^{m+1}) (I - M)^-1 U~^-1 g and the landmark update is
    -V~^-1 (b~_l + W~^T dx_p).  At lambda = 1 (spectral radius < 0.5 here) a
    long series reaches the direct solution of the joint system; at small
    lambda the 15 directions of the projective gauge (4x4 H up to scale) keep
    eigenvalues of M near 1 - lambda, and only the partial sums are checked."""
    prob = problem(n_cams=5, n_pts=40, seed=11)
    P, Xh = random_state(prob, 12)
    A, rhs, B = dense_tangent_system(prob, P, Xh, lam)
    k = 11 * prob.n_cams
    Ut, Wt, Vt = A[:k, :k], A[:k, k:], A[k:, k:]
    bp, bl = -rhs[:k], -rhs[k:]
    M = np.linalg.solve(Ut, Wt @ np.linalg.solve(Vt, Wt.T))
    g = bp - Wt @ np.linalg.solve(Vt, bl)
    u0 = np.linalg.solve(Ut, g)
    I = np.eye(k)
    rs = R.riemannian_system(P, Xh, R.linearize(P, Xh, prob), lam)
    for m in (0, 1, 4, 20):
        xp = -(I - np.linalg.matrix_power(M, m + 1)) @ np.linalg.solve(I - M, u0)
        xl = -np.linalg.solve(Vt, bl + Wt.T @ xp)
        dxp, dxl = R.series_solve(rs, order=m)
        np.testing.assert_allclose(dxp, xp, rtol=1e-8, atol=1e-10 * np.abs(xp).max())
        np.testing.assert_allclose(dxl, xl, rtol=1e-8, atol=1e-10 * np.abs(xl).max())
    if lam == 1.0:
        direct = np.linalg.solve(A, rhs)
        dxp, dxl = R.series_solve(rs, order=200)
        np.testing.assert_allclose(np.r_[dxp, dxl], direct, rtol=1e-8, atol=1e-10 * np.abs(direct).max())
    # the ambient updates lie in the tangent spaces
    dP, dX = R.back_project(rs, dxp, dxl)
    assert np.abs(np.sum(dP * P, axis=1)).max() < 1e-12 * np.abs(dP).max()
    assert np.abs(np.sum(dX * Xh, axis=1)).max() < 1e-12 * np.abs(dX).max()


@pytest.mark.parametrize("lam", [1e-4, 1e-2, 1.0])
def test_lemma2_spectrum_in_unit_interval(lam):
    """Lemma 2: the eigenvalues of U~^-1 W~ V~^-1 W~^T lie in [0, 1)."""
    prob = problem(n_cams=5, n_pts=40, seed=13)
    P, Xh = random_state(prob, 14)
    rs = R.riemannian_system(P, Xh, R.linearize(P, Xh, prob), lam)
    n = 11 * prob.n_cams
    M = np.stack([rs.apply_M(e) for e in np.eye(n)], axis=1)
    mu = np.linalg.eigvals(M)
    assert np.abs(mu.imag).max() < 1e-8
    assert mu.real.min() > -1e-10 and mu.real.max() < 1.0


def test_noise_free_data_has_a_zero_minimum_the_solver_reaches():
    prob = problem(n_cams=6, n_pts=80, seed=15, sigma=0.0)
    P, Xh = gt_state(prob)
    assert R.cost(P, Xh, prob) < 1e-25
    P0, X0 = random_state(prob, 16)
    res = R.lm_solve(prob, P0, X0, R.Options(max_iters=40, ftol=0.0))
    assert res.cost < 1e-16 * res.cost0
    acc = np.array(res.trace_accept, bool)
    costs = np.array(res.trace_cost)[acc]
    assert np.all(np.diff(costs) < 0)                       # accepted steps strictly decrease
    np.testing.assert_allclose(np.linalg.norm(res.P, axis=1), 1.0, rtol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(res.Xh, axis=1), 1.0, rtol=1e-14)


def test_cost_is_invariant_under_projective_transformations():
    """(7) only sees P_i X_j up to scale: P_i H^-1 and H X_j give the same
    residuals for any invertible 4x4 H."""
    prob = problem(seed=17)
    P, Xh = random_state(prob, 18)
    H = np.random.default_rng(19).standard_normal((4, 4)) + 3 * np.eye(4)
    Ph = np.einsum("nab,bc->nac", P.reshape(-1, 3, 4), np.linalg.inv(H)).reshape(-1, 12)
    Xt = Xh @ H.T
    Ph, Xt = Ph / np.linalg.norm(Ph, axis=1, keepdims=True), Xt / np.linalg.norm(Xt, axis=1, keepdims=True)
    assert abs(R.cost(Ph, Xt, prob) - R.cost(P, Xh, prob)) <= 1e-10 * R.cost(P, Xh, prob)


def test_first_stage_solution_hands_over_to_the_refinement():
    """The stratified pipeline of Sec. 3: PoVar (stage 1, from random cameras)
    then RiPoBA on (7) from its solution; the refinement ends near the noise
    floor of the measurements, sigma^2 per coordinate."""
    from oracle import povar_oracle as O1
    prob = problem(n_cams=8, n_pts=150, seed=21)
    r1 = O1.lm_solve(prob, opts=O1.Options(order=20, max_iters=60, ftol=1e-10))
    P0, Xh0 = R.from_first_stage(r1.P, r1.X)
    res = R.lm_solve(prob, P0, Xh0, R.Options(max_iters=30, ftol=1e-12))
    floor = synth.SIGMA ** 2 * 2 * prob.n_obs
    assert res.cost <= res.cost0
    assert res.cost < 3.0 * floor


@pytest.mark.parametrize("lam", [1e-2, 1.0])
def test_series_early_stop_against_dense_partial_sums(lam):
    """The early stop of Sec. 5.2 (reading R6) on the second stage: the
    stopping term is the first t >= 1 where the t-th Neumann term of the dense
    joint system is at most rtol times the partial sum, and the update equals
    that partial sum."""
    prob = problem(n_cams=5, n_pts=40, seed=11)
    P, Xh = random_state(prob, 12)
    A, rhs, B = dense_tangent_system(prob, P, Xh, lam)
    k = 11 * prob.n_cams
    Ut, Wt, Vt = A[:k, :k], A[:k, k:], A[k:, k:]
    M = np.linalg.solve(Ut, Wt @ np.linalg.solve(Vt, Wt.T))
    g = -rhs[:k] - Wt @ np.linalg.solve(Vt, -rhs[k:])
    x = -np.linalg.solve(Ut, g)
    acc = x.copy()
    rtol = 0.05
    t_ref = 20
    for t in range(1, 21):
        x = M @ x
        acc = acc + x
        if np.linalg.norm(x) <= rtol * np.linalg.norm(acc):
            t_ref = t
            break
    rs = R.riemannian_system(P, Xh, R.linearize(P, Xh, prob), lam)
    info = {}
    dxp, _ = R.series_solve(rs, 20, rtol, info)
    assert info["terms"] == t_ref
    np.testing.assert_allclose(dxp, acc, rtol=1e-8, atol=1e-10 * np.abs(acc).max())
