"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formulas: each one compares the oracle
with a worked example derived by hand, a finite-difference derivative, a
library least-squares / Cholesky solve of an explicitly formed dense system, a
closed form of the Neumann partial sum (Proposition 1), the spectral statement
of Lemma 1, a geometric invariant, or a known zero minimum.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import povar_oracle as O
from paper_2405_05079_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(n_cams=5, n_pts=40, seed=7, eta=0.01, track=("uniform", 3, 5), **kw):
    return synth.make_problem(n_cams, n_pts, track=track, seed=seed, eta=eta, **kw)


class _Obs:
    """A problem with a single observation, for per-observation checks."""
    def __init__(self, P, X, m, eta):
        self.n_cams, self.n_pts = 1, 1
        self.cam_idx = np.zeros(1, np.int32)
        self.pt_idx = np.zeros(1, np.int32)
        self.meas = np.asarray(m, float).reshape(1, 2)
        self.eta = eta


# --------------------------------------------------------------------------- residual (6)
def test_residual_matches_hand_worked_examples():
    cases = json.load(open(os.path.join(GOLDEN, "pose_residual_worked_example.json")))["cases"]
    for c in cases:
        P = np.asarray(c["camera_row_major"], float).reshape(1, 12)
        X = np.asarray(c["point"], float).reshape(1, 3)
        p = _Obs(P, X, c["meas"], c["eta"])
        r = O.pose_residual(P, X, p.cam_idx, p.pt_idx, p.meas, p.eta)[0]
        np.testing.assert_allclose(r, c["residual"], rtol=1e-14, atol=1e-15)
        assert abs(O.cost(P, X, p) - c["residual_sq_norm"]) < 1e-12


def test_residual_special_cases_eta():
    """eta = 1: only the affine reprojection error remains; eta = 0: only the OSE rows."""
    rng = np.random.default_rng(1)
    P = rng.standard_normal((1, 12)); X = rng.standard_normal((1, 3)); m = rng.standard_normal(2)
    C = P.reshape(3, 4); xh = np.r_[X[0], 1.0]; y = C @ xh
    p = _Obs(P, X, m, 1.0)
    r = O.pose_residual(P, X, p.cam_idx, p.pt_idx, p.meas, 1.0)[0]
    np.testing.assert_allclose(r, [0, 0, y[0] - m[0], y[1] - m[1]], atol=1e-14)
    r0 = O.pose_residual(P, X, p.cam_idx, p.pt_idx, p.meas, 0.0)[0]
    np.testing.assert_allclose(r0, [y[0] - m[0] * y[2], y[1] - m[1] * y[2], 0, 0], atol=1e-14)


def test_known_zero_minimum_for_noise_free_affine_cameras():
    """Affine cameras (third row (0,0,0,1)) and exact measurements: the ground
    truth is a zero-cost minimum of (6) for every eta, and the closed form (8)
    recovers the true points."""
    prob = synth.make_problem(6, 50, track=("uniform", 3, 5), seed=3, sigma=0.0, affine=True)
    P = prob.cams_gt
    assert O.cost(P, prob.pts_gt, prob) < 1e-25
    X, _ = O.solve_landmarks(P, prob)
    np.testing.assert_allclose(X, prob.pts_gt, atol=1e-10)
    assert O.reduced_cost(P, prob) < 1e-20


# --------------------------------------------------------------------------- Jacobians
def test_jacobians_match_central_differences():
    prob = tiny()
    rng = np.random.default_rng(2)
    P = rng.standard_normal((prob.n_cams, 12)); X = rng.standard_normal((prob.n_pts, 3))
    Jp, Jl = O.pose_jacobians(P, X, prob.cam_idx, prob.pt_idx, prob.meas, prob.eta)
    h = 1e-3   # the residual is affine in every single parameter: central FD is exact
    res = lambda P_, X_: O.pose_residual(P_, X_, prob.cam_idx, prob.pt_idx, prob.meas, prob.eta)
    for q in range(12):
        dP = np.zeros_like(P); dP[:, q] = h
        fd = (res(P + dP, X) - res(P - dP, X)) / (2 * h)
        np.testing.assert_allclose(Jp[:, :, q], fd, atol=1e-10)
    for q in range(3):
        dX = np.zeros_like(X); dX[:, q] = h
        fd = (res(P, X + dX) - res(P, X - dX)) / (2 * h)
        np.testing.assert_allclose(Jl[:, :, q], fd, atol=1e-10)


# --------------------------------------------------------------------------- closed form (8)
def _stacked_landmark_system(P, prob, j):
    """Rows of the residual of landmark j as an affine map A X - b, found by
    evaluating the residual at X = 0 and at the unit vectors."""
    sel = np.nonzero(prob.pt_idx == j)[0]
    cam, meas = prob.cam_idx[sel], prob.meas[sel]
    pt = np.zeros(sel.shape[0], np.int32)
    r = lambda x: O.pose_residual(P, x.reshape(1, 3), cam, pt, meas, prob.eta).ravel()
    r0 = r(np.zeros(3))
    A = np.stack([r(e) - r0 for e in np.eye(3)], axis=1)
    return A, -r0


def test_closed_form_landmarks_equal_lstsq_and_zero_gradient():
    prob = tiny(n_pts=25)
    P = synth.init_cameras(prob.n_cams, 11)
    X, _ = O.solve_landmarks(P, prob)
    for j in range(prob.n_pts):
        A, b = _stacked_landmark_system(P, prob, j)
        x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
        np.testing.assert_allclose(X[j], x_ls, rtol=1e-9, atol=1e-9)
    lin = O.linearize(P, X, prob)
    scale = np.abs(lin.V).max() * np.abs(X).max()
    assert np.abs(lin.bl).max() < 1e-12 * scale


def test_singular_landmark_block_gives_minimum_norm_solution():
    """One observation at m = 0: N = diag(1,1,0) makes V rank 2.  The
    pseudo-inverse must return the minimum-norm least-squares point."""
    rng = np.random.default_rng(5)
    P = rng.standard_normal((1, 12))
    p = _Obs(P, np.zeros((1, 3)), [0.0, 0.0], 0.01)
    X, Vp = O.solve_landmarks(P, p)
    A, b = _stacked_landmark_system(P, p, 0)
    assert np.linalg.matrix_rank(A) == 2
    np.testing.assert_allclose(X[0], np.linalg.lstsq(A, b, rcond=None)[0], atol=1e-12)
    np.testing.assert_allclose(Vp[0], np.linalg.pinv(A.T @ A), atol=1e-10)


# --------------------------------------------------------------------------- reduced gradient
def test_envelope_theorem_reduced_gradient_is_twice_bp():
    """d f*/d p = 2 J_p^T r at x_l*(p): the landmark term drops out because b_l = 0."""
    prob = tiny(n_cams=4, n_pts=30)
    P = synth.init_cameras(prob.n_cams, 12)
    X, _ = O.solve_landmarks(P, prob)
    lin = O.linearize(P, X, prob)
    h = 1e-6
    for i in range(prob.n_cams):
        for q in (0, 5, 11):
            dP = np.zeros_like(P); dP[i, q] = h
            fd = (O.reduced_cost(P + dP, prob) - O.reduced_cost(P - dP, prob)) / (2 * h)
            assert abs(fd - 2 * lin.bp[i, q]) <= 1e-6 * max(1.0, abs(fd))


# --------------------------------------------------------------------------- dense references
def _dense_problem(prob, P, lam, manifold="sphere"):
    """Explicit dense J = [J_p B | J_l] of the whole problem and the damped joint
    normal equations, built without the oracle's assembly code."""
    X, _ = O.solve_landmarks(P, prob)
    Jp, Jl = O.pose_jacobians(P, X, prob.cam_idx, prob.pt_idx, prob.meas, prob.eta)
    r = O.pose_residual(P, X, prob.cam_idx, prob.pt_idx, prob.meas, prob.eta).ravel()
    n, nc, npt = prob.n_obs, prob.n_cams, prob.n_pts
    if manifold == "sphere":
        Bs = [sla.null_space(P[i][None, :]) for i in range(nc)]       # SVD-based basis
    else:
        Bs = [np.eye(12) for _ in range(nc)]
    k = Bs[0].shape[1]
    JP = np.zeros((4 * n, k * nc)); JL = np.zeros((4 * n, 3 * npt)); JPa = np.zeros((4 * n, 12 * nc))
    for o in range(n):
        i, j = prob.cam_idx[o], prob.pt_idx[o]
        JPa[4 * o:4 * o + 4, 12 * i:12 * i + 12] = Jp[o]
        JP[4 * o:4 * o + 4, k * i:k * i + k] = Jp[o] @ Bs[i]
        JL[4 * o:4 * o + 4, 3 * j:3 * j + 3] = Jl[o]
    Ua = JPa.T @ JPa
    damp = np.zeros(12 * nc)
    for i in range(nc):
        d = np.diag(Ua)[12 * i:12 * i + 12]
        damp[12 * i:12 * i + 12] = np.maximum(d, 1e-12 * d.max())
    Bd = sla.block_diag(*Bs)
    Ut = JP.T @ JP + lam * Bd.T @ np.diag(damp) @ Bd
    W = JP.T @ JL
    V = JL.T @ JL
    bp, bl = JP.T @ r, JL.T @ r
    return dict(Ut=Ut, W=W, V=V, bp=bp, bl=bl, Bd=Bd, k=k, JP=JP, JL=JL, r=r)


@pytest.mark.parametrize("manifold", ["sphere", "euclidean"])
def test_series_converges_to_joint_and_schur_cholesky_solves(manifold):
    prob = tiny(n_cams=4, n_pts=30, seed=21)
    P = synth.init_cameras(prob.n_cams, 22)
    lam = 1.0
    D = _dense_problem(prob, P, lam, manifold)
    # joint damped system (10) with only the camera block damped, dense least squares
    K = np.block([[D["Ut"], D["W"]], [D["W"].T, D["V"]]])
    rhs = -np.r_[D["bp"], D["bl"]]
    sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
    dx_joint = D["Bd"] @ sol[:D["Ut"].shape[0]]
    # explicit Schur complement (14)-(15) solved by Cholesky
    Vp = np.linalg.pinv(D["V"], rcond=1e-12, hermitian=True)
    S = D["Ut"] - D["W"] @ Vp @ D["W"].T
    rhs_s = -(D["bp"] - D["W"] @ Vp @ D["bl"])
    c = sla.cho_factor(S)
    dx_schur = D["Bd"] @ sla.cho_solve(c, rhs_s)
    np.testing.assert_allclose(dx_schur, dx_joint, rtol=1e-8, atol=1e-10)
    # oracle: series of high order
    X, _ = O.solve_landmarks(P, prob)
    lin = O.linearize(P, X, prob)
    dP = O.camera_step(P, lin, lam, order=600, manifold=manifold)
    np.testing.assert_allclose(dP.ravel(), dx_schur, rtol=1e-7, atol=1e-9 * np.abs(dx_schur).max())


def test_series_partial_sums_match_neumann_closed_form_and_bound():
    """Proposition 1 with M = U~^-1 W~ V^+ W~^T: the order-m sum equals
    -(I - M^{m+1}) (I - M)^-1 U~^-1 g, and its U~-norm error is bounded by
    mu_max^{m+1} ||x*||_U (Lemma 1: M is U~-self-adjoint with spectrum in [0,1))."""
    prob = tiny(n_cams=4, n_pts=30, seed=31)
    P = synth.init_cameras(prob.n_cams, 32)
    lam = 0.3
    D = _dense_problem(prob, P, lam)
    Ut, W, V = D["Ut"], D["W"], D["V"]
    Vp = np.linalg.pinv(V, rcond=1e-12, hermitian=True)
    M = np.linalg.solve(Ut, W @ Vp @ W.T)
    g = D["bp"] - W @ Vp @ D["bl"]
    u0 = np.linalg.solve(Ut, g)
    I = np.eye(M.shape[0])
    x_star = -np.linalg.solve(I - M, u0)
    mu = np.linalg.eigvals(M).real.max()
    X, _ = O.solve_landmarks(P, prob)
    lin = O.linearize(P, X, prob)
    unorm = lambda v: np.sqrt(v @ Ut @ v)
    q_prev = np.inf
    for m in (0, 1, 2, 5, 10, 30):
        closed = -(I - np.linalg.matrix_power(M, m + 1)) @ np.linalg.solve(I - M, u0)
        dP = O.camera_step(P, lin, lam, order=m).ravel()
        np.testing.assert_allclose(dP, D["Bd"] @ closed, rtol=1e-8, atol=1e-12 * np.abs(closed).max())
        assert unorm(closed - x_star) <= mu ** (m + 1) * unorm(x_star) * (1 + 1e-9)
        # the quadratic model g^T x + x^T S x / 2 never increases with the order
        S = Ut - W @ Vp @ W.T
        q = g @ closed + 0.5 * closed @ S @ closed
        assert q <= q_prev + 1e-12 * abs(q)
        q_prev = q


def test_series_early_stop_is_the_first_small_term():
    """The optional early stop of the series (reading of the undefined
    "threshold" of Sec. 5.2): the sum ends after the first term t >= 1 with
    ||x_t|| <= rtol ||x_0 + ... + x_t||.  The stopping order is found here from
    dense powers of M, and the oracle's step equals the Neumann closed form at
    that order."""
    prob = tiny(n_cams=4, n_pts=30, seed=31)
    P = synth.init_cameras(prob.n_cams, 32)
    X, _ = O.solve_landmarks(P, prob)
    lin = O.linearize(P, X, prob)
    stops = []
    for lam, rtol in ((0.3, 0.05), (0.3, 0.01), (3.0, 0.01), (1e-3, 0.01)):
        D = _dense_problem(prob, P, lam)
        Ut, W, V = D["Ut"], D["W"], D["V"]
        Vp = np.linalg.pinv(V, rcond=1e-12, hermitian=True)
        M = np.linalg.solve(Ut, W @ Vp @ W.T)
        u0 = np.linalg.solve(Ut, D["bp"] - W @ Vp @ D["bl"])
        x, acc, t_stop = -u0, -u0, 20
        for t in range(1, 21):
            x = M @ x
            acc = acc + x
            if np.linalg.norm(x) <= rtol * np.linalg.norm(acc):
                t_stop = t
                break
        _, used = O.power_series(O.reduced_system(P, lin, lam), 20, rtol)
        assert used == t_stop
        I = np.eye(M.shape[0])
        closed = -(I - np.linalg.matrix_power(M, t_stop + 1)) @ np.linalg.solve(I - M, u0)
        dP = O.camera_step(P, lin, lam, 20, rtol=rtol).ravel()
        np.testing.assert_allclose(dP, D["Bd"] @ closed, rtol=1e-8, atol=1e-12 * np.abs(closed).max())
        stops.append(t_stop)
    assert min(stops) < 20       # the stop is exercised


@pytest.mark.parametrize("manifold,lam", [("sphere", 1e-4), ("sphere", 1.0), ("euclidean", 1e-2)])
def test_lemma1_spectrum_in_unit_interval(manifold, lam):
    prob = tiny(n_cams=5, n_pts=40, seed=41)
    P = synth.init_cameras(prob.n_cams, 42)
    D = _dense_problem(prob, P, lam, manifold)
    Vp = np.linalg.pinv(D["V"], rcond=1e-12, hermitian=True)
    M = np.linalg.solve(D["Ut"], D["W"] @ Vp @ D["W"].T)
    ev = np.linalg.eigvals(M)
    assert np.abs(ev.imag).max() < 1e-8
    assert ev.real.min() > -1e-10 and ev.real.max() < 1.0


@pytest.mark.parametrize("manifold,lam", [("sphere", 1.0), ("sphere", 0.1), ("euclidean", 1.0)])
def test_mu_max_by_power_iteration_matches_dense_spectrum(manifold, lam):
    """The oracle's mu_max (power iteration in the U~ inner product) equals the
    largest eigenvalue of the densely assembled M (in another tangent basis),
    and the terms of the series (17) shrink at that rate.  With little damping
    (eigenvalues clustered below 1) the iteration gives a lower bound."""
    prob = tiny(n_cams=5, n_pts=40, seed=41)
    P = synth.init_cameras(prob.n_cams, 42)
    D = _dense_problem(prob, P, lam, manifold)
    Vp = np.linalg.pinv(D["V"], rcond=1e-12, hermitian=True)
    M = np.linalg.solve(D["Ut"], D["W"] @ Vp @ D["W"].T)
    ev = np.sort(np.linalg.eigvals(M).real)
    X, _ = O.solve_landmarks(P, prob)
    rs = O.reduced_system(P, O.linearize(P, X, prob), lam, manifold)
    mu = O.spectral_radius(rs)
    assert abs(mu - ev[-1]) <= 1e-8 * ev[-1], (mu, ev[-1])
    # |x_{t+1}|_U / |x_t|_U of the series terms from x_0 = -U~^-1 g tends to
    # mu_max at the rate (second eigenvalue / mu_max)^t
    n, k = rs.Ut.shape[0], rs.Ut.shape[1]
    unorm = lambda v: np.sqrt(v @ np.einsum("nkl,nl->nk", rs.Ut, v.reshape(n, k)).reshape(-1))
    x = -rs.apply_Uinv(rs.g)
    t_end = 400
    for _ in range(t_end):
        x_prev, x = x, rs.apply_M(x)
    ratio = unorm(x) / unorm(x_prev)
    assert abs(ratio - mu) <= 2 * mu * (ev[-2] / ev[-1]) ** t_end + 1e-9 * mu, (ratio, mu, ev[-2])
    # clustered spectrum (lambda = 1e-4): a lower bound within the iteration's reach
    rs4 = O.reduced_system(P, O.linearize(P, X, prob), 1e-4, manifold)
    D4 = _dense_problem(prob, P, 1e-4, manifold)
    Vp4 = np.linalg.pinv(D4["V"], rcond=1e-12, hermitian=True)
    top4 = np.linalg.eigvals(np.linalg.solve(D4["Ut"], D4["W"] @ Vp4 @ D4["W"].T)).real.max()
    mu4 = O.spectral_radius(rs4, iters=2000)
    assert top4 - 1e-3 <= mu4 <= top4 + 1e-12


def test_lm_diagnostics_mu_bl_and_gradient():
    """lm_solve's diagnostics: mu_max of every step's system is in [0, 1)
    (Lemma 1 with damping), |b_l| at each trial point's closed-form landmarks
    is zero to rounding (they minimise over X), and the final gradient norm is
    that of riemannian_gradient at the returned cameras."""
    prob = tiny(n_cams=5, n_pts=40, seed=43)
    res = O.lm_solve(prob, opts=O.Options(order=10, max_iters=6, ftol=0.0, diag=True))
    assert len(res.trace_mu) == len(res.trace_bl) == res.iters == 6
    assert all(0.0 <= m < 1.0 for m in res.trace_mu)
    for P_scale_bl in res.trace_bl:
        assert P_scale_bl < 1e-8
    g = O.riemannian_gradient(res.P, O.linearize(res.P, res.X, prob))
    assert res.grad_norm == float(np.linalg.norm(g)) and res.grad_norm > 0.0


# --------------------------------------------------------------------------- tangent space
def test_update_is_tangent_and_retraction_normalises():
    prob = tiny(seed=51)
    P = synth.init_cameras(prob.n_cams, 52)
    X, _ = O.solve_landmarks(P, prob)
    lin = O.linearize(P, X, prob)
    dP = O.camera_step(P, lin, 1e-3, order=10)
    assert np.abs(np.sum(P * dP, axis=1)).max() < 1e-12 * np.abs(dP).max()
    Pn = O.retract(P, dP)
    np.testing.assert_allclose(np.linalg.norm(Pn, axis=1), 1.0, atol=1e-14)
    # |p + dp|^2 = 1 + |dp|^2 because dp is orthogonal to the unit vector p
    np.testing.assert_allclose(np.linalg.norm(P + dP, axis=1) ** 2,
                               1 + np.linalg.norm(dP, axis=1) ** 2, rtol=1e-12)


def test_update_does_not_depend_on_the_tangent_basis(monkeypatch):
    prob = tiny(seed=61)
    P = synth.init_cameras(prob.n_cams, 62)
    X, _ = O.solve_landmarks(P, prob)
    lin = O.linearize(P, X, prob)
    ref = O.camera_step(P, lin, 1e-2, order=7)
    rng = np.random.default_rng(63)
    Q = np.linalg.qr(rng.standard_normal((prob.n_cams, 11, 11)))[0]
    orig = O.tangent_basis
    monkeypatch.setattr(O, "tangent_basis", lambda P_: orig(P_) @ Q)
    alt = O.camera_step(P, lin, 1e-2, order=7)
    np.testing.assert_allclose(alt, ref, rtol=1e-10, atol=1e-13)


# --------------------------------------------------------------------------- gauge invariance
def test_reduced_cost_is_invariant_under_affine_gauge():
    """P_i -> P_i H with H = [[A, t], [0, 1]] keeps the last landmark coordinate
    at 1 (x~ -> H^-1 x~), so f* cannot change (Euclidean form)."""
    prob = tiny(seed=71)
    P = synth.init_cameras(prob.n_cams, 72)
    rng = np.random.default_rng(73)
    H = np.eye(4); H[:3, :3] = rng.standard_normal((3, 3)) + 2 * np.eye(3); H[:3, 3] = rng.standard_normal(3)
    PH = (P.reshape(-1, 3, 4) @ H).reshape(-1, 12)
    f0, f1 = O.reduced_cost(P, prob), O.reduced_cost(PH, prob)
    assert abs(f1 - f0) <= 1e-10 * f0
    # an orthogonal A keeps every camera on the unit sphere as well
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    G = np.eye(4); G[:3, :3] = R
    PR = (P.reshape(-1, 3, 4) @ G).reshape(-1, 12)
    np.testing.assert_allclose(np.linalg.norm(PR, axis=1), 1.0, atol=1e-14)
    assert abs(O.reduced_cost(PR, prob) - f0) <= 1e-12 * f0


# --------------------------------------------------------------------------- LM loop
def test_lm_loop_accepts_only_decreases_and_updates_lambda():
    prob = synth.workload(1)
    res = O.lm_solve(prob, opts=O.Options(order=10, max_iters=25, ftol=0.0))
    f = res.cost0
    lam = 1e-4
    for fc, acc, lu in zip(res.trace_cost, res.trace_accept, res.trace_lambda):
        assert lu == pytest.approx(lam, rel=1e-12)
        assert acc == (fc < f)
        if acc:
            f = fc
            lam = max(lam / 10, 1e-12)
        else:
            lam = min(lam * 10, 1e12)
    assert res.cost == f
    assert res.cost < 0.05 * res.cost0


def test_lm_reaches_known_zero_minimum_on_noise_free_affine_problem():
    """From random cameras the Euclidean (paper-literal) update reaches the known
    zero minimum of exact affine data — a check of the whole loop.  On the unit
    sphere pOSE is not scale invariant (its affine term is not), so the zero-cost
    cameras are not on the constraint set; there the check is a large decrease."""
    prob = synth.make_problem(8, 200, track=("uniform", 4, 6), seed=81, sigma=0.0, affine=True)
    res = O.lm_solve(prob, opts=O.Options(order=20, max_iters=50, ftol=0.0, manifold="euclidean"))
    assert res.cost < 1e-12 * res.cost0
    res = O.lm_solve(prob, opts=O.Options(order=20, max_iters=50, ftol=0.0, manifold="sphere"))
    assert res.cost < 1e-3 * res.cost0


# --------------------------------------------------------------------------- series from a given start
def test_series_from_a_given_start_matches_dense_closed_form():
    """The series of (17) from an arbitrary ambient start x0 (the operator
    povar_debug_series exposes).  With the dense tangent-space matrix
    M = U~^-1 W~ V^+ W~^T and M0 = U~^-1 B^T W V^+ W^T (the first application,
    from ambient coordinates), the order-m sum is
    x0 + Bd (I - M^m)(I - M)^-1 M0 x0; a tangent start x0 = Bd u gives
    Bd (I - M^{m+1})(I - M)^-1 u, and the start -Bd U~^-1 g gives the camera
    step itself."""
    prob = tiny(n_cams=4, n_pts=30, seed=41)
    P = synth.init_cameras(prob.n_cams, 42)
    lam = 0.3
    D = _dense_problem(prob, P, lam)
    Ut, W, V, Bd = D["Ut"], D["W"], D["V"], D["Bd"]
    Vp = np.linalg.pinv(V, rcond=1e-12, hermitian=True)
    M = np.linalg.solve(Ut, W @ Vp @ W.T)
    X, _ = O.solve_landmarks(P, prob)
    lin = O.linearize(P, X, prob)
    # ambient W from the dense literal Jacobians, not from the oracle's assembly
    Jp, Jl = O.pose_jacobians(P, X, prob.cam_idx, prob.pt_idx, prob.meas, prob.eta)
    JPa = np.zeros((4 * prob.n_obs, 12 * prob.n_cams))
    for o in range(prob.n_obs):
        i = prob.cam_idx[o]
        JPa[4 * o:4 * o + 4, 12 * i:12 * i + 12] = Jp[o]
    Wamb = JPa.T @ D["JL"]
    Mt = np.linalg.solve(Ut, Bd.T @ Wamb @ Vp @ Wamb.T)     # ambient start -> tangent coordinates
    I = np.eye(M.shape[0])
    rng = np.random.default_rng(43)
    x0 = rng.standard_normal((prob.n_cams, 12))              # not tangent
    u = rng.standard_normal(M.shape[0])
    for m in (0, 1, 3, 12):
        got = O.series_from(P, lin, lam, x0, m)
        if m == 0:
            closed = x0.ravel()
        else:
            closed = x0.ravel() + Bd @ ((I - np.linalg.matrix_power(M, m)) @ np.linalg.solve(I - M, Mt @ x0.ravel()))
        np.testing.assert_allclose(got.ravel(), closed, rtol=1e-9, atol=1e-11 * np.abs(closed).max())
        # the terms after the first are tangent
        assert np.abs(np.sum((got - x0) * P, axis=1)).max() <= 1e-12 * np.abs(got - x0).max() + 1e-300
        got_t = O.series_from(P, lin, lam, (Bd @ u).reshape(-1, 12), m)
        closed_t = Bd @ ((I - np.linalg.matrix_power(M, m + 1)) @ np.linalg.solve(I - M, u))
        np.testing.assert_allclose(got_t.ravel(), closed_t, rtol=1e-9, atol=1e-11 * np.abs(closed_t).max())
    # the camera step is the series from -U~^-1 g
    g = D["bp"] - W @ Vp @ D["bl"]
    start = (Bd @ -np.linalg.solve(Ut, g)).reshape(-1, 12)
    np.testing.assert_allclose(O.series_from(P, lin, lam, start, 7), O.camera_step(P, lin, lam, 7),
                               rtol=1e-9, atol=1e-12)


def test_riemannian_gradient_matches_tangent_finite_differences():
    """grad f* (the report's gradient norm): orthogonal to each camera and,
    along tangent directions v, equal to the central difference of the
    reduced cost (landmarks re-solved), which the envelope theorem predicts."""
    prob = tiny(n_cams=4, n_pts=40, seed=51)
    P = synth.init_cameras(prob.n_cams, 52)
    X, _ = O.solve_landmarks(P, prob)
    lin = O.linearize(P, X, prob)
    g = O.riemannian_gradient(P, lin)
    assert np.abs(np.sum(g * P, axis=1)).max() <= 1e-12 * np.abs(g).max()
    rng = np.random.default_rng(53)
    for _ in range(3):
        v = rng.standard_normal(P.shape)
        v -= np.sum(v * P, axis=1, keepdims=True) * P
        h = 1e-6
        fd = (O.reduced_cost(P + h * v, prob) - O.reduced_cost(P - h * v, prob)) / (2 * h)
        assert abs(fd - np.sum(g * v)) <= 1e-6 * max(1.0, abs(fd))
    ge = O.riemannian_gradient(P, lin, "euclidean")
    np.testing.assert_allclose(ge, 2 * lin.bp, rtol=0, atol=0)


# --------------------------------------------------------------------------- R12: no Cholesky factor
def _camera_without_measurement_signal(seed=61):
    """A problem whose camera 0 sees every point at m = (0, 0): the columns of
    J_p for the third camera row are -sqrt(1-eta) m x~ = 0, so U_0 has four
    exactly zero rows and columns (the row P^3 of that camera does not enter
    its residuals)."""
    prob = tiny(n_cams=5, n_pts=60, seed=seed)
    meas = prob.meas.copy()
    meas[prob.cam_idx == 0] = 0.0
    return synth.Problem(prob.n_cams, prob.n_pts, prob.cam_idx, prob.pt_idx, meas, prob.cams0, prob.eta,
                         prob.order)


def test_r12_a_damped_block_without_cholesky_factor_is_rejected():
    """R12.  Mathematically, U + lambda D (D = the floored diagonal of U,
    positive) is positive definite for every lambda > 0, so a Cholesky factor
    exists.  It fails only where lambda D underflows: with the damping floor
    1e-12 of the largest diagonal entry and lambda = 1e-320, the zero diagonal
    entries of U_0 stay exactly zero in FP64, the damped block is exactly
    singular (four zero rows), and no Cholesky factor exists.  The oracle then
    rejects the step: the trial cost is +inf, the cameras stay, and lambda
    goes to min(10 lambda, lambda_max)."""
    prob = _camera_without_measurement_signal()
    P, X, f = O.initial_state(prob, prob.cams0, "euclidean")
    lin = O.linearize(P, X, prob)
    assert np.all(lin.U[0][8:, :] == 0.0) and np.all(lin.U[0][:, 8:] == 0.0)
    tiny_lam = 1e-320
    rs = O.reduced_system(P, lin, tiny_lam, "euclidean")
    assert np.all(rs.Ut[0][8:, 8:] == 0.0)          # lambda * floor underflowed to zero
    assert np.linalg.matrix_rank(rs.Ut[0]) == 8      # singular: no Cholesky factor exists
    assert not O.factorizable(rs)
    assert O.factorizable(O.reduced_system(P, lin, 1e-4, "euclidean"))
    # the branch is not only reachable through underflow: on the sphere at the
    # default smallest damping (1e-12) this camera's tangent block has
    # eigenvalues of the order of 1e-24 of its largest, far below FP64
    # rounding of the block's entries, so whether a factor is found is decided
    # by rounding (the oracle and the GPU may then both reject, by R12 or by
    # a non-finite or larger trial cost)
    Ps, Xs, _ = O.initial_state(prob, prob.cams0)
    ev = np.linalg.eigvalsh(O.reduced_system(Ps, O.linearize(Ps, Xs, prob), 1e-12).Ut[0])
    assert abs(ev[0]) <= 1e-15 * ev[-1]
    # the LM loop: every step rejected, nothing moves
    res = O.lm_solve(prob, opts=O.Options(order=3, max_iters=4, ftol=0.0, lambda0=tiny_lam, lambda_min=tiny_lam,
                                          lambda_max=tiny_lam, manifold="euclidean"))
    assert res.trace_accept == [False] * 4
    assert all(np.isinf(c) for c in res.trace_cost)
    assert res.trace_lambda == [tiny_lam] * 4
    np.testing.assert_array_equal(res.P, P)
    assert res.cost == f
    # with room to grow, lambda rises x10 per rejected step
    res = O.lm_solve(prob, opts=O.Options(order=3, max_iters=3, ftol=0.0, lambda0=tiny_lam, lambda_min=tiny_lam,
                                          lambda_max=1.0, manifold="euclidean"))
    assert res.trace_lambda[1] == min(10 * tiny_lam, 1.0) and not res.trace_accept[0]


# --------------------------------------------------------------------------- seeded initial cameras
def test_philox_matches_numpy_bit_generator():
    """synth's Philox4x64-10 (written from its published definition) against
    numpy's Philox bit generator: numpy's n-th block is counter n + 1."""
    for key in (0, 7, 2 ** 63 + 12345):
        bg = np.random.Philox(key=np.array([key, 0], dtype=np.uint64), counter=np.zeros(4, dtype=np.uint64))
        raw = bg.random_raw(12)
        mine = [w for c in (1, 2, 3) for w in synth.philox4x64([c, 0, 0, 0], [key, 0])]
        assert [int(x) for x in raw] == mine


def test_seeded_cameras_are_unit_gaussian_directions():
    C = synth.seeded_cameras(3000, 11)
    np.testing.assert_allclose(np.linalg.norm(C, axis=1), 1.0, rtol=1e-15)
    # the normals behind them: mean 0, variance 1 (36,000 draws: 5 sigma bounds)
    w = C * np.sqrt(12.0)
    assert abs(w.mean()) < 5 / np.sqrt(w.size)
    assert abs((w * w).mean() - 1.0) < 0.05
    assert not np.array_equal(C, synth.seeded_cameras(3000, 12))


def test_large_problem_step_equals_the_assembled_one():
    """The memory-bounded step (per-observation W_k, observations in ranges)
    is the same computation as the assembled one: equal to rounding, with
    ranges that cut landmarks and cameras apart."""
    prob = tiny(n_cams=9, n_pts=200, seed=81, track=("uniform", 3, 6))
    P = synth.init_cameras(prob.n_cams, 82)
    for manifold in ("sphere", "euclidean"):
        Pm = P if manifold == "sphere" else P * 1.7
        Xm, _ = O.solve_landmarks(Pm, prob)
        ref = O.camera_step(Pm, O.linearize(Pm, Xm, prob), 1e-2, 7, manifold)
        got, Xg, f = O.camera_step_large(Pm, prob, 1e-2, 7, manifold, chunk=97)
        np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
        np.testing.assert_allclose(Xg, Xm, rtol=0, atol=0)
        assert f == O.cost(Pm, Xm, prob)
