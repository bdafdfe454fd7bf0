"""Plain FP64 CPU oracle for one PoVar outer iteration and the LM loop around it.

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library and does not import the package's binding; the only thing
both sides share is the seeded input generator (``paper_2405_05079_amd.synth``),
which holds none of the method's arithmetic.

Everything here is FP64, written for a reader checking it against the paper:

* residual and Jacobians are the literal pOSE residual (6) and its derivative,
  one 4x12 camera block and one 4x3 landmark block per observation;
* the normal-equation blocks (10)-(13) are formed as J^T J products of those
  literal blocks and summed with sparse incidence matrices;
* landmarks are eliminated in closed form (8) with the Moore-Penrose inverse
  of each 3x3 V_j (eigendecomposition, relative cutoff 1e-12);
* the camera step is the truncated power series (17) of the inverse Schur
  complement (14)-(15), taken in the tangent space of the unit sphere in R^12
  with an explicit orthonormal 12x11 basis per camera (Sec. 4.3, (18)-(29));
* the update is back-projected and retracted by normalisation (end of Sec. 4.3);
* the LM loop follows the settings of Sec. 5.2 (lambda0 = 1e-4, ftol).

Readings of points the paper leaves open (each is also listed with the design
notes of the repository):
  R1  camera update on the unit sphere of R^12 (tangent projection + retraction),
      landmarks Euclidean with the last coordinate fixed to 1; the paper-literal
      Euclidean update is kept as ``manifold="euclidean"``;
  R3  sign: dx_p = -S^-1 (b_p - W V^+ b_l), as in (10) and (17);
  R5  "order m" = the terms i = 0..m of (17), i.e. m applications of M;
  R6  optional stop of the series when ||x_t|| <= rtol * ||acc|| (rtol = 0: off);
  R7  damping D_p^T D_p = diag(U_i) per camera (Marquardt), each entry floored
      at 1e-12 * the largest diagonal entry of that camera; damping applied in
      ambient coordinates, then projected: U~ = B^T (U + lambda D) B;
  R8  LM: accept iff f_new < f (NaN rejects); lambda /= 10 (>= lambda_min) on
      accept, *= 10 (<= lambda_max) on reject; relinearise only after accept;
      stop when the relative decrease of an accepted step is below ftol;
  R11 V_j^+ with eigenvalues below 1e-12 * lambda_max(V_j) dropped;
  R12 a step whose damped camera block has no Cholesky factor is rejected
      (lambda x10), as any failed LM step.

parity pinned: see tests/test_oracle_pins.py (finite differences, lstsq,
envelope theorem, dense joint solve, Neumann closed form and bound, Lemma 1,
tangency and basis invariance, gauge invariance, known zero minimum, the R12
branch on a block without a Cholesky factor, the series from a given start
against its dense closed form, the Riemannian gradient against central
differences, the memory-bounded step against the assembled one, mu_max by
power iteration against the dense spectrum and the decay of the series
terms).  lm_solve:
each step and the accept rule R8 are pinned; the trajectory over many
iterations has no closed form of its own: parity unpinned beyond those pins.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

PINV_RTOL = 1e-12
DAMP_FLOOR = 1e-12


# ----------------------------------------------------------------------------
# pOSE residual (6) and its Jacobian blocks
# ----------------------------------------------------------------------------
def homogeneous(X: np.ndarray) -> np.ndarray:
    """x~ = (X, 1): the last landmark coordinate is fixed to 1 (Sec. 3.2, (5))."""
    return np.concatenate([X, np.ones((X.shape[0], 1))], axis=1)


def pose_residual(P: np.ndarray, X: np.ndarray, cam, pt, meas, eta: float) -> np.ndarray:
    """Residual of (6) for every observation, shape (n_obs, 4).

    P: (n_cams, 12) row-major 3x4 cameras; X: (n_pts, 3).
    Rows: sqrt(1-eta) * (P^{1:2} x~ - (P^3 x~) m)  and  sqrt(eta) * (P^{1:2} x~ - m).
    """
    C = P[cam].reshape(-1, 3, 4)
    xh = homogeneous(X[pt])
    proj = np.einsum("nab,nb->na", C, xh)          # (P^1 x~, P^2 x~, P^3 x~)
    top = proj[:, :2] - proj[:, 2:3] * meas        # OSE part
    aff = proj[:, :2] - meas                       # affine part
    return np.concatenate([np.sqrt(1.0 - eta) * top, np.sqrt(eta) * aff], axis=1)


def pose_jacobians(P: np.ndarray, X: np.ndarray, cam, pt, meas, eta: float):
    """Derivatives of (6): J_p (n_obs, 4, 12) w.r.t. the row-major camera vector
    and J_l (n_obs, 4, 3) w.r.t. the three free landmark coordinates."""
    n = cam.shape[0]
    sa, se = np.sqrt(1.0 - eta), np.sqrt(eta)
    C = P[cam].reshape(n, 3, 4)
    xh = homogeneous(X[pt])
    m1, m2 = meas[:, 0:1], meas[:, 1:2]
    Jp = np.zeros((n, 4, 12))
    # d/dP of P^1 x~ is x~ in columns 0..3, of P^2 x~ in 4..7, of P^3 x~ in 8..11
    Jp[:, 0, 0:4] = sa * xh
    Jp[:, 0, 8:12] = -sa * m1 * xh
    Jp[:, 1, 4:8] = sa * xh
    Jp[:, 1, 8:12] = -sa * m2 * xh
    Jp[:, 2, 0:4] = se * xh
    Jp[:, 3, 4:8] = se * xh
    Pbar = C[:, :, :3]
    Jl = np.zeros((n, 4, 3))
    Jl[:, 0] = sa * (Pbar[:, 0] - m1 * Pbar[:, 2])
    Jl[:, 1] = sa * (Pbar[:, 1] - m2 * Pbar[:, 2])
    Jl[:, 2] = se * Pbar[:, 0]
    Jl[:, 3] = se * Pbar[:, 1]
    return Jp, Jl


# ----------------------------------------------------------------------------
# small helpers: per-index sums and the Moore-Penrose inverse of 3x3 blocks
# ----------------------------------------------------------------------------
def sum_by(idx: np.ndarray, n: int, vals: np.ndarray) -> np.ndarray:
    """out[k] = sum of vals[o] over observations o with idx[o] == k."""
    m = vals.shape[0]
    inc = sp.csr_matrix((np.ones(m), (idx, np.arange(m))), shape=(n, m))
    flat = vals.reshape(m, -1)
    return np.asarray(inc @ flat).reshape((n,) + vals.shape[1:])


def pinv_sym(V: np.ndarray, rtol: float = PINV_RTOL) -> np.ndarray:
    """Moore-Penrose inverse of a stack of symmetric PSD matrices by
    eigendecomposition; eigenvalues <= rtol * largest are treated as zero."""
    w, Q = np.linalg.eigh(V)
    cut = rtol * w[..., -1:]
    inv = np.where(w > cut, 1.0 / np.where(w > cut, w, 1.0), 0.0)
    return np.einsum("...ik,...k,...jk->...ij", Q, inv, Q)


# ----------------------------------------------------------------------------
# closed-form landmark elimination (8) and the reduced cost (9)
# ----------------------------------------------------------------------------
def solve_landmarks(P: np.ndarray, prob) -> tuple[np.ndarray, np.ndarray]:
    """x~_l*(x_p) = G^+ z for every landmark (8).  Per landmark the residual is
    affine in X: r = J_l X + r(X=0), so the least-squares X is
    V^+ (-sum J_l^T r(X=0)) with V = sum J_l^T J_l.  Returns (X*, V^+)."""
    zeros = np.zeros((prob.n_pts, 3))
    r0 = pose_residual(P, zeros, prob.cam_idx, prob.pt_idx, prob.meas, prob.eta)
    _, Jl = pose_jacobians(P, zeros, prob.cam_idx, prob.pt_idx, prob.meas, prob.eta)
    V = sum_by(prob.pt_idx, prob.n_pts, np.einsum("nri,nrj->nij", Jl, Jl))
    h = -sum_by(prob.pt_idx, prob.n_pts, np.einsum("nri,nr->ni", Jl, r0))
    Vp = pinv_sym(V)
    X = np.einsum("nij,nj->ni", Vp, h)
    return X, Vp


def cost(P: np.ndarray, X: np.ndarray, prob) -> float:
    """F = sum ||r||^2 over all observations (5)-(6)."""
    r = pose_residual(P, X, prob.cam_idx, prob.pt_idx, prob.meas, prob.eta)
    return float(np.sum(r * r))


def reduced_cost(P: np.ndarray, prob) -> float:
    """f*(x_p) = F(x_p, x_l*(x_p)) (9)."""
    X, _ = solve_landmarks(P, prob)
    return cost(P, X, prob)


# ----------------------------------------------------------------------------
# linearisation: normal-equation blocks (10)-(13)
# ----------------------------------------------------------------------------
@dataclass
class Linearization:
    U: np.ndarray        # (n_cams, 12, 12)   J_p^T J_p per camera
    V: np.ndarray        # (n_pts, 3, 3)      J_l^T J_l per landmark
    Vp: np.ndarray       # (n_pts, 3, 3)      V^+
    W: sp.csr_matrix     # (12 n_cams, 3 n_pts)  J_p^T J_l
    bp: np.ndarray       # (n_cams, 12)       J_p^T r
    bl: np.ndarray       # (n_pts, 3)         J_l^T r
    cost: float


def linearize(P: np.ndarray, X: np.ndarray, prob) -> Linearization:
    cam, pt = prob.cam_idx, prob.pt_idx
    r = pose_residual(P, X, cam, pt, prob.meas, prob.eta)
    Jp, Jl = pose_jacobians(P, X, cam, pt, prob.meas, prob.eta)
    U = sum_by(cam, prob.n_cams, np.einsum("nri,nrj->nij", Jp, Jp))
    V = sum_by(pt, prob.n_pts, np.einsum("nri,nrj->nij", Jl, Jl))
    bp = sum_by(cam, prob.n_cams, np.einsum("nri,nr->ni", Jp, r))
    bl = sum_by(pt, prob.n_pts, np.einsum("nri,nr->ni", Jl, r))
    Wk = np.einsum("nri,nrj->nij", Jp, Jl)                       # (n, 12, 3)
    rows = (12 * cam.astype(np.int64))[:, None, None] + np.arange(12)[None, :, None]
    cols = (3 * pt.astype(np.int64))[:, None, None] + np.arange(3)[None, None, :]
    rows, cols = np.broadcast_arrays(rows, cols)
    W = sp.csr_matrix((Wk.ravel(), (rows.ravel(), cols.ravel())),
                      shape=(12 * prob.n_cams, 3 * prob.n_pts))
    return Linearization(U=U, V=V, Vp=pinv_sym(V), W=W, bp=bp, bl=bl, cost=float(np.sum(r * r)))


def damped(U: np.ndarray, lam: float) -> np.ndarray:
    """U_lambda = U + lambda D^T D with D^T D = diag(U) (floored), per camera (R7)."""
    d = np.diagonal(U, axis1=1, axis2=2).copy()
    d = np.maximum(d, DAMP_FLOOR * d.max(axis=1, keepdims=True))
    Ul = U.copy()
    idx = np.arange(12)
    Ul[:, idx, idx] += lam * d
    return Ul


def tangent_basis(P: np.ndarray) -> np.ndarray:
    """Orthonormal basis of the tangent space {d : p_i^T d = 0} of the unit
    sphere at each camera, (n_cams, 12, 11), from a Householder QR of p_i."""
    Q, _ = np.linalg.qr(P[:, :, None], mode="complete")
    return Q[:, :, 1:]


def block_diag_sparse(blocks: np.ndarray) -> sp.csr_matrix:
    n, r, c = blocks.shape
    rows = (np.arange(n)[:, None, None] * r + np.arange(r)[None, :, None])
    cols = (np.arange(n)[:, None, None] * c + np.arange(c)[None, None, :])
    rows, cols = np.broadcast_arrays(rows, cols)
    return sp.csr_matrix((blocks.ravel(), (rows.ravel(), cols.ravel())), shape=(n * r, n * c))


# ----------------------------------------------------------------------------
# the PoVar camera step: truncated power series of the inverse Schur complement
# ----------------------------------------------------------------------------
@dataclass
class ReducedSystem:
    """Tangent-space reduced camera system of one linearisation and lambda."""
    B: np.ndarray             # (n_cams, 12, k) basis; k = 11 (sphere) or 12 (euclidean)
    Ut: np.ndarray            # (n_cams, k, k)  U~_lambda
    Wt: sp.csr_matrix         # (k n_cams, 3 n_pts)
    Vp_blk: sp.csr_matrix     # (3 n_pts, 3 n_pts) block-diagonal V^+
    g: np.ndarray             # (k n_cams,)  b~_p - W~ V^+ b_l

    def apply_Uinv(self, v: np.ndarray) -> np.ndarray:
        n, k = self.Ut.shape[0], self.Ut.shape[1]
        return np.linalg.solve(self.Ut, v.reshape(n, k, 1)).reshape(-1)

    def apply_M(self, x: np.ndarray) -> np.ndarray:
        """M x = U~^-1 W~ V^+ W~^T x (the matrix of Lemma 1 / (17))."""
        return self.apply_Uinv(self.Wt @ (self.Vp_blk @ (self.Wt.T @ x)))


def reduced_system(P: np.ndarray, lin: Linearization, lam: float,
                   manifold: str = "sphere") -> ReducedSystem:
    n = P.shape[0]
    if manifold == "sphere":
        B = tangent_basis(P)
    elif manifold == "euclidean":
        B = np.broadcast_to(np.eye(12), (n, 12, 12)).copy()
    else:
        raise ValueError(manifold)
    Ul = damped(lin.U, lam)
    Ut = np.einsum("nik,nij,njl->nkl", B, Ul, B)
    Bs = block_diag_sparse(B)
    Wt = (Bs.T @ lin.W).tocsr()
    Vp_blk = block_diag_sparse(lin.Vp)
    bt = Bs.T @ lin.bp.reshape(-1)
    g = bt - Wt @ (Vp_blk @ lin.bl.reshape(-1))
    return ReducedSystem(B=B, Ut=Ut, Wt=Wt, Vp_blk=Vp_blk, g=g)


def power_series(rs: ReducedSystem, order: int, rtol: float = 0.0):
    """x(m) = -sum_{i=0..m} M^i U~^-1 g  (17) / (29), in tangent coordinates.
    Returns (x(m), number of terms applied after the first)."""
    x = -rs.apply_Uinv(rs.g)
    acc = x.copy()
    used = 0
    for _ in range(order):
        x = rs.apply_M(x)
        acc = acc + x
        used += 1
        if rtol > 0 and np.linalg.norm(x) <= rtol * np.linalg.norm(acc):
            break
    return acc, used


def spectral_radius(rs: ReducedSystem, iters: int = 20000, tol: float = 1e-10, seed: int = 0) -> float:
    """mu_max, the largest eigenvalue of M = U~^-1 W~ V^+ W~^T, by power
    iteration: the series (17) converges when it is below 1 (Lemma 1 /
    Prop. 1), and its terms shrink like mu_max^t.  M is self-adjoint in the
    inner product <x, y> = x^T U~ y (U~ M = W~ V^+ W~^T is symmetric), so its
    eigenvalues are real and non-negative and the Rayleigh quotient
    mu = x^T W~ V^+ W~^T x / x^T U~ x of the iterate converges to the largest.
    Stops when the residual |M x - mu x|_U is below tol |x|_U (then mu is
    within tol^2 / gap of mu_max) or after `iters` steps: the quotient never
    exceeds mu_max, and with eigenvalues clustered near it (little damping)
    it approaches it at the rate of their ratio.  A diagnostic for small
    problems."""
    n, k = rs.Ut.shape[0], rs.Ut.shape[1]
    x = np.random.default_rng(seed).standard_normal(n * k)
    mu = 0.0
    for _ in range(iters):
        wvw = rs.Wt @ (rs.Vp_blk @ (rs.Wt.T @ x))            # W~ V^+ W~^T x = U~ M x
        ux = np.einsum("nkl,nl->nk", rs.Ut, x.reshape(n, k)).reshape(-1)
        xux = float(x @ ux)
        mu = float(x @ wvw) / xux
        y = rs.apply_Uinv(wvw)                             # M x
        d = y - mu * x
        res2 = float(d @ np.einsum("nkl,nl->nk", rs.Ut, d.reshape(n, k)).reshape(-1))
        if res2 <= tol * tol * xux:
            break
        x = y / np.linalg.norm(y)
    return mu


def series_from(P: np.ndarray, lin: Linearization, lam: float, x0: np.ndarray, order: int,
                manifold: str = "sphere") -> np.ndarray:
    """The truncated series of (17) started from a given ambient camera vector:
    sum_{t=0..m} x_t with x_0 = x0 (n_cams, 12) as given and
    x_t = B U~^-1 B^T W V^+ W^T x_{t-1}, i.e. the operator of Lemma 1 mapped
    to ambient coordinates by each camera's tangent basis B (identity in
    Euclidean mode).  For x0 = B x~ the partial sums are B times those of
    (17) from x~."""
    rs = reduced_system(P, lin, lam, manifold)
    Bs = block_diag_sparse(rs.B)
    x = np.asarray(x0, dtype=np.float64).reshape(-1).copy()
    acc = x.copy()
    for _ in range(order):
        z = rs.Vp_blk @ (lin.W.T @ x)          # V^+ W^T x, per landmark
        x = Bs @ rs.apply_Uinv(rs.Wt @ z)      # B U~^-1 B^T W z, per camera
        acc = acc + x
    return acc.reshape(P.shape[0], 12)


def riemannian_gradient(P: np.ndarray, lin: Linearization, manifold: str = "sphere") -> np.ndarray:
    """Gradient of the reduced cost f* (9) at P, projected onto each camera's
    tangent space: by the envelope theorem the Euclidean gradient is
    2 J_p^T r = 2 b_p when the landmarks are at X*(P)."""
    g = 2.0 * lin.bp
    if manifold == "sphere":
        g = g - np.sum(g * P, axis=1, keepdims=True) * P
    return g


def back_project(rs: ReducedSystem, xt: np.ndarray) -> np.ndarray:
    """Ambient camera update dx~_p = x~_p^perp dx_p, (n_cams, 12)."""
    n, _, k = rs.B.shape
    return np.einsum("nik,nk->ni", rs.B, xt.reshape(n, k))


def retract(P: np.ndarray, dP: np.ndarray, manifold: str = "sphere") -> np.ndarray:
    """Add the update and, on the sphere, normalise each camera vector."""
    Q = P + dP
    if manifold == "sphere":
        Q = Q / np.linalg.norm(Q, axis=1, keepdims=True)
    return Q


def factorizable(rs: ReducedSystem) -> bool:
    """True if every damped tangent camera block has a Cholesky factor."""
    try:
        np.linalg.cholesky(rs.Ut)
        return True
    except np.linalg.LinAlgError:
        return False


def camera_step(P, lin, lam, order, manifold="sphere", rtol=0.0):
    """One PoVar camera update (ambient, (n_cams, 12)) for a linearisation."""
    rs = reduced_system(P, lin, lam, manifold)
    xt, _ = power_series(rs, order, rtol)
    return back_project(rs, xt)


# ----------------------------------------------------------------------------
# Levenberg-Marquardt outer loop (Sec. 4.1-4.2 and the settings of Sec. 5.2)
# ----------------------------------------------------------------------------
@dataclass
class Options:
    order: int = 20
    max_iters: int = 50
    ftol: float = 1e-6
    lambda0: float = 1e-4
    lambda_min: float = 1e-12
    lambda_max: float = 1e12
    manifold: str = "sphere"
    rtol: float = 0.0
    diag: bool = False        # record |b_l|, mu_max per step and the final gradient norm (small problems)
    mu_iters: int = 2000      # power iterations for each step's mu_max (a lower bound when not converged)


@dataclass
class Result:
    P: np.ndarray
    X: np.ndarray
    cost: float
    cost0: float
    lam: float
    iters: int
    trace_cost: list = field(default_factory=list)      # trial cost of each iteration
    trace_accept: list = field(default_factory=list)
    trace_lambda: list = field(default_factory=list)    # lambda used by each iteration
    # with Options.diag: |b_l| at each trial point's landmarks, mu_max of each
    # step's system, |Riemannian gradient| at the final cameras
    trace_bl: list = field(default_factory=list)
    trace_mu: list = field(default_factory=list)
    grad_norm: float = float("nan")
    stop: str = "max_iters"


def initial_state(prob, cams0, manifold="sphere"):
    P = np.array(cams0, dtype=np.float64).reshape(prob.n_cams, 12)
    if manifold == "sphere":
        P = P / np.linalg.norm(P, axis=1, keepdims=True)
    X, _ = solve_landmarks(P, prob)
    return P, X, cost(P, X, prob)


def lm_solve(prob, cams0=None, opts: Options | None = None, lam=None, P=None) -> Result:
    """Run the PoVar LM loop from cams0 (or from state P, lam)."""
    opts = opts or Options()
    if P is None:
        P, X, f = initial_state(prob, prob.cams0 if cams0 is None else cams0, opts.manifold)
    else:
        X, _ = solve_landmarks(P, prob)
        f = cost(P, X, prob)
    lam = opts.lambda0 if lam is None else lam
    res = Result(P=P, X=X, cost=f, cost0=f, lam=lam, iters=0)
    lin = None
    for it in range(opts.max_iters):
        if lin is None:
            lin = linearize(P, X, prob)
        rs = reduced_system(P, lin, lam, opts.manifold)
        res.trace_lambda.append(lam)
        if not factorizable(rs):
            # R12: a step whose damped camera block has no Cholesky factor is rejected
            fn, accepted = np.inf, False
            if opts.diag:
                res.trace_bl.append(float("nan"))
                res.trace_mu.append(float("nan"))
        else:
            if opts.diag:
                res.trace_mu.append(spectral_radius(rs, iters=opts.mu_iters))
            xt, _ = power_series(rs, opts.order, opts.rtol)
            Pn = retract(P, back_project(rs, xt), opts.manifold)
            Xn, _ = solve_landmarks(Pn, prob)
            fn = cost(Pn, Xn, prob)
            if opts.diag:
                res.trace_bl.append(float(np.linalg.norm(linearize(Pn, Xn, prob).bl)))
            accepted = bool(np.isfinite(fn) and fn < f)
        res.trace_cost.append(fn)
        res.trace_accept.append(accepted)
        res.iters = it + 1
        if accepted:
            rel = (f - fn) / f
            P, X, f = Pn, Xn, fn
            lam = max(lam / 10.0, opts.lambda_min)
            lin = None
            if rel < opts.ftol:
                res.stop = "ftol"
                break
        else:
            lam = min(lam * 10.0, opts.lambda_max)
    res.P, res.X, res.cost, res.lam = P, X, f, lam
    if opts.diag:
        res.grad_norm = float(np.linalg.norm(riemannian_gradient(P, linearize(P, X, prob), opts.manifold)))
    return res


# ----------------------------------------------------------------------------
# the same camera step for problems too large for the sparse assembly above
# ----------------------------------------------------------------------------
def camera_step_large(P: np.ndarray, prob, lam: float, order: int, manifold: str = "sphere",
                      chunk: int = 1_000_000):
    """camera_step(P, linearize(P, X*(P), prob), lam, order) for problems with
    tens of millions of observations (memory-bounded; the 13,700-camera
    workload).  The same definitions as above: the literal Jacobians of (6)
    per observation, U and b_p summed per camera, V^+ per landmark, the
    reduced system in an explicit tangent basis and the series (17).  Instead
    of the assembled sparse W (which would not fit in host memory), each
    observation keeps its own W_k = J_p^T J_l (12 x 3), and W z / W^T x are
    their per-camera / per-landmark sums; the observations are processed in
    consecutive ranges of `chunk`, whose partial sums are added.  Returns the
    ambient step (n_cams, 12), X*(P) and the cost at P."""
    cam, pt, n = prob.cam_idx, prob.pt_idx, prob.n_obs
    X, Vp = solve_landmarks(P, prob)
    f = cost(P, X, prob)
    U = np.zeros((prob.n_cams, 12, 12))
    bp = np.zeros((prob.n_cams, 12))
    bl = np.zeros((prob.n_pts, 3))
    Wk = np.empty((n, 12, 3))
    ranges = [(a, min(a + chunk, n)) for a in range(0, n, chunk)]
    for a, b in ranges:
        c, p_, m = cam[a:b], pt[a:b], prob.meas[a:b]
        r = pose_residual(P, X, c, p_, m, prob.eta)
        Jp, Jl = pose_jacobians(P, X, c, p_, m, prob.eta)
        U += sum_by(c, prob.n_cams, np.einsum("nri,nrj->nij", Jp, Jp))
        bp += sum_by(c, prob.n_cams, np.einsum("nri,nr->ni", Jp, r))
        bl += sum_by(p_, prob.n_pts, np.einsum("nri,nr->ni", Jl, r))
        Wk[a:b] = np.einsum("nri,nrj->nij", Jp, Jl)

    def W_times(z):         # sum_{k in i} W_k z_j, per camera
        out = np.zeros((prob.n_cams, 12))
        for a, b in ranges:
            out += sum_by(cam[a:b], prob.n_cams, np.einsum("nij,nj->ni", Wk[a:b], z[pt[a:b]]))
        return out

    def WT_times(x):        # sum_{k in j} W_k^T x_i, per landmark
        out = np.zeros((prob.n_pts, 3))
        for a, b in ranges:
            out += sum_by(pt[a:b], prob.n_pts, np.einsum("nij,ni->nj", Wk[a:b], x[cam[a:b]]))
        return out

    B = tangent_basis(P) if manifold == "sphere" else np.broadcast_to(np.eye(12), (prob.n_cams, 12, 12))
    Ut = np.einsum("nik,nij,njl->nkl", B, damped(U, lam), B)
    Vp_times = lambda y: np.einsum("nij,nj->ni", Vp, y)
    Ut_solve = lambda v: np.linalg.solve(Ut, v[..., None])[..., 0]
    g = np.einsum("nik,ni->nk", B, bp - W_times(Vp_times(bl)))
    x = -Ut_solve(g)                                    # tangent coordinates, per camera
    acc = x.copy()
    for _ in range(order):
        s = np.einsum("nik,ni->nk", B, W_times(Vp_times(WT_times(np.einsum("nik,nk->ni", B, x)))))
        x = Ut_solve(s)
        acc = acc + x
    return np.einsum("nik,nk->ni", B, acc), X, f
