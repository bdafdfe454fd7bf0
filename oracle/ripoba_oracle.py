"""Plain FP64 CPU oracle for the second stage, projective refinement with the
Riemannian power-series solver (RiPoBA): objective (7) of Sec. 3 and the
method of Sec. 4.3.

TEST INFRASTRUCTURE.  Only the tests may import this module.  It shares no
code with the HIP library and does not import the package's binding; it uses
the first-stage oracle only for small generic helpers (per-index sums, sparse
block diagonals).

Everything here is FP64, written for a reader checking it against the paper:

* residual (7): r_ij = pi(P_i X_j) - m_ij with pi(y) = (y_1/y_3, y_2/y_3);
  P_i (row-major 3x4) on the unit sphere of R^12, X_j (homogeneous) on the
  unit sphere of R^4;
* per observation one 2x12 camera block and one 2x4 landmark block of the
  Jacobian, by the chain rule through pi;
* the normal-equation blocks U, V, W, b_p, b_l of the joint problem, projected
  with explicit orthonormal tangent bases (12x11 per camera, 4x3 per
  landmark): the Riemannian normal equations (20)-(26);
* damping in ambient coordinates, then projected: U~ = B_p^T (U + lam D_p) B_p
  and V~ = B_l^T (V + lam D_l) B_l with Marquardt D^T D = diag (reading R7 of
  the first stage, applied to both blocks);
* the Riemannian Schur complement (27) and its truncated power series (29)
  for the camera update, the landmark update by back-substitution, both
  back-projected and retracted by normalisation (end of Sec. 4.3);
* the LM loop of the first stage (reading R8; settings of Sec. 5.2).

parity pinned: see tests/test_ripoba_pins.py (worked example of (7), central
finite differences, degree-0 homogeneity of the residual, the dense joint
Riemannian system and its Neumann partial sums with and without the early
stop, Lemma 2's spectrum, the zero minimum of noise-free data, projective
gauge invariance, the hand-over from the first stage).  lm_solve: its steps
and the accept rule (R8) are pinned; the many-iteration trajectory has no
closed form of its own: parity unpinned beyond those pins.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from oracle.povar_oracle import block_diag_sparse, sum_by

DAMP_FLOOR = 1e-12


# ----------------------------------------------------------------------------
# projective residual (7) and its Jacobian blocks
# ----------------------------------------------------------------------------
def project(P: np.ndarray, Xh: np.ndarray, cam, pt) -> np.ndarray:
    """y = P_i X_j for every observation, (n_obs, 3)."""
    return np.einsum("nab,nb->na", P[cam].reshape(-1, 3, 4), Xh[pt])


def residual(P: np.ndarray, Xh: np.ndarray, cam, pt, meas) -> np.ndarray:
    """r = pi(P_i X_j) - m, (n_obs, 2)."""
    y = project(P, Xh, cam, pt)
    return y[:, :2] / y[:, 2:3] - meas


def jacobians(P: np.ndarray, Xh: np.ndarray, cam, pt):
    """d r / d vec(P_i) (n_obs, 2, 12) and d r / d X_j (n_obs, 2, 4)."""
    Pc = P[cam].reshape(-1, 3, 4)
    X = Xh[pt]
    y = np.einsum("nab,nb->na", Pc, X)
    w = y[:, 2]
    dpi = np.zeros((len(w), 2, 3))            # d pi / d y
    dpi[:, 0, 0] = 1.0 / w
    dpi[:, 1, 1] = 1.0 / w
    dpi[:, 0, 2] = -y[:, 0] / w ** 2
    dpi[:, 1, 2] = -y[:, 1] / w ** 2
    Jl = np.einsum("nra,nab->nrb", dpi, Pc)
    # y_a = sum_c P[a, c] X_c, so d y_a / d P[a', c] = delta(a, a') X_c
    Jp = np.einsum("nra,nc->nrac", dpi, X).reshape(-1, 2, 12)
    return Jp, Jl


def cost(P: np.ndarray, Xh: np.ndarray, prob) -> float:
    r = residual(P, Xh, prob.cam_idx, prob.pt_idx, prob.meas)
    return float(np.sum(r * r))


# ----------------------------------------------------------------------------
# normal equations, tangent bases, damping
# ----------------------------------------------------------------------------
@dataclass
class Linearization:
    U: np.ndarray        # (n_cams, 12, 12)  J_p^T J_p per camera
    V: np.ndarray        # (n_pts, 4, 4)     J_l^T J_l per landmark
    W: sp.csr_matrix     # (12 n_cams, 4 n_pts)  J_p^T J_l
    bp: np.ndarray       # (n_cams, 12)      J_p^T r
    bl: np.ndarray       # (n_pts, 4)        J_l^T r
    cost: float


def linearize(P: np.ndarray, Xh: np.ndarray, prob) -> Linearization:
    cam, pt = prob.cam_idx, prob.pt_idx
    r = residual(P, Xh, cam, pt, prob.meas)
    Jp, Jl = jacobians(P, Xh, cam, pt)
    U = sum_by(cam, prob.n_cams, np.einsum("nri,nrj->nij", Jp, Jp))
    V = sum_by(pt, prob.n_pts, np.einsum("nri,nrj->nij", Jl, Jl))
    bp = sum_by(cam, prob.n_cams, np.einsum("nri,nr->ni", Jp, r))
    bl = sum_by(pt, prob.n_pts, np.einsum("nri,nr->ni", Jl, r))
    Wk = np.einsum("nri,nrj->nij", Jp, Jl)                       # (n, 12, 4)
    rows = (12 * cam.astype(np.int64))[:, None, None] + np.arange(12)[None, :, None]
    cols = (4 * pt.astype(np.int64))[:, None, None] + np.arange(4)[None, None, :]
    rows, cols = np.broadcast_arrays(rows, cols)
    W = sp.csr_matrix((Wk.ravel(), (rows.ravel(), cols.ravel())), shape=(12 * prob.n_cams, 4 * prob.n_pts))
    return Linearization(U=U, V=V, W=W, bp=bp, bl=bl, cost=float(np.sum(r * r)))


def tangent_basis(x: np.ndarray) -> np.ndarray:
    """Orthonormal basis of {d : x_k^T d = 0} for each row x_k of a stack of
    unit vectors, (n, d, d-1), from a Householder QR of x_k."""
    Q, _ = np.linalg.qr(x[:, :, None], mode="complete")
    return Q[:, :, 1:]


def damped(A: np.ndarray, lam: float) -> np.ndarray:
    """A + lam D^T D with D^T D = diag(A) per block, floored at DAMP_FLOOR
    times the largest diagonal entry of the block (Marquardt)."""
    d = np.diagonal(A, axis1=1, axis2=2).copy()
    d = np.maximum(d, DAMP_FLOOR * d.max(axis=1, keepdims=True))
    out = A.copy()
    idx = np.arange(A.shape[1])
    out[:, idx, idx] += lam * d
    return out


@dataclass
class RiemannianSystem:
    Bp: np.ndarray           # (n_cams, 12, 11)
    Bl: np.ndarray           # (n_pts, 4, 3)
    Ut: np.ndarray           # (n_cams, 11, 11)  U~_lambda
    Vt: np.ndarray           # (n_pts, 3, 3)     V~_lambda
    Wt: sp.csr_matrix        # (11 n_cams, 3 n_pts)
    bpt: np.ndarray          # (11 n_cams,)
    blt: np.ndarray          # (3 n_pts,)

    def apply_Uinv(self, v: np.ndarray) -> np.ndarray:
        n = self.Ut.shape[0]
        return np.linalg.solve(self.Ut, v.reshape(n, 11, 1)).reshape(-1)

    def apply_Vinv(self, v: np.ndarray) -> np.ndarray:
        n = self.Vt.shape[0]
        return np.linalg.solve(self.Vt, v.reshape(n, 3, 1)).reshape(-1)

    def apply_M(self, x: np.ndarray) -> np.ndarray:
        """M x = U~^-1 W~ V~^-1 W~^T x, the operator of the series (29)."""
        return self.apply_Uinv(self.Wt @ self.apply_Vinv(self.Wt.T @ x))


def riemannian_system(P: np.ndarray, Xh: np.ndarray, lin: Linearization, lam: float) -> RiemannianSystem:
    """The projected, damped normal equations (20)-(26) at (P, Xh)."""
    Bp, Bl = tangent_basis(P), tangent_basis(Xh)
    Ut = np.einsum("nai,nab,nbj->nij", Bp, damped(lin.U, lam), Bp)
    Vt = np.einsum("nai,nab,nbj->nij", Bl, damped(lin.V, lam), Bl)
    Bps, Bls = block_diag_sparse(Bp), block_diag_sparse(Bl)
    Wt = (Bps.T @ lin.W @ Bls).tocsr()
    bpt = Bps.T @ lin.bp.reshape(-1)
    blt = Bls.T @ lin.bl.reshape(-1)
    return RiemannianSystem(Bp=Bp, Bl=Bl, Ut=Ut, Vt=Vt, Wt=Wt, bpt=bpt, blt=blt)


def series_solve(rs: RiemannianSystem, order: int, rtol: float = 0.0, info: dict | None = None):
    """Camera update by the truncated power series of the inverse Riemannian
    Schur complement (27)-(29), dx_p = -sum_{i=0..m} M^i U~^-1 g with
    g = b~_p - W~ V~^-1 b~_l; then the landmarks by back-substitution,
    dx_l = -V~^-1 (b~_l + W~^T dx_p).  Tangent coordinates.  rtol > 0: the
    early stop of Sec. 5.2 as in the first stage (reading R6): after the first
    term t >= 1 with ||x_t|| <= rtol ||x_0 + ... + x_t||, norms over all
    cameras; info["terms"] receives the number of terms after the first."""
    g = rs.bpt - rs.Wt @ rs.apply_Vinv(rs.blt)
    x = -rs.apply_Uinv(g)
    acc = x.copy()
    used = 0
    for _ in range(order):
        x = rs.apply_M(x)
        acc = acc + x
        used += 1
        if rtol > 0 and np.linalg.norm(x) <= rtol * np.linalg.norm(acc):
            break
    if info is not None:
        info["terms"] = used
    dxl = -rs.apply_Vinv(rs.blt + rs.Wt.T @ acc)
    return acc, dxl


def back_project(rs: RiemannianSystem, dxp: np.ndarray, dxl: np.ndarray):
    """Ambient updates dP = B_p dx_p (n_cams, 12) and dX = B_l dx_l (n_pts, 4)."""
    n_p, n_l = rs.Bp.shape[0], rs.Bl.shape[0]
    dP = np.einsum("nik,nk->ni", rs.Bp, dxp.reshape(n_p, 11))
    dX = np.einsum("nik,nk->ni", rs.Bl, dxl.reshape(n_l, 3))
    return dP, dX


def retract(x: np.ndarray, dx: np.ndarray) -> np.ndarray:
    """Add the update and normalise each row (unit sphere)."""
    y = x + dx
    return y / np.linalg.norm(y, axis=1, keepdims=True)


def step(P: np.ndarray, Xh: np.ndarray, lin: Linearization, lam: float, order: int, rtol: float = 0.0,
         info: dict | None = None):
    """One RiPoBA update: ambient (dP, dX) in the tangent spaces."""
    rs = riemannian_system(P, Xh, lin, lam)
    return back_project(rs, *series_solve(rs, order, rtol, info))


# ----------------------------------------------------------------------------
# Levenberg-Marquardt loop and the hand-over from the first stage
# ----------------------------------------------------------------------------
@dataclass
class Options:
    order: int = 20
    max_iters: int = 50
    ftol: float = 1e-6
    lambda0: float = 1e-4
    lambda_min: float = 1e-12
    lambda_max: float = 1e12
    series_rtol: float = 0.0


@dataclass
class Result:
    P: np.ndarray
    Xh: np.ndarray
    cost: float
    cost0: float
    lam: float
    iters: int
    trace_cost: list = field(default_factory=list)
    trace_accept: list = field(default_factory=list)
    stop: str = "max_iters"


def from_first_stage(P: np.ndarray, X: np.ndarray):
    """Stage-2 variables from a stage-1 solution: each camera and each
    homogeneous landmark (X, 1) normalised to unit length."""
    Xh = np.concatenate([X, np.ones((X.shape[0], 1))], axis=1)
    return P / np.linalg.norm(P, axis=1, keepdims=True), Xh / np.linalg.norm(Xh, axis=1, keepdims=True)


def lm_solve(prob, P0: np.ndarray, Xh0: np.ndarray, opts: Options | None = None) -> Result:
    """Joint LM over cameras and landmarks on their spheres, each step the
    RiPoBA update; accept iff the cost decreases (NaN rejects); lambda / 10 on
    accept, x 10 on reject, clamped; stop on ftol of an accepted step."""
    opts = opts or Options()
    P, Xh = P0.copy(), Xh0.copy()
    f = cost(P, Xh, prob)
    res = Result(P=P, Xh=Xh, cost=f, cost0=f, lam=opts.lambda0, iters=0)
    lam = opts.lambda0
    lin = linearize(P, Xh, prob)
    for it in range(opts.max_iters):
        dP, dX = step(P, Xh, lin, lam, opts.order, opts.series_rtol)
        Pn, Xn = retract(P, dP), retract(Xh, dX)
        fn = cost(Pn, Xn, prob)
        res.trace_cost.append(fn)
        res.iters = it + 1
        if fn < f:
            res.trace_accept.append(1)
            rel = (f - fn) / f
            P, Xh, f = Pn, Xn, fn
            lam = max(lam / 10.0, opts.lambda_min)
            lin = linearize(P, Xh, prob)
            if opts.ftol > 0 and rel < opts.ftol:
                res.stop = "ftol"
                break
        else:
            res.trace_accept.append(0)
            lam = min(lam * 10.0, opts.lambda_max)
    res.P, res.Xh, res.cost, res.lam = P, Xh, f, lam
    return res
