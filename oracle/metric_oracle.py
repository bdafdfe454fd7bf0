"""Plain FP64 CPU oracle for the metric upgrade (autocalibration) that
follows the projective refinement: the supplement's "Metric Upgrade"
section (App. D), with the projective-to-metric matrix
H = [[A, 0], [c^T, 1]] and its three left columns H~.

TEST INFRASTRUCTURE.  Only the tests may import this module.  It shares no
code with the HIP library and does not import the package's binding.

What it computes, in the paper's order:

* the SE(3) constraint: for every camera i, Q_i = K_i^-1 P_i (P_i the
  projective camera, K_i its known intrinsics) must satisfy
  alpha_i Q_i H~ H~^T Q_i^T = I for some scale alpha_i;
* the objective: the sum over cameras of ||alpha_i Q_i H~(c) H~(c)^T Q_i^T - I||_F^2,
  minimised over the plane at infinity c (3 values) and the scales alpha_i by
  variable projection: each alpha_i is linear, eliminated in closed form, and
  the reduced residual is minimised over c with Levenberg-Marquardt;
* the derivative of H~ H~^T with respect to H~ (the theorem quoted in App. D),
  chained through H~(c) and Q_i ... Q_i^T.

Readings where the supplement is silent (the same in the HIP path):

* H~ depends on c alone, so A is fixed: the projective frame is first moved
  so that the reference camera (camera 0) is [I | 0]; with its intrinsics
  known, A = K_0 and camera 0 becomes K_0 [I | 0] (its own term then
  vanishes for every c);
* the theorem's Kronecker expression depends on the vec convention; here
  vec stacks columns, and d vec(H~ H~^T) = (I_16 + T)(H~ (x) I_4) d vec(H~)
  with T the 16 x 16 matrix taking vec(Y) to vec(Y^T);
* alpha_i = tr(M_i) / ||M_i||_F^2 with M_i = Q_i H~ H~^T Q_i^T (the
  least-squares scale); the Jacobian of the reduced residual is the full one,
  d(alpha_i M_i) = alpha_i dM_i + M_i d alpha_i;
* LM as in the first stage: Marquardt damping on the diagonal of J^T J
  (floored at 1e-12 of its largest entry), accept iff the cost decreases,
  lambda / 10 on accept and x 10 on reject, c starting at 0, stop after
  max_iters, when an accepted step changes the cost by less than ftol
  (relative), or when lambda reaches its cap of 1e12 (no step lowers the
  cost any more);
* Euclidean cameras: P_i H = s_i K_i [R_i | t_i] with s_i^2 = 1 / alpha_i;
  the sign of s_i makes det(R_i) positive, and R_i is the orthogonal polar
  factor of K_i^-1 P_i H~ / s_i (the nearest rotation).

parity pinned: see tests/test_metric_pins.py (exact calibrated scenes seen
through a random projective frame are recovered, the closed-form scale is
the least-squares one, the derivative theorem and the Jacobian against
central differences, the reference camera's term vanishes, invariance to the
projective frame and to camera scales).  lm_solve is pinned by its end point
(exact recovery on noise-free scenes); its iterates in between are parity
unpinned.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def reference_frame(P: np.ndarray) -> np.ndarray:
    """T (4x4) with P_0 T = [I | 0]: P_0 = [M | m], T = [[M^-1, -M^-1 m], [0, 1]]."""
    M, m = P[0, :, :3], P[0, :, 3]
    Mi = np.linalg.inv(M)
    T = np.eye(4)
    T[:3, :3] = Mi
    T[:3, 3] = -Mi @ m
    return T


def normalized_cameras(P: np.ndarray, K: np.ndarray):
    """Q_i = K_i^-1 P_i T in the reference frame; returns (Q (n,3,4), T)."""
    T = reference_frame(P)
    return np.linalg.solve(K, P @ T), T


def h_tilde(c: np.ndarray, K0: np.ndarray) -> np.ndarray:
    """The three left columns of H = [[K_0, 0], [c^T, 1]]."""
    Ht = np.zeros((4, 3))
    Ht[:3] = K0
    Ht[3] = c
    return Ht


def transpose_matrix(m: int, n: int) -> np.ndarray:
    """T with T vec(Y) = vec(Y^T) for Y of size m x n (vec stacks columns)."""
    T = np.zeros((m * n, m * n))
    for i in range(m):
        for j in range(n):
            T[i * n + j, j * m + i] = 1.0
    return T


def d_omega_d_htilde(Ht: np.ndarray) -> np.ndarray:
    """d vec(H~ H~^T) / d vec(H~), 16 x 12: (I + T)(H~ (x) I_4)."""
    return (np.eye(16) + transpose_matrix(4, 4)) @ np.kron(Ht, np.eye(4))


@dataclass
class Reduced:
    M: np.ndarray       # (n, 3, 3)  Q_i H~ H~^T Q_i^T
    alpha: np.ndarray   # (n,)       closed-form scales
    r: np.ndarray       # (n, 3, 3)  alpha_i M_i - I
    J: np.ndarray       # (n, 3, 3, 3) d r_i / d c_k in the last axis
    cost: float


def reduced(c: np.ndarray, Q: np.ndarray, K0: np.ndarray) -> Reduced:
    Ht = h_tilde(c, K0)
    Om = Ht @ Ht.T
    M = Q @ Om @ np.transpose(Q, (0, 2, 1))
    mm = np.einsum("nab,nab->n", M, M)
    alpha = np.trace(M, axis1=1, axis2=2) / mm
    r = alpha[:, None, None] * M - np.eye(3)
    D = d_omega_d_htilde(Ht)
    J = np.zeros(M.shape + (3,))
    for k in range(3):
        # c_k is the entry (3, k) of H~: column-stacked index 4 k + 3
        dOm = D[:, 4 * k + 3].reshape(4, 4, order="F")
        dM = Q @ dOm @ np.transpose(Q, (0, 2, 1))
        dalpha = (np.trace(dM, axis1=1, axis2=2) - 2.0 * alpha * np.einsum("nab,nab->n", M, dM)) / mm
        J[..., k] = alpha[:, None, None] * dM + dalpha[:, None, None] * M
    return Reduced(M=M, alpha=alpha, r=r, J=J, cost=float(np.sum(r * r)))


@dataclass
class Options:
    max_iters: int = 100
    ftol: float = 1e-14
    lambda0: float = 1e-4


@dataclass
class Result:
    c: np.ndarray
    alpha: np.ndarray
    cost: float
    cost0: float
    iters: int
    T: np.ndarray
    H: np.ndarray          # T [[K_0, 0], [c^T, 1]]: projective -> metric frame
    trace_cost: list = field(default_factory=list)
    trace_accept: list = field(default_factory=list)


def lm_solve(P: np.ndarray, K: np.ndarray, opts: Options | None = None) -> Result:
    opts = opts or Options()
    Q, T = normalized_cameras(P, K)
    K0 = K[0]
    c = np.zeros(3)
    red = reduced(c, Q, K0)
    cost0 = red.cost
    lam = opts.lambda0
    tc, ta = [], []
    it = 0
    while it < opts.max_iters:
        Jm = red.J.reshape(-1, 3)
        A = Jm.T @ Jm
        g = Jm.T @ red.r.reshape(-1)
        d = np.diag(A).copy()
        d = np.maximum(d, 1e-12 * d.max())
        it += 1
        try:
            delta = np.linalg.solve(A + lam * np.diag(d), -g)
            trial = reduced(c + delta, Q, K0)
            f_new = trial.cost
        except np.linalg.LinAlgError:
            f_new = np.inf
        ok = bool(np.isfinite(f_new) and f_new < red.cost)
        tc.append(float(f_new))
        ta.append(ok)
        if ok:
            done = red.cost - f_new <= opts.ftol * red.cost
            c, red = c + delta, trial
            lam = max(lam / 10.0, 1e-12)
            if done:
                break
        else:
            lam = min(lam * 10.0, 1e12)
            if lam >= 1e12:
                break
    H = np.zeros((4, 4))
    H[:3, :3] = K0
    H[3, :3] = c
    H[3, 3] = 1.0
    return Result(c=c, alpha=red.alpha, cost=red.cost, cost0=cost0, iters=it, T=T, H=T @ H,
                  trace_cost=tc, trace_accept=ta)


def euclidean_cameras(P: np.ndarray, K: np.ndarray, res: Result):
    """(R (n,3,3), t (n,3), s (n,)) with P_i H = s_i K_i [R_i | t_i]."""
    Pm = P @ res.H
    B = np.linalg.solve(K, Pm)
    s = 1.0 / np.sqrt(res.alpha)
    s = np.where(np.linalg.det(B[:, :, :3]) < 0, -s, s)
    B = B / s[:, None, None]
    U, _, Vt = np.linalg.svd(B[:, :, :3])
    R = U @ Vt
    return R, B[:, :, 3], s


def metric_points(Xh: np.ndarray, res: Result) -> np.ndarray:
    """Landmarks in the metric frame: H^-1 X, then divided by the last coordinate."""
    Y = np.linalg.solve(res.H, Xh.T).T
    return Y[:, :3] / Y[:, 3:]
