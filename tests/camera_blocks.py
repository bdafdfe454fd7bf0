"""Checks of the damped camera block inverses K_i (Sec. 4.3, Eq. (22)) against
the oracle, shared by the parity and full-size GPU tests."""
import numpy as np

from oracle import povar_oracle as O


def oracle_K(P, U, lam, manifold="sphere"):
    """K_i = B_i (B_i^T U_i,lambda B_i)^-1 B_i^T with the oracle's damping and
    its orthonormal tangent basis B_i (the identity in Euclidean mode)."""
    n = len(P)
    B = O.tangent_basis(P) if manifold == "sphere" else np.broadcast_to(np.eye(12), (n, 12, 12))
    Ut = np.einsum("nik,nij,njl->nkl", B, O.damped(U, lam), B)
    return np.einsum("nik,nkl,njl->nij", B, np.linalg.inv(Ut), B)


def err_over_bound(K, Kr, U, Ur, lam):
    """Per camera, |K - Kr|_2 over the first-order perturbation bound of an
    inverse, 2 |Kr|_2^2 ((1 + lam) |U - Ur|_F + 2 n^2 eps |Ur_lam|_2): U is the
    GPU's U_i and Ur the oracle's, and the second term the backward error of a
    12 x 12 Cholesky factorisation and inversion.  Values <= 1 pass."""
    nK = np.linalg.norm(Kr, 2, axis=(1, 2))
    dU = np.linalg.norm((U - Ur).reshape(len(U), -1), axis=1)
    nUl = np.linalg.norm(O.damped(Ur, lam), 2, axis=(1, 2))
    bound = 2 * nK ** 2 * ((1 + lam) * dU + 2 * 144 * np.finfo(float).eps * nUl)
    return np.linalg.norm(K - Kr, 2, axis=(1, 2)) / bound
