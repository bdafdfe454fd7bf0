"""The check that the GPU tests apply to the damped camera block inverses
K_i (Sec. 4.3, Eq. (22)), exercised on the CPU: an independent FP64 form of
K_i with rounding-level noise in U_i passes it, and plausible mistakes fail
it (no tangent projection, the wrong damping, one camera's block lost)."""
import numpy as np
import pytest

from oracle import povar_oracle as O
from paper_2405_05079_amd import synth

from camera_blocks import err_over_bound, oracle_K


@pytest.fixture(scope="module")
def scene():
    prob = synth.make_problem(30, 129, track=("geom", 0.25), seed=7)
    P, X, f = O.initial_state(prob, prob.cams0)
    return P, O.linearize(P, X, prob).U


def kkt_K(P, U, lam, project=True):
    """K_i = U_l^-1 - w w^T / (p^T w), w = U_l^-1 p, through a Cholesky
    factor (the form the kernels take), independent of the tangent basis."""
    L = np.linalg.cholesky(O.damped(U, lam))
    Li = np.linalg.inv(L)
    Ui = Li.transpose(0, 2, 1) @ Li
    if not project:
        return Ui
    w = np.einsum("nij,nj->ni", Ui, P)
    h = np.einsum("ni,ni->n", P, w)
    return Ui - w[:, :, None] * w[:, None, :] / h[:, None, None]


@pytest.mark.parametrize("lam", [1e-12, 1e-4, 1.0])
def test_rounding_level_differences_pass(scene, lam):
    P, U = scene
    rng = np.random.default_rng(3)
    Up = U * (1 + 1e-13 * rng.standard_normal(U.shape))
    Up = (Up + Up.transpose(0, 2, 1)) / 2
    assert err_over_bound(kkt_K(P, Up, lam), oracle_K(P, U, lam), Up, U, lam).max() <= 1.0


@pytest.mark.parametrize("lam", [1e-4, 1.0])
def test_planted_mistakes_fail(scene, lam):
    P, U = scene
    Kr = oracle_K(P, U, lam)
    assert err_over_bound(kkt_K(P, U, lam, project=False), Kr, U, U, lam).max() > 1.0   # no projection
    Ui_eye = np.linalg.inv(U + lam * np.eye(12))                                        # lambda I damping
    w = np.einsum("nij,nj->ni", Ui_eye, P)
    K_eye = Ui_eye - w[:, :, None] * w[:, None, :] / np.einsum("ni,ni->n", P, w)[:, None, None]
    assert err_over_bound(K_eye, Kr, U, U, lam).max() > 1.0
    assert err_over_bound(kkt_K(P, U, 2 * lam), Kr, U, U, lam).max() > 1.0              # damping doubled
    K = kkt_K(P, U, lam)
    K[5] = 0.0                                                                           # a block lost
    assert err_over_bound(K, Kr, U, U, lam).max() > 1.0
