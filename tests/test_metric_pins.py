"""Pins of the metric-upgrade oracle (App. D) against what geometry and
calculus fix, independently of the oracle's own code paths (CPU only)."""
import numpy as np
import pytest

from oracle import metric_oracle as MO
from paper_2405_05079_amd import synth


def scene(n_cams=12, seed=3):
    p = synth.make_problem(n_cams, 100, seed=seed, calibrated=True, sigma=0.0)
    return p, p.cams_gt.reshape(-1, 3, 4), p.K_gt


def projective_view(G, seed):
    """The calibrated cameras through a random projective frame H_p, each
    with a random scale and sign: what a projective reconstruction returns."""
    rng = np.random.default_rng(seed)
    Hp = np.eye(4) + 0.3 * rng.standard_normal((4, 4))
    s = rng.uniform(0.5, 2.0, len(G)) * rng.choice([-1.0, 1.0], len(G))
    return s[:, None, None] * (G @ Hp), Hp


def ground_truth_pose(G, K):
    """R_i, t_i of G_i = s_i K_i [R_i | t_i] (det R_i = 1)."""
    B = np.linalg.solve(K, G)
    s = np.cbrt(np.linalg.det(B[:, :, :3]))
    return B[:, :, :3] / s[:, None, None], B[:, :, 3] / s[:, None]


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_exact_calibrated_scene_is_recovered_up_to_similarity(seed):
    """A metric reconstruction is fixed up to a similarity; with camera 0 as
    the reference the recovered poses are R_i R_0^T and
    sigma (t_i - R_i R_0^T t_0) for one scale sigma, at zero cost; the
    landmarks map to sigma (R_0 X + t_0)."""
    p, G, K = scene(seed=seed)
    P, Hp = projective_view(G, seed)
    res = MO.lm_solve(P, K)
    assert res.cost < 1e-24 * res.cost0
    R, t, _ = MO.euclidean_cameras(P, K, res)
    Rg, tg = ground_truth_pose(G, K)
    Rrel = Rg @ Rg[0].T
    trel = tg - np.einsum("nab,b->na", Rrel, tg[0])
    np.testing.assert_allclose(R, Rrel, atol=1e-10)
    sigma = np.sum(t * trel) / np.sum(trel * trel)
    np.testing.assert_allclose(t, sigma * trel, atol=1e-10 * np.abs(t).max())
    Xp = np.linalg.solve(Hp, np.c_[p.pts_gt, np.ones(p.n_pts)].T).T     # the landmarks in the projective frame
    Xm = MO.metric_points(Xp, res)
    np.testing.assert_allclose(Xm, sigma * (p.pts_gt @ Rg[0].T + tg[0]), atol=1e-9 * np.abs(Xm).max())


def test_scale_is_the_least_squares_one():
    """alpha_i minimises ||alpha M_i - I||_F: a one-column least-squares problem."""
    rng = np.random.default_rng(4)
    Q = rng.standard_normal((7, 3, 4))
    red = MO.reduced(rng.standard_normal(3), Q, np.diag([1.1, 0.9, 1.0]))
    for i in range(7):
        a, *_ = np.linalg.lstsq(red.M[i].reshape(9, 1), np.eye(3).reshape(9), rcond=None)
        assert abs(red.alpha[i] - a[0]) <= 1e-12 * abs(a[0])


def test_derivative_theorem_against_central_differences():
    """H~ H~^T is quadratic in H~, so central differences are exact up to
    rounding."""
    rng = np.random.default_rng(5)
    Ht = rng.standard_normal((4, 3))
    D = MO.d_omega_d_htilde(Ht)
    h = 1e-3
    for k in range(12):
        E = np.zeros(12)
        E[k] = h
        Ep = (Ht.reshape(-1, order="F") + E).reshape(4, 3, order="F")
        Em = (Ht.reshape(-1, order="F") - E).reshape(4, 3, order="F")
        fd = ((Ep @ Ep.T) - (Em @ Em.T)).reshape(-1, order="F") / (2 * h)
        np.testing.assert_allclose(D[:, k], fd, rtol=0, atol=1e-12)


def test_reduced_jacobian_against_central_differences():
    rng = np.random.default_rng(6)
    _, G, K = scene(n_cams=6, seed=7)
    P, _ = projective_view(G, 8)
    Q, _ = MO.normalized_cameras(P, K)
    c = 0.2 * rng.standard_normal(3)
    red = MO.reduced(c, Q, K[0])
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (MO.reduced(c + e, Q, K[0]).r - MO.reduced(c - e, Q, K[0]).r) / (2 * h)
        np.testing.assert_allclose(red.J[..., k], fd, rtol=1e-6, atol=1e-8 * np.abs(red.J).max())


def test_reference_camera_term_vanishes():
    """In the reference frame camera 0 is K_0 [I | 0]: Q_0 H~ = I for every c."""
    _, G, K = scene(n_cams=5, seed=9)
    P, _ = projective_view(G, 10)
    Q, T = MO.normalized_cameras(P, K)
    np.testing.assert_allclose(P[0] @ T, np.c_[np.eye(3), np.zeros(3)], atol=1e-12)
    for c in (np.zeros(3), np.array([0.3, -1.0, 2.0])):
        red = MO.reduced(c, Q, K[0])
        assert abs(red.alpha[0] - 1.0) < 1e-12
        assert np.abs(red.r[0]).max() < 1e-12


def test_invariant_to_projective_frame_and_camera_scales():
    """Another projective frame and other camera scales give the same metric
    poses: the upgrade sees the cameras only through their projective class."""
    p, G, K = scene(seed=14)
    P, _ = projective_view(G, 15)
    rng = np.random.default_rng(16)
    H2 = np.eye(4) + 0.2 * rng.standard_normal((4, 4))
    P2 = rng.uniform(0.3, 3.0, len(P))[:, None, None] * (P @ H2)
    R1, t1, _ = MO.euclidean_cameras(P, K, MO.lm_solve(P, K))
    R2, t2, _ = MO.euclidean_cameras(P2, K, MO.lm_solve(P2, K))
    np.testing.assert_allclose(R2, R1, atol=1e-10)
    k = np.sum(t2 * t1) / np.sum(t1 * t1)
    np.testing.assert_allclose(t2, k * t1, atol=1e-10 * np.abs(t2).max())


def test_stratified_pipeline_on_a_calibrated_scene():
    """Sec. 3 end to end on noisy measurements: PoVar from random cameras, the
    projective refinement, then the metric upgrade; the relative rotations
    come back within 2 degrees (noise 1e-3 on image coordinates of ~0.3)."""
    from oracle import povar_oracle as O1
    from oracle import ripoba_oracle as R
    prob = synth.make_problem(8, 150, seed=21, calibrated=True, track=("uniform", 3, 5))
    r1 = O1.lm_solve(prob, opts=O1.Options(order=20, max_iters=60, ftol=1e-10))
    r2 = R.lm_solve(prob, *R.from_first_stage(r1.P, r1.X), R.Options(max_iters=30, ftol=1e-12))
    assert r2.cost < synth.SIGMA ** 2 * 2 * prob.n_obs
    P = r2.P.reshape(-1, 3, 4)
    res = MO.lm_solve(P, prob.K_gt)
    assert res.cost < 1e-2 * res.cost0
    Rr, _, _ = MO.euclidean_cameras(P, prob.K_gt, res)
    Rg, _ = ground_truth_pose(prob.cams_gt.reshape(-1, 3, 4), prob.K_gt)
    cosang = (np.einsum("nab,nab->n", Rr, Rg @ Rg[0].T) - 1.0) / 2.0
    assert np.degrees(np.arccos(np.clip(cosang, -1.0, 1.0))).max() < 2.0
