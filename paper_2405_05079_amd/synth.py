"""Seeded synthetic bundle-adjustment problems shaped like the paper's BAL workloads.

The paper evaluates on the BAL problems (Sec. 5, "Dataset"; supplement table of
problem sizes): it keeps only the image measurements, draws every camera from an
isotropic Gaussian and derives landmarks by the closed form (8).  Those files are
not available here, so this module builds stand-ins with the same sizes and
track statistics.  It holds no arithmetic of the solver itself: it only draws
geometry, projects it with a pinhole model and draws the random initial cameras
that both the solver and its checker take as input.

Recipe (identical on every machine for a given numpy version):
  * ground-truth camera G (3x4) with iid N(0,1) entries; its third row is
    rescaled so that G[2,:3] has unit l1 norm and G[2,3] = 5, which puts every
    point of [-1,1]^3 at depth 4..6; the camera is then scaled to unit Frobenius
    norm (a projective camera is defined up to scale);
  * points uniform in [-1,1]^3;
  * measurement = perspective projection + N(0, sigma^2 I2), sigma = 1e-3;
  * tracks: each point is seen by L distinct cameras, L depending on the
    workload (uniform 4..8, or 1 + geometric), cameras drawn uniformly or with
    Zipf weights rank^-0.8 over a shuffled rank (heavy-tailed views per camera);
  * optional outliers: a Bernoulli fraction of measurements replaced by uniform
    draws over the bounding box of the inliers;
  * initial cameras: unit-norm Gaussian 12-vectors from a separate seed stream
    (Sec. 5 draws cameras from an isotropic Gaussian; they are normalised here
    because the solver keeps every camera on the unit sphere of R^12).
  * calibrated scenes (for the metric upgrade, which needs known intrinsics):
    camera centres at distance 5 from the origin in uniformly random
    directions, optical axis through the origin, random roll; intrinsics
    K = [[f, 0, u], [0, f, v], [0, 0, 1]] with f ~ U(0.8, 1.2) and
    u, v ~ U(-0.05, 0.05); G = K [R | t] scaled to unit Frobenius norm.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Workload shapes.  Key = workload number; the names say what each one is.
WORKLOADS = {
    1: dict(name="plain-20cam-500pt", n_cams=20, n_pts=500, track=("uniform", 4, 8),
            cam_choice="uniform", outlier_frac=0.0, eta=0.01, order=10, iters=50,
            precision="fp64"),
    2: dict(name="mid-250cam-60kpt", n_cams=250, n_pts=60_000, track=("geom", 0.25),
            cam_choice="uniform", outlier_frac=0.0, eta=0.01, order=20, iters=100,
            precision="fp32_bulk"),
    3: dict(name="large-1800cam-1Mpt", n_cams=1800, n_pts=1_000_000, track=("geom", 0.25),
            cam_choice="uniform", outlier_frac=0.01, eta=0.01, order=20, iters=50,
            precision="fp32_bulk"),
    5: dict(name="xl-13700cam-4.5Mpt", n_cams=13_700, n_pts=4_500_000, track=("geom", 1 / 5.5),
            cam_choice="zipf", outlier_frac=0.0, eta=0.01, order=30, iters=50,
            precision="fp32_bulk"),
}

SIGMA = 1e-3


@dataclass
class Problem:
    """One bundle-adjustment instance: observations (camera, point, 2-D measurement)."""
    n_cams: int
    n_pts: int
    cam_idx: np.ndarray      # (n_obs,) int32
    pt_idx: np.ndarray       # (n_obs,) int32
    meas: np.ndarray         # (n_obs, 2) float64
    cams0: np.ndarray        # (n_cams, 12) float64, row-major 3x4, unit norm
    eta: float = 0.01
    order: int = 20
    iters: int = 50
    cams_gt: np.ndarray | None = None   # diagnostics only
    pts_gt: np.ndarray | None = None
    K_gt: np.ndarray | None = None      # (n_cams, 3, 3) intrinsics of calibrated scenes
    seeds: dict = field(default_factory=dict)
    name: str = ""

    @property
    def n_obs(self) -> int:
        return int(self.cam_idx.shape[0])


def _gt_cameras(rng: np.random.Generator, n_cams: int) -> np.ndarray:
    G = rng.standard_normal((n_cams, 3, 4))
    G[:, 2, :3] /= np.abs(G[:, 2, :3]).sum(axis=1, keepdims=True)
    G[:, 2, 3] = 5.0
    G /= np.linalg.norm(G.reshape(n_cams, 12), axis=1)[:, None, None]
    return G


def _calibrated_cameras(rng: np.random.Generator, n_cams: int):
    """Cameras K [R | t] looking at the origin from distance 5; returns
    (G unit-norm 3x4, K 3x3)."""
    d = rng.standard_normal((n_cams, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    C = 5.0 * d
    z = -d
    a = rng.standard_normal((n_cams, 3))
    x = a - np.sum(a * z, axis=1, keepdims=True) * z
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    R = np.stack([x, y, z], axis=1)                       # rows: camera axes
    t = -np.einsum("nab,nb->na", R, C)
    K = np.zeros((n_cams, 3, 3))
    f = rng.uniform(0.8, 1.2, size=n_cams)
    K[:, 0, 0] = f
    K[:, 1, 1] = f
    K[:, 0, 2] = rng.uniform(-0.05, 0.05, size=n_cams)
    K[:, 1, 2] = rng.uniform(-0.05, 0.05, size=n_cams)
    K[:, 2, 2] = 1.0
    G = np.einsum("nab,nbc->nac", K, np.concatenate([R, t[:, :, None]], axis=2))
    G /= np.linalg.norm(G.reshape(n_cams, 12), axis=1)[:, None, None]
    return G, K


def calibrated_cameras(n_cams: int, seed: int):
    """Only the cameras of a calibrated scene (no points): (G (n, 3, 4) unit
    norm, K (n, 3, 3)), for checks of the metric upgrade at any size."""
    return _calibrated_cameras(np.random.default_rng(seed), n_cams)


def _track_lengths(rng, n_pts, n_cams, track):
    kind = track[0]
    if kind == "uniform":
        lo, hi = track[1], track[2]
        L = rng.integers(lo, hi + 1, size=n_pts)
    elif kind == "geom":
        L = 1 + rng.geometric(track[1], size=n_pts)
    else:
        raise ValueError(kind)
    return np.minimum(L, n_cams).astype(np.int64)


def _draw_distinct(rng, L, n_cams, weights):
    """For each point p draw L[p] distinct cameras (uniform or weighted).

    Draws with replacement, then redraws the duplicate entries of a row until
    every row is duplicate-free."""
    n_pts = L.shape[0]
    row = np.repeat(np.arange(n_pts, dtype=np.int64), L)
    if weights is None:
        draw = lambda k: rng.integers(0, n_cams, size=k)
    else:
        cdf = np.cumsum(weights / weights.sum())
        cdf[-1] = 1.0
        draw = lambda k: np.minimum(np.searchsorted(cdf, rng.random(k), side="right"), n_cams - 1)
    cam = draw(row.shape[0]).astype(np.int64)
    for _ in range(1000):
        key = row * n_cams + cam
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup_sorted = np.zeros(ks.shape[0], dtype=bool)
        dup_sorted[1:] = ks[1:] == ks[:-1]
        if not dup_sorted.any():
            break
        dup = order[dup_sorted]
        cam[dup] = draw(dup.shape[0])
    else:  # pragma: no cover
        raise RuntimeError("could not draw distinct cameras")
    return row, cam


def make_problem(n_cams: int, n_pts: int, *, track=("geom", 0.25), cam_choice="uniform",
                 outlier_frac=0.0, eta=0.01, order=20, iters=50, seed=0, init_seed=None,
                 sigma=SIGMA, affine=False, calibrated=False, name="") -> Problem:
    """Draw one problem.  `affine=True` gives cameras with third row (0,0,0,1)
    (depth 1 everywhere), used by checks that need a known zero-cost minimum;
    `calibrated=True` gives cameras K [R | t] with known intrinsics (K_gt)."""
    if init_seed is None:
        init_seed = seed + 1
    for attempt in range(64):
        rng = np.random.default_rng([seed, attempt]) if attempt else np.random.default_rng(seed)
        K = None
        if calibrated:
            G, K = _calibrated_cameras(rng, n_cams)
        else:
            G = _gt_cameras(rng, n_cams)
        if affine:
            G[:, 2, :] = 0.0
            G[:, 2, 3] = 1.0
        X = rng.uniform(-1.0, 1.0, size=(n_pts, 3))
        L = _track_lengths(rng, n_pts, n_cams, track)
        weights = None
        if cam_choice == "zipf":
            rank = rng.permutation(n_cams) + 1
            weights = rank.astype(np.float64) ** -0.8
        row, cam = _draw_distinct(rng, L, n_cams, weights)
        if np.bincount(cam, minlength=n_cams).min() > 0:
            break
    else:  # pragma: no cover
        raise RuntimeError("could not cover every camera")
    Xh = np.concatenate([X[row], np.ones((row.shape[0], 1))], axis=1)
    y = np.einsum("nab,nb->na", G[cam], Xh)
    meas = y[:, :2] / y[:, 2:3]
    if sigma > 0:
        meas = meas + sigma * rng.standard_normal(meas.shape)
    if outlier_frac > 0:
        lo, hi = meas.min(axis=0), meas.max(axis=0)
        out = rng.random(meas.shape[0]) < outlier_frac
        meas[out] = rng.uniform(lo, hi, size=(int(out.sum()), 2))
    perm = rng.permutation(row.shape[0])
    cam_idx = cam[perm].astype(np.int32)
    pt_idx = row[perm].astype(np.int32)
    meas = np.ascontiguousarray(meas[perm], dtype=np.float64)
    cams0 = init_cameras(n_cams, init_seed)
    return Problem(n_cams=n_cams, n_pts=n_pts, cam_idx=cam_idx, pt_idx=pt_idx, meas=meas,
                   cams0=cams0, eta=eta, order=order, iters=iters,
                   cams_gt=G.reshape(n_cams, 12), pts_gt=X, K_gt=K,
                   seeds=dict(data=seed, init=init_seed), name=name)


def init_cameras(n_cams: int, init_seed: int) -> np.ndarray:
    """Random initial cameras: unit-norm Gaussian 12-vectors (row-major 3x4)."""
    rng = np.random.default_rng(init_seed)
    c = rng.standard_normal((n_cams, 12))
    return c / np.linalg.norm(c, axis=1, keepdims=True)


# Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
# as 1, 2, 3", SC 2011): the published round multipliers and Weyl key bumps.
_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
_MASK64 = (1 << 64) - 1


def philox4x64(ctr, key, rounds: int = 10):
    """One Philox4x64 block: four 64-bit outputs for a 4-word counter and a
    2-word key (Python integers)."""
    c, k = list(ctr), list(key)
    for r in range(rounds):
        if r:
            k = [(k[0] + _PHILOX_W[0]) & _MASK64, (k[1] + _PHILOX_W[1]) & _MASK64]
        p0, p1 = _PHILOX_M[0] * c[0], _PHILOX_M[1] * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & _MASK64, (p0 >> 64) ^ c[3] ^ k[1], p0 & _MASK64]
    return c


def seeded_cameras(n_cams: int, seed: int) -> np.ndarray:
    """Initial cameras the library draws itself when it is given none
    (povar_options.init_seed): camera c takes the Philox4x64-10 blocks with key
    (seed, 0) and counters (c, b, 0, 0), b = 0, 1, 2; each output w gives the
    uniform ((w >> 11) + 0.5) 2^-53, each output pair (u0, u1) two normals by
    the Box-Muller transform (Box and Muller, 1958), and the 12 normals are
    scaled to unit norm."""
    out = np.empty((n_cams, 12))
    for cam in range(n_cams):
        for b in range(3):
            w = philox4x64([cam, b, 0, 0], [seed & _MASK64, 0])
            for h in range(2):
                u0 = ((w[2 * h] >> 11) + 0.5) * 2.0 ** -53
                u1 = ((w[2 * h + 1] >> 11) + 0.5) * 2.0 ** -53
                rho = math.sqrt(-2.0 * math.log(u0))
                out[cam, 4 * b + 2 * h] = rho * math.cos(2.0 * math.pi * u1)
                out[cam, 4 * b + 2 * h + 1] = rho * math.sin(2.0 * math.pi * u1)
    return out / np.linalg.norm(out, axis=1, keepdims=True)


def workload(number: int, k: int = 0, **overrides) -> Problem:
    """Problem number `k` of workload `number`; data seed = 1000*number + k,
    initial-camera seed = data seed + 1."""
    w = dict(WORKLOADS[number])
    w.update(overrides)
    name = w.pop("name")
    w.pop("precision", None)
    seed = 1000 * number + k
    return make_problem(w.pop("n_cams"), w.pop("n_pts"), seed=seed, init_seed=seed + 1,
                        name=name, **w)


def serving_stream(n_requests: int = 512, seed: int = 4000, cams_lo=20, cams_hi=400,
                   pts_per_cam=250):
    """Size list of the serving workload: cameras log-uniform in [20, 400],
    points = 250 x cameras, mean track length 5.  Returns (n_cams, n_pts, seed)
    triples; each request is then drawn with make_problem."""
    rng = np.random.default_rng(seed)
    nc = np.rint(np.exp(rng.uniform(math.log(cams_lo), math.log(cams_hi), size=n_requests)))
    nc = nc.astype(np.int64)
    return [(int(c), int(c) * pts_per_cam, seed + 1 + 2 * i) for i, c in enumerate(nc)]


def serving_problem(n_cams: int, n_pts: int, seed: int, order=20, iters=50, eta=0.01) -> Problem:
    return make_problem(n_cams, n_pts, track=("geom", 0.25), seed=seed, init_seed=seed + 1,
                        order=order, iters=iters, eta=eta, name=f"serve-{n_cams}cam")
