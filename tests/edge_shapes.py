"""Seeded problems whose observations sit on the edges of the device layout
(shared by the CPU layout test and the GPU parity test)."""
import numpy as np

from paper_2405_05079_amd import synth


def boundary_problem(seed=41):
    """Observations placed on the layout's edges: camera 0 with exactly one
    full 2048-observation chunk, camera 1 with 2049 (a second chunk of one),
    camera 2 with exactly two full chunks; landmarks with exactly 64
    observations (one full packet slot), 65 (the first length that takes the
    long-landmark slots) and 63.  Projective ground truth, pixel noise 1e-3,
    random unit-norm initial cameras."""
    rng = np.random.default_rng(seed)
    n_cams, n_pts = 80, 5000
    tracks = []
    for j in range(n_pts):
        cams = [c for c, lim in ((0, 2048), (1, 2049), (2, 4096)) if j < lim]
        if j >= n_pts - 3:
            want = (64, 65, 63)[j - (n_pts - 3)]
        else:
            want = max(len(cams), int(rng.integers(2, 5)))
        extra = rng.choice(np.arange(3, n_cams), size=want - len(cams), replace=False)
        tracks.append(cams + [int(c) for c in extra])
    cam = np.array([c for t in tracks for c in t], dtype=np.int32)
    pt = np.array([j for j, t in enumerate(tracks) for _ in t], dtype=np.int32)
    G = rng.standard_normal((n_cams, 3, 4))
    G[:, 2, :3] *= 0.1
    G[:, 2, 3] = 5.0
    Xw = rng.uniform(-1.0, 1.0, size=(n_pts, 3))
    y = np.einsum("nab,nb->na", G[cam], np.c_[Xw[pt], np.ones(len(pt))])
    meas = y[:, :2] / y[:, 2:3] + 1e-3 * rng.standard_normal((len(pt), 2))
    perm = rng.permutation(len(pt))
    cams0 = rng.standard_normal((n_cams, 12))
    cams0 /= np.linalg.norm(cams0, axis=1, keepdims=True)
    return synth.Problem(n_cams, n_pts, cam[perm], pt[perm], meas[perm], cams0, order=8)

