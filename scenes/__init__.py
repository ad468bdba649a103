"""Seeded synthetic scenes for scaled bundle adjustment (SBA).

This module only draws inputs: camera poses, landmarks, the view graph and the
lifted 3D keypoints u_ik with weights w_ik that enter the SBA cost (Section
"BA with learned depth", eq. sba).  It holds none of the solver's arithmetic:
no data matrix, no cost, no elimination.  Both the FP64 CPU oracle and the HIP
path read the same arrays from here.

Conventions
-----------
* The generator draws world->camera poses (R_cfg, c): a world point x is seen
  in camera i at R_cfg[i] @ (x - c[i]).  The lifted keypoint is
  u = d_i * (R_cfg[i] @ (x - c[i]) + eps), with a per-frame depth scale d_i and
  eps ~ N(0, sigma^2 I).
* SBA uses camera->world transforms (footnote to eq. sba):
  R_i (s_i u) + t_i = p_k.  Anchoring frame 0 (R=I, s=1, t=0; Section
  "Anchoring") gives the ground truth returned in ``gt``:
      R_i = R_cfg[0] @ R_cfg[i].T,   s_i = d_0 / d_i,
      t_i = d_0 R_cfg[0] (c_i - c_0), p_k = d_0 R_cfg[0] (x_k - c_0).
* Indices are 0-based int32; u is float64 [n, 3]; w is float64 [n].

Workload shapes (sizes, track-length mixes and noise follow the five
benchmark configurations; where those leave a choice open, the choice made
here is written next to the code):
  tiny       N=50,    M=2000,  4 random frames per landmark          (8000 obs)
  unordered  N=1000,  M=100k,  L~U{2..8} among 30 nearest cameras    (~500k)
  sequential N=2000,  M=400k,  L~U{3..12} within +-10 frames on a loop (~2.4M)
  large      N=10155, M=2M,    L=1+Geom(1/3) among 50 nearest, 20 clusters,
                               5% outliers                             (~8M)
  diff       N=500,   M=50k,   L~U{3..6} random frames, w~U[0.5,1.5]  (~225k)
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

__all__ = ["Scene", "haar_rotations", "make_scene", "random_scene", "CONFIGS"]


@dataclasses.dataclass
class Scene:
    N: int
    M: int
    frame: np.ndarray      # int32 [n]
    landmark: np.ndarray   # int32 [n]
    u: np.ndarray          # float64 [n, 3]
    w: np.ndarray          # float64 [n]
    gt: Dict[str, np.ndarray]
    name: str = ""

    @property
    def n_obs(self) -> int:
        return int(self.frame.shape[0])

    def shuffled(self, seed: int) -> "Scene":
        """Same scene with the observation order permuted (order must not matter)."""
        rng = np.random.Generator(np.random.PCG64(seed))
        p = rng.permutation(self.n_obs)
        return Scene(self.N, self.M, self.frame[p].copy(), self.landmark[p].copy(),
                     self.u[p].copy(), self.w[p].copy(), self.gt, self.name)


def haar_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-uniform rotations from normalised 4-D Gaussian quaternions (Shoemake)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    a, b, c, d = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = a * a + b * b - c * c - d * d
    R[:, 0, 1] = 2 * (b * c - a * d)
    R[:, 0, 2] = 2 * (b * d + a * c)
    R[:, 1, 0] = 2 * (b * c + a * d)
    R[:, 1, 1] = a * a - b * b + c * c - d * d
    R[:, 1, 2] = 2 * (c * d - a * b)
    R[:, 2, 0] = 2 * (b * d - a * c)
    R[:, 2, 1] = 2 * (c * d + a * b)
    R[:, 2, 2] = a * a - b * b - c * c + d * d
    return R


def _rot_axis(axis: int, ang: np.ndarray) -> np.ndarray:
    c, s = np.cos(ang), np.sin(ang)
    n = ang.shape[0]
    R = np.zeros((n, 3, 3))
    i, j = [(1, 2), (0, 2), (0, 1)][axis]
    R[:, axis, axis] = 1.0
    R[:, i, i] = c
    R[:, j, j] = c
    R[:, i, j] = -s
    R[:, j, i] = s
    return R


def _distinct_choice(rng: np.random.Generator, cand: np.ndarray, L: np.ndarray) -> np.ndarray:
    """For each row of ``cand`` [m, K], pick L[row] distinct entries (uniformly).

    Returns a flat array of the chosen entries, row-major, rows in order."""
    m, K = cand.shape
    keys = rng.random((m, K))
    order = np.argsort(keys, axis=1)
    picked = np.take_along_axis(cand, order, axis=1)
    mask = np.arange(K)[None, :] < L[:, None]
    return picked[mask]


def _lift(rng, R_cfg, c, d, x, fr, lm, sigma, outlier_frac=0.0, bbox=None, local=None, mask_out=None):
    """u = d_i (R_cfg[i] (x_k - c_i) + eps); a fraction of rows replaced by random points.

    Outlier points are uniform in ``bbox`` (lo, hi) when given, else uniform in
    the cube of half-side ``local`` centred at the true landmark.  ``mask_out``
    (a list) receives the boolean outlier mask."""
    n = fr.shape[0]
    pts = x[lm]
    bad = np.zeros(n, bool)
    if outlier_frac > 0.0:
        bad = rng.random(n) < outlier_frac
        pts = pts.copy()
        if bbox is not None:
            lo, hi = bbox
            pts[bad] = rng.uniform(lo, hi, size=(int(bad.sum()), 3))
        else:
            pts[bad] = pts[bad] + rng.uniform(-local, local, size=(int(bad.sum()), 3))
    cam = np.einsum("nij,nj->ni", R_cfg[fr], pts - c[fr])
    if sigma > 0:
        cam = cam + sigma * rng.standard_normal((n, 3))
    if mask_out is not None:
        mask_out.append(bad)
    return d[fr][:, None] * cam


def _ground_truth(R_cfg, c, d, x) -> Dict[str, np.ndarray]:
    R0 = R_cfg[0]
    R = np.einsum("ij,nkj->nik", R0, R_cfg)          # R0 @ R_i^T
    s = d[0] / d
    t = d[0] * (c - c[0]) @ R0.T
    p = d[0] * (x - c[0]) @ R0.T
    return {"R": R, "s": s, "t": t, "p": p, "R_cfg": R_cfg, "c": c, "d": d, "x": x}


def _finish(name, N, M, fr, lm, u, w, gt) -> Scene:
    order = np.lexsort((fr, lm))
    if "outlier" in gt:
        gt["outlier"] = gt["outlier"][order]
    return Scene(N, M, fr[order].astype(np.int32), lm[order].astype(np.int32),
                 np.ascontiguousarray(u[order], dtype=np.float64),
                 np.ascontiguousarray(w[order], dtype=np.float64), gt, name)


def _components(N: int, fr: np.ndarray, lm: np.ndarray) -> np.ndarray:
    """Connected components of frames linked through shared landmarks."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    order = np.argsort(lm, kind="stable")
    lms, frs = lm[order], fr[order]
    starts = np.flatnonzero(np.r_[True, lms[1:] != lms[:-1]])
    first = np.repeat(frs[starts], np.diff(np.r_[starts, lms.shape[0]]))
    A = coo_matrix((np.ones(frs.shape[0]), (first, frs)), shape=(N, N)).tocsr()
    _, labels = connected_components(A, directed=False)
    return labels


def _distinct_uniform(rng: np.random.Generator, N: int, L: np.ndarray) -> np.ndarray:
    """For each row pick L[row] distinct frames uniformly from range(N) (rejection)."""
    m = L.shape[0]
    K = int(L.max())
    out = rng.integers(0, N, size=(m, K))
    valid = np.arange(K)[None, :] < L[:, None]
    while True:
        srt = np.sort(np.where(valid, out, -1 - np.arange(K)[None, :]), axis=1)
        dup = np.any((srt[:, 1:] == srt[:, :-1]) & (srt[:, 1:] >= 0), axis=1)
        if not dup.any():
            break
        out[dup] = rng.integers(0, N, size=(int(dup.sum()), K))
    return out[valid]


# ---------------------------------------------------------------------------
def random_scene(N: int, M: int, L: int = 4, sigma: float = 0.01, seed: int = 0,
                 depth=(0.5, 2.0), weights=None, center_box: float = 5.0,
                 ball: float = 3.0, name: str = "random", outlier: float = 0.0,
                 outlier_local: float = 0.0) -> Scene:
    """Tiny-scene recipe: Haar rotations, centres U[-b,b]^3, landmarks uniform in a
    ball, each landmark seen by L distinct frames chosen uniformly.

    ``weights``: None for w=1, or (lo, hi) for w~U[lo,hi].  L may be >= N only
    if L == N (every frame sees every landmark).  ``outlier``: fraction of
    observations whose 3D point is replaced by one uniform in the box of the
    camera centres, or, with ``outlier_local`` > 0, in the cube of that
    half-side around the true landmark (their mask is ``gt["outlier"]``)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R_cfg = haar_rotations(rng, N)
    c = rng.uniform(-center_box, center_box, size=(N, 3))
    d = rng.uniform(depth[0], depth[1], size=N)
    dirs = rng.standard_normal((M, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    x = ball * rng.random(M)[:, None] ** (1.0 / 3.0) * dirs
    L = min(L, N)
    fr = _distinct_uniform(rng, N, np.full(M, L))
    lm = np.repeat(np.arange(M), L)
    bad = []
    u = _lift(rng, R_cfg, c, d, x, fr, lm, sigma, outlier_frac=outlier,
              bbox=None if outlier_local > 0 else (-center_box, center_box),
              local=outlier_local, mask_out=bad)
    w = np.ones(fr.shape[0]) if weights is None else rng.uniform(weights[0], weights[1], fr.shape[0])
    gt = _ground_truth(R_cfg, c, d, x)
    gt["outlier"] = bad[0]
    return _finish(name, N, M, fr, lm, u, w, gt)


def _tiny(seed, sigma=0.01):
    # 50 frames, 2000 landmarks in a radius-3 ball, each seen by 4 random frames.
    return random_scene(50, 2000, L=4, sigma=sigma, seed=seed, name="tiny")


def _unordered(seed, N=1000, M=100_000, k=30, sigma=0.02):
    from scipy.spatial import cKDTree
    rng = np.random.Generator(np.random.PCG64(seed))
    R_cfg = haar_rotations(rng, N)
    c = rng.uniform(-10.0, 10.0, size=(N, 3))          # choice: centres U[-10,10]^3
    d = rng.uniform(0.5, 2.0, size=N)
    x = rng.uniform(-10.0, 10.0, size=(M, 3))          # choice: landmarks U[-10,10]^3
    L = rng.integers(2, 9, size=M)                     # track length U{2..8}
    _, nn = cKDTree(c).query(x, k=k, workers=-1)
    fr = _distinct_choice(rng, nn.astype(np.int64), L)
    lm = np.repeat(np.arange(M), L)
    u = _lift(rng, R_cfg, c, d, x, fr, lm, sigma)
    return _finish("unordered", N, M, fr, lm, u, np.ones(fr.shape[0]), _ground_truth(R_cfg, c, d, x))


def _sequential(seed, N=2000, M=400_000, window=10, sigma=0.01):
    rng = np.random.Generator(np.random.PCG64(seed))
    phi = 2.0 * np.pi * np.arange(N) / N
    c = np.stack([10.0 * np.cos(phi), 10.0 * np.sin(phi), np.zeros(N)], 1)
    # camera z-axis points to the loop centre (looking inward), x-axis along the
    # tangent; small yaw/pitch jitter N(0, (2 deg)^2).
    z = -c / 10.0
    xax = np.stack([-np.sin(phi), np.cos(phi), np.zeros(N)], 1)
    yax = np.cross(z, xax)
    R_c2w = np.stack([xax, yax, z], 2)                 # columns = camera axes in world
    jit = np.deg2rad(2.0)
    J = _rot_axis(1, jit * rng.standard_normal(N)) @ _rot_axis(0, jit * rng.standard_normal(N))
    R_c2w = R_c2w @ J
    R_cfg = np.transpose(R_c2w, (0, 2, 1))
    d = rng.uniform(0.7, 1.4, size=N)
    i0 = rng.integers(0, N, size=M)
    # landmark: ray in a 60-degree cone around the optical axis, depth U[2,8]
    half = np.deg2rad(30.0)
    cz = rng.uniform(np.cos(half), 1.0, size=M)
    az = rng.uniform(0.0, 2 * np.pi, size=M)
    sz = np.sqrt(1.0 - cz * cz)
    ray = np.stack([sz * np.cos(az), sz * np.sin(az), cz], 1) * rng.uniform(2.0, 8.0, size=M)[:, None]
    x = c[i0] + np.einsum("nij,nj->ni", R_c2w[i0], ray)
    L = rng.integers(3, 13, size=M)                    # U{3..12}
    offs = np.arange(-window, window + 1)
    cand = (i0[:, None] + offs[None, :]) % N
    fr = _distinct_choice(rng, cand, L)
    lm = np.repeat(np.arange(M), L)
    u = _lift(rng, R_cfg, c, d, x, fr, lm, sigma)
    return _finish("sequential", N, M, fr, lm, u, np.ones(fr.shape[0]), _ground_truth(R_cfg, c, d, x))


def _large(seed, N=10155, M=2_000_000, k=50, clusters=20, sigma=0.02, outlier=0.05,
           chunk=250_000, box=15.0, outlier_model="local", local=3.0):
    from scipy.spatial import cKDTree
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = rng.uniform(-box, box, size=(clusters, 3))   # choice: cluster centres U[-15,15]^3
    lab = rng.integers(0, clusters, size=N)
    c = mu[lab] + 6.0 * rng.standard_normal((N, 3))    # choice: N(mu, 6^2 I)
    R_cfg = haar_rotations(rng, N)
    d = rng.uniform(0.5, 2.0, size=N)
    seedf = rng.integers(0, N, size=M)
    x = c[seedf] + 3.0 * rng.standard_normal((M, 3))   # choice: N(c_seed, 3^2 I)
    L = np.minimum(1 + rng.geometric(1.0 / 3.0, size=M), k)   # mean 4, min 2
    tree = cKDTree(c)
    frs = []
    for a in range(0, M, chunk):
        _, nn = tree.query(x[a:a + chunk], k=k, workers=-1)
        frs.append(_distinct_choice(rng, nn.astype(np.int64), L[a:a + chunk]))
    fr = np.concatenate(frs)
    lm = np.repeat(np.arange(M), L)
    # Connectivity (choice): while the view graph has several components, add
    # bridge landmarks seen by the two mutually nearest frames of each pair of
    # neighbouring components (2+2 frames, 200 landmarks per bridge).
    comp = _components(N, fr, lm)
    roots = np.unique(comp)
    extra_x, extra_fr, extra_lm = [], [], []
    nextlm = M
    if roots.size > 1:
        cent = np.stack([c[comp == r_].mean(0) for r_ in roots])
        # spanning chain over components by nearest-centroid order
        order = [0]
        left = set(range(1, roots.size))
        while left:
            last = order[-1]
            nxt = min(left, key=lambda j: np.linalg.norm(cent[j] - cent[last]))
            order.append(nxt)
            left.remove(nxt)
        for a_, b_ in zip(order[:-1], order[1:]):
            fa = np.flatnonzero(comp == roots[a_])
            fb = np.flatnonzero(comp == roots[b_])
            dd = np.linalg.norm(c[fa][:, None, :] - c[fb][None, :, :], axis=2)
            ia, ib = np.unravel_index(np.argmin(dd), dd.shape)
            a2 = fa[np.argsort(np.linalg.norm(c[fa] - c[fa[ia]], axis=1))[:2]]
            b2 = fb[np.argsort(np.linalg.norm(c[fb] - c[fb[ib]], axis=1))[:2]]
            mid = 0.5 * (c[fa[ia]] + c[fb[ib]])
            for _ in range(200):
                extra_x.append(mid + 3.0 * rng.standard_normal(3))
                extra_fr.extend([a2[0], a2[1], b2[0], b2[1]])
                extra_lm.extend([nextlm] * 4)
                nextlm += 1
    if extra_x:
        x = np.concatenate([x, np.array(extra_x)])
        fr = np.concatenate([fr, np.array(extra_fr, dtype=np.int64)])
        lm = np.concatenate([lm, np.array(extra_lm, dtype=np.int64)])
    Mtot = x.shape[0]
    lo, hi = c.min(0) - 3.0, c.max(0) + 3.0
    bad = []
    if outlier_model == "box":
        u = _lift(rng, R_cfg, c, d, x, fr, lm, sigma, outlier_frac=outlier, bbox=(lo, hi), mask_out=bad)
    else:
        u = _lift(rng, R_cfg, c, d, x, fr, lm, sigma, outlier_frac=outlier, local=local, mask_out=bad)
    gt = _ground_truth(R_cfg, c, d, x)
    gt["outlier"] = bad[0]
    return _finish("large", N, Mtot, fr, lm, u, np.ones(fr.shape[0]), gt)


def _diff(seed, N=500, M=50_000, sigma=0.01):
    rng = np.random.Generator(np.random.PCG64(seed))
    R_cfg = haar_rotations(rng, N)
    c = rng.uniform(-5.0, 5.0, size=(N, 3))
    d = rng.uniform(0.5, 2.0, size=N)
    dirs = rng.standard_normal((M, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    x = 3.0 * rng.random(M)[:, None] ** (1.0 / 3.0) * dirs
    L = rng.integers(3, 7, size=M)                     # U{3..6}
    fr = _distinct_uniform(rng, N, L)
    lm = np.repeat(np.arange(M), L)
    u = _lift(rng, R_cfg, c, d, x, fr, lm, sigma)
    w = rng.uniform(0.5, 1.5, size=fr.shape[0])
    return _finish("diff", N, M, fr, lm, u, w, _ground_truth(R_cfg, c, d, x))


CONFIGS = {
    "tiny": _tiny,
    "unordered": _unordered,
    "sequential": _sequential,
    "large": _large,
    "diff": _diff,
}


def make_scene(cfg: str, seed: int = 0, **kw) -> Scene:
    """Build one of the named workloads (see module docstring) from a seed."""
    return CONFIGS[cfg](seed, **kw)
