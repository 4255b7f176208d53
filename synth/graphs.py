"""Seeded general (non-grid) networks as vertex-pair lists, and region assignments.

Layout contract (shared with the C ABI of the general-graph solver):

* ``pu[i], pv[i]`` (int32, ``0 <= pu, pv < n``, ``pu != pv``) is the i-th vertex
  pair; ``cuv[i] = c(pu, pv)`` and ``cvu[i] = c(pv, pu)``, int32 >= 0.  Several
  pairs may join the same two vertices.
* ``cs[v] = c(s, v)`` and ``ct[v] = c(v, t)``, int32 >= 0.
* ``region[v]`` (int32 >= 0) is the region of v; any assignment is allowed
  (regions need not be contiguous in the vertex numbering).

Two families stand in for the paper's non-grid instances: 3D volumes with the
26-neighbourhood and capacities up to 100 (the "n26c100" segmentation
instances), and sparse random networks with mostly local and some long-range
pairs (the structure of stereo and multiview instances, whose graphs add
non-grid edges to a regular layout).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np


@dataclass
class GraphInstance:
    n: int
    pu: np.ndarray
    pv: np.ndarray
    cuv: np.ndarray
    cvu: np.ndarray
    cs: np.ndarray
    ct: np.ndarray
    region: np.ndarray = None   # int32 [n] or None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def npairs(self) -> int:
        return int(self.pu.shape[0])

    def arrays(self):
        return self.pu, self.pv, self.cuv, self.cvu, self.cs, self.ct


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def random_graph(n, deg, seed, cap_hi=20, tlink_hi=30, long_frac=0.1, window=64, zero_p=0.2,
                 tlink_p=0.35, shuffle=True, region=None, name=None):
    """A sparse network: about ``deg`` pairs per vertex, each joining v to a vertex
    within ``window`` positions of it or, with probability ``long_frac``, to a
    uniformly random vertex.  Capacities are independent uniform integers with a
    share ``zero_p`` of zeros per direction; s- and t-links are present at a share
    ``tlink_p`` of the vertices each.  ``shuffle`` permutes the vertex numbers, so
    that a region of consecutive numbers is no longer a neighbourhood."""
    rng = np.random.default_rng(seed)
    m = int(round(n * deg / 2))
    if n < 2:
        m = 0
    u = rng.integers(0, max(n, 1), size=m)
    off = rng.integers(1, window + 1, size=m) * rng.choice([-1, 1], size=m)
    v = np.clip(u + off, 0, max(n - 1, 0))
    far = rng.uniform(size=m) < long_frac
    v = np.where(far, rng.integers(0, max(n, 1), size=m), v)
    keep = u != v
    u, v = u[keep], v[keep]
    m = u.shape[0]
    cuv = rng.integers(0, cap_hi + 1, size=m) * (rng.uniform(size=m) >= zero_p)
    cvu = rng.integers(0, cap_hi + 1, size=m) * (rng.uniform(size=m) >= zero_p)
    cs = rng.integers(1, tlink_hi + 1, size=n) * (rng.uniform(size=n) < tlink_p)
    ct = rng.integers(1, tlink_hi + 1, size=n) * (rng.uniform(size=n) < tlink_p)
    if shuffle and n > 0:
        perm = rng.permutation(n)
        u, v = perm[u], perm[v]
        inv = np.empty(n, dtype=np.int64)
        inv[perm] = np.arange(n)
        cs, ct = cs[inv], ct[inv]
    return GraphInstance(n=int(n), pu=_i32(u), pv=_i32(v), cuv=_i32(cuv), cvu=_i32(cvu),
                         cs=_i32(cs), ct=_i32(ct), region=None if region is None else _i32(region),
                         name=name or f"rgraph_{n}_{deg}_{seed}")


OFFSETS_26 = tuple(o for o in itertools.product((-1, 0, 1), repeat=3) if o > (0, 0, 0))


def grid26_graph(dims, seed, nblobs=4, cap=100, tlink_hi=100, name=None):
    """3D volume with the 26-neighbourhood (13 pairs per interior vertex) and
    capacities up to ``cap``: a sum of Gaussian blobs, normalised and passed
    through a steep sigmoid (objects with sharp borders) plus Gaussian noise of
    0.08, gives each voxel an intensity in [0, 1]; a pair gets
    ``cap * exp(-(dI / 0.1)^2) / |offset|`` (contrast-sensitive, rounded), its
    reverse the same; the t-links put intensities above 0.5 on the source side,
    below it on the sink side, with a strength of up to ``tlink_hi``."""
    D, H, W = (int(d) for d in dims)
    n = D * H * W
    rng = np.random.default_rng(seed)
    img = np.zeros((D, H, W))
    z, y, x = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
    for _ in range(nblobs):
        c = rng.uniform(0, 1, size=3) * np.array([D, H, W])
        sig = rng.uniform(0.1, 0.3) * max(D, H, W)
        img += rng.uniform(0.5, 1.0) * np.exp(-((z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2)
                                              / (2 * sig * sig))
    # objects with sharp borders: a steep sigmoid of the blob sum, then noise
    img = img / max(img.max(), 1e-9)
    img = 1.0 / (1.0 + np.exp(-(img - 0.35) * 25.0))
    img = np.clip(img + rng.normal(scale=0.08, size=img.shape), 0, 1)
    idx = np.arange(n).reshape(D, H, W)
    pus, pvs, cs_ = [], [], []
    for dz, dy, dx in OFFSETS_26:
        zs = slice(max(0, -dz), D - max(0, dz))
        ys = slice(max(0, -dy), H - max(0, dy))
        xs = slice(max(0, -dx), W - max(0, dx))
        zt = slice(max(0, dz), D - max(0, -dz))
        yt = slice(max(0, dy), H - max(0, -dy))
        xt = slice(max(0, dx), W - max(0, -dx))
        a, b = idx[zs, ys, xs].reshape(-1), idx[zt, yt, xt].reshape(-1)
        di = img[zs, ys, xs].reshape(-1) - img[zt, yt, xt].reshape(-1)
        w = np.rint(cap * np.exp(-(di / 0.1) ** 2) / np.sqrt(dz * dz + dy * dy + dx * dx))
        pus.append(a)
        pvs.append(b)
        cs_.append(w)
    pu = np.concatenate(pus) if pus else np.zeros(0)
    pv = np.concatenate(pvs) if pvs else np.zeros(0)
    c = np.concatenate(cs_) if cs_ else np.zeros(0)
    f = img.reshape(-1)
    strength = np.rint(tlink_hi * np.abs(f - 0.5) * 2 * rng.uniform(0.5, 1.0, size=n))
    cs = np.where(f > 0.5, strength, 0)
    ct = np.where(f <= 0.5, strength, 0)
    return GraphInstance(n=n, pu=_i32(pu), pv=_i32(pv), cuv=_i32(c), cvu=_i32(c), cs=_i32(cs),
                         ct=_i32(ct), name=name or f"grid26_{D}x{H}x{W}_{seed}",
                         meta=dict(dims=(D, H, W)))


def block_regions(dims, tile):
    """Region of every vertex of a row-major 3D volume cut into boxes of ``tile``."""
    D, H, W = dims
    tz, ty, tx = tile
    z, y, x = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
    nz, ny, nx = -(-D // tz), -(-H // ty), -(-W // tx)
    r = ((z // tz) * ny + (y // ty)) * nx + (x // tx)
    return _i32(r.reshape(-1))


def index_regions(n, size):
    """Regions of ``size`` consecutive vertex numbers (the splitter's default)."""
    return _i32(np.arange(n) // max(int(size), 1))


def random_regions(n, K, seed):
    """Every vertex in a uniformly random one of K regions (scattered regions)."""
    return _i32(np.random.default_rng(seed).integers(0, K, size=n))
