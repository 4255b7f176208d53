"""Seeded grid instances with the shapes and value ranges of vision max-flow problems.

Layout contract (shared with the C ABI):

* ``dims`` is row-major, last axis fastest: 2D ``(H, W)``, 3D ``(D, H, W)``.
  Vertex ``v`` has linear index ``y*W + x`` (2D) or ``z*H*W + y*W + x`` (3D).
* ``nbr[k, v] = c(v, v + o_k)`` for the canonical offsets below; opposite
  directions are adjacent so the reverse of direction ``k`` is ``k ^ 1``.
  Arcs that leave the grid carry capacity 0.
* ``cs[v] = c(s, v)`` and ``ct[v] = c(v, t)``, all int32 and >= 0.

The generator recipe (blob image -> contrast-sensitive n-links, intensity
t-links) follows the stated configurations of the measured workloads; every
free choice they leave open is fixed here, in the functions below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Offsets as (dz, dy, dx) tuples trimmed to the grid rank.  Order: +x, -x, +y, -y, ...
OFFSETS_2D4 = ((0, 1), (0, -1), (1, 0), (-1, 0))
OFFSETS_2D8 = OFFSETS_2D4 + ((1, 1), (-1, -1), (-1, 1), (1, -1))
OFFSETS_3D6 = ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0))


def offsets_for(ndim: int, conn: int):
    if ndim == 2 and conn == 4:
        return OFFSETS_2D4
    if ndim == 2 and conn == 8:
        return OFFSETS_2D8
    if ndim == 3 and conn == 6:
        return OFFSETS_3D6
    raise ValueError(f"unsupported grid: ndim={ndim} connectivity={conn}")


@dataclass
class GridInstance:
    dims: tuple
    conn: int
    cs: np.ndarray            # int32 [n]
    ct: np.ndarray            # int32 [n]
    nbr: np.ndarray           # int32 [K, n]
    tile: tuple = None        # region shape (same rank as dims), or None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(np.prod(self.dims))

    @property
    def ndim(self) -> int:
        return len(self.dims)

    @property
    def K(self) -> int:
        return self.nbr.shape[0]


def _shift_valid(dims, off):
    """Boolean mask over the grid: True where v + off stays inside the grid."""
    masks = []
    for ax, (n, o) in enumerate(zip(dims, off)):
        idx = np.arange(n)
        m = (idx + o >= 0) & (idx + o < n)
        shape = [1] * len(dims)
        shape[ax] = n
        masks.append(m.reshape(shape))
    out = masks[0]
    for m in masks[1:]:
        out = out & m
    return np.broadcast_to(out, dims)


def _neighbor_view(a, off):
    """b[v] = a[v + off] where valid, 0 elsewhere (same shape as a)."""
    b = np.zeros_like(a)
    src = []
    dst = []
    for n, o in zip(a.shape, off):
        if o >= 0:
            src.append(slice(o, n))
            dst.append(slice(0, n - o))
        else:
            src.append(slice(0, n + o))
            dst.append(slice(-o, n))
    b[tuple(dst)] = a[tuple(src)]
    return b


def _add_blob(img, centre, sigma):
    """img += exp(-|x-c|^2 / (2 sigma^2)), truncated to a box of half-width ceil(4 sigma)."""
    r = int(math.ceil(4.0 * sigma))
    sl = []
    factors = []
    for ax, (n, c) in enumerate(zip(img.shape, centre)):
        lo = max(0, int(math.floor(c)) - r)
        hi = min(n, int(math.floor(c)) + r + 1)
        coords = np.arange(lo, hi, dtype=np.float64)
        f = np.exp(-((coords - c) ** 2) / (2.0 * sigma * sigma))
        shape = [1] * img.ndim
        shape[ax] = hi - lo
        factors.append(f.reshape(shape))
        sl.append(slice(lo, hi))
    blob = factors[0]
    for f in factors[1:]:
        blob = blob * f
    img[tuple(sl)] += blob


def blob_grid(dims, conn, seed, nblobs, sigma_lo, sigma_hi, zero_frac=0.0,
              tile=None, name="", nblobs_from_rng=None, float_dtype=np.float64):
    """Blob image -> int32 caps.

    Draw order from ``numpy.random.default_rng(seed)``: (optional blob count),
    centres, sigmas, noise, zero mask.  Intensity
    ``I = clip(0.2 + sum_b blob_b + N(0, 0.05^2), 0, 1)``; n-link
    ``rint(50 exp(-(I_p - I_q)^2 / (2 * 0.1^2)))`` (divided by sqrt(2) before
    rounding on diagonal arcs); ``cs = rint(20 I)``, ``ct = rint(20 (1 - I))``.
    ``zero_frac`` zeroes each undirected n-link independently (both directions).
    """
    dims = tuple(int(d) for d in dims)
    ndim = len(dims)
    offs = offsets_for(ndim, conn)
    rng = np.random.default_rng(seed)
    if nblobs_from_rng is not None:
        lo, hi = nblobs_from_rng
        nblobs = int(rng.integers(lo, hi + 1))
    centres = rng.uniform(0.0, 1.0, size=(nblobs, ndim)) * np.array(dims, dtype=np.float64)
    sigmas = rng.uniform(sigma_lo, sigma_hi, size=nblobs)
    img = np.full(dims, 0.2, dtype=np.float64)
    for b in range(nblobs):
        _add_blob(img, centres[b], float(sigmas[b]))
    img += rng.normal(0.0, 0.05, size=dims)
    np.clip(img, 0.0, 1.0, out=img)
    img = img.astype(float_dtype, copy=False)

    n = int(np.prod(dims))
    K = len(offs)
    nbr = np.zeros((K, n), dtype=np.int32)
    for k in range(0, K, 2):
        off = offs[k]
        diag = sum(1 for o in off if o != 0) > 1
        q = _neighbor_view(img, off)
        diff = img - q
        w = 50.0 * np.exp(-(diff * diff) / (2.0 * 0.1 * 0.1))
        if diag:
            w = w / math.sqrt(2.0)
        cap = np.rint(w).astype(np.int32)
        valid = _shift_valid(dims, off)
        cap = np.where(valid, cap, 0).astype(np.int32)
        if zero_frac > 0.0:
            keep = rng.uniform(0.0, 1.0, size=dims) >= zero_frac
            cap = np.where(keep, cap, 0).astype(np.int32)
        nbr[k] = cap.reshape(-1)
        # reverse arc (v + o_k, k^1) carries the same capacity
        neg = tuple(-o for o in off)
        rev = _neighbor_view(cap, neg)
        nbr[k + 1] = rev.reshape(-1)
    cs = np.rint(20.0 * img).astype(np.int32).reshape(-1)
    ct = np.rint(20.0 * (1.0 - img)).astype(np.int32).reshape(-1)
    return GridInstance(dims=dims, conn=conn, cs=cs, ct=ct, nbr=nbr, tile=tile, name=name,
                        meta=dict(seed=seed, nblobs=nblobs))


# --------------------------------------------------------------------------
# The five measured workloads.
# --------------------------------------------------------------------------

def config(i: int) -> GridInstance:
    """Workload i in {0, 1, 2, 4}; workload 3 is a batch, see config3_instances."""
    if i == 0:
        return blob_grid((64, 64), 4, 0, 2, 8.0, 8.0, tile=(32, 32), name="grid2d4_64")
    if i == 1:
        return blob_grid((2048, 2048), 8, 1, 64, 10.0, 80.0, zero_frac=0.1,
                         tile=(64, 64), name="grid2d8_2048")
    if i == 2:
        return blob_grid((256, 256, 256), 6, 2, 32, 8.0, 32.0, tile=(32, 32, 32),
                         name="grid3d6_256")
    if i == 4:
        return blob_grid((464, 464, 464), 6, 4, 256, 8.0, 32.0, tile=(64, 64, 64),
                         name="grid3d6_464", float_dtype=np.float32)
    raise ValueError(f"no single-instance workload {i}")


def config3_sizes(count: int = 512, meta_seed: int = 3):
    meta = np.random.default_rng(meta_seed)
    logs = meta.uniform(math.log(32.0), math.log(512.0), size=(count, 2))
    return np.rint(np.exp(logs)).astype(np.int64)


def config3_instances(count: int = 512, first: int = 0):
    """Batch workload: instance i has side lengths from the meta stream, seed 3000+i,
    blob count uniform in {2..16}, sigma 8, 4-connected for even i, 8-connected for odd i."""
    sizes = config3_sizes(512)
    out = []
    for i in range(first, first + count):
        h, w = int(sizes[i, 0]), int(sizes[i, 1])
        conn = 4 if i % 2 == 0 else 8
        out.append(blob_grid((h, w), conn, 3000 + i, 0, 8.0, 8.0, nblobs_from_rng=(2, 16),
                             name=f"batch_{i}"))
    return out


# --------------------------------------------------------------------------
# Fuzz families for tests.
# --------------------------------------------------------------------------

def random_grid(dims, conn, seed, cap_hi=10, tlink_hi=20, zero_p=0.3, asym=True, tile=None):
    """Small grid with independent random caps: many zeros, asymmetric pairs."""
    dims = tuple(int(d) for d in dims)
    ndim = len(dims)
    offs = offsets_for(ndim, conn)
    rng = np.random.default_rng(seed)
    n = int(np.prod(dims))
    K = len(offs)
    nbr = np.zeros((K, n), dtype=np.int32)
    for k in range(K):
        c = rng.integers(0, cap_hi + 1, size=dims)
        z = rng.uniform(size=dims) < zero_p
        c = np.where(z, 0, c)
        valid = _shift_valid(dims, offs[k])
        nbr[k] = np.where(valid, c, 0).astype(np.int32).reshape(-1)
    if not asym:
        for k in range(0, K, 2):
            rev = _neighbor_view(nbr[k].reshape(dims), tuple(-o for o in offs[k]))
            nbr[k + 1] = rev.reshape(-1)
    cs = rng.integers(0, tlink_hi + 1, size=n)
    ct = rng.integers(0, tlink_hi + 1, size=n)
    zs = rng.uniform(size=n) < 0.3
    zt = rng.uniform(size=n) < 0.3
    cs = np.where(zs, 0, cs).astype(np.int32)
    ct = np.where(zt, 0, ct).astype(np.int32)
    return GridInstance(dims=dims, conn=conn, cs=cs, ct=ct, nbr=nbr, tile=tile,
                        name=f"rand_{dims}_{conn}_{seed}")


def paper_e1_grid(dims, conn, seed, strength, tile=None):
    """The paper's synthetic family (Sec. 7.1) on our canonical offsets: integer
    excess/deficit uniform in [-500, 500] (positive -> source link, negative ->
    sink link) and a constant capacity 'strength' on every n-link."""
    dims = tuple(int(d) for d in dims)
    offs = offsets_for(len(dims), conn)
    rng = np.random.default_rng(seed)
    n = int(np.prod(dims))
    e = rng.integers(-500, 501, size=n)
    cs = np.where(e > 0, e, 0).astype(np.int32)
    ct = np.where(e < 0, -e, 0).astype(np.int32)
    nbr = np.zeros((len(offs), n), dtype=np.int32)
    for k, off in enumerate(offs):
        nbr[k] = np.where(_shift_valid(dims, off), strength, 0).astype(np.int32).reshape(-1)
    return GridInstance(dims=dims, conn=conn, cs=cs, ct=ct, nbr=nbr, tile=tile,
                        name=f"e1_{dims}_{conn}_{strength}_{seed}")


def random_digraph(n, seed, p_edge=0.35, cap_hi=10):
    """Random small network for brute-force checks: vertex pairs with independent
    capacities in each direction (many zeros), plus random s- and t-links.
    Returns (pu, pv, cuv, cvu, cs, ct) as int32 arrays."""
    rng = np.random.default_rng(seed)
    pu, pv, cuv, cvu = [], [], [], []
    for u in range(n):
        for v in range(u + 1, n):
            if rng.uniform() < p_edge:
                a = int(rng.integers(0, cap_hi + 1)) if rng.uniform() < 0.8 else 0
                b = int(rng.integers(0, cap_hi + 1)) if rng.uniform() < 0.5 else 0
                pu.append(u); pv.append(v); cuv.append(a); cvu.append(b)
    cs = rng.integers(0, cap_hi + 1, size=n) * (rng.uniform(size=n) < 0.5)
    ct = rng.integers(0, cap_hi + 1, size=n) * (rng.uniform(size=n) < 0.5)
    as32 = lambda x: np.asarray(x, dtype=np.int32)
    return as32(pu), as32(pv), as32(cuv), as32(cvu), as32(cs), as32(ct)
