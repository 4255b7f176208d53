"""CPU oracle for exact s-t max-flow / min-cut (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU solver:
the C part (``oracle.c`` -> ``liboracle.so``) is built from its own source with
gcc, and the helpers below are plain numpy.

What it computes (all integer, int64 accumulators):

* ``solve_pairs`` / ``solve_grid`` -- the maximum flow value and the two extremal
  minimum cuts of the network of the paper's Sec. 2 (excess form), by a textbook
  highest-label push-relabel (``method="pr"``) or by Dinic on the explicit s-t
  network (``method="dinic"``).
* ``ard_grid`` -- the paper's own method run step by step on the CPU: Init,
  Alg. 2 (P-ARD) or Alg. 1 (S-ARD), Proc. ARD with Augment (Sec. 4.2), region
  relabel (Alg. 3) and the global gap (Sec. 5.1), with the per-sweep checks of
  the statements of Sec. 4 switched on by ``checks``; optionally with the
  partial discharges (Sec. 6.2) and the boundary relabel heuristic (Sec. 6.1).
* ``prd_grid`` -- the push-relabel region discharge of Sec. 3 (Proc. PRD,
  first-in first-out Push/Relabel on each region network) under Alg. 2
  (P-PRD) or Alg. 1 (S-PRD), with the global gap over all labels and per-sweep
  checks of label validity and monotonicity.
* ``region_reduction`` -- Alg. 5 (Sec. 8) on every region of a grid instance:
  strong and weak source and sink nodes from three augmentations per region;
  ``region_reduction_union`` the same classes for large grids from the two
  auxiliary problems of the section, all regions in one network.
* ``boundary_relabel`` -- the heuristic of Sec. 6.1 on a given state, written
  separately in Python (groups, the two kinds of arcs, Dijkstra by heapq).
* ``region_relabel`` -- the region relabel of Alg. 3 of every region on a given
  state (the labels a region discharge writes).
* ``brute_force`` -- every cut of a network of at most ~20 vertices.
* ``certify`` -- feasibility, conservation and max-flow = min-cut duality of a
  residual state, from the original capacities.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

CHK_VALID = 1
CHK_MONO = 2
CHK_ACTIVE_B = 4
CHK_LOWER = 8
CHK_DISCHARGE = 16
CHK_ALL = 31

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC",
                               "-o", _LIB_PATH, _SRC])
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        common = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, P, P, P, P, P, P, P, P, P]
        lib.orc_pushrelabel.argtypes = common
        lib.orc_pushrelabel.restype = ctypes.c_int
        lib.orc_dinic.argtypes = common
        lib.orc_dinic.restype = ctypes.c_int
        lib.orc_cuts.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, P, P, P, P]
        lib.orc_cuts.restype = ctypes.c_int
        lib.orc_ard.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, P, P, P,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                P, P, P, P, P, P, P, P, P, P, P]
        lib.orc_ard.restype = ctypes.c_int
        lib.orc_boundary_relabel.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, P,
                                             ctypes.c_int32, P]
        lib.orc_boundary_relabel.restype = ctypes.c_int
        lib.orc_prd.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, P, P, P,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                P, P, P, P, P, P, P, P, P, P]
        lib.orc_prd.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------------------
# Grid -> vertex pairs
# ---------------------------------------------------------------------------

def grid_pairs(dims, nbr, offsets):
    """Every geometric neighbour pair {v, v+o_k} of the grid (zero arcs included),
    one per undirected arc, with c(v, v+o_k) and c(v+o_k, v)."""
    dims = tuple(dims)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64).reshape(dims)
    pu, pv, cuv, cvu = [], [], [], []
    for k in range(0, len(offsets), 2):
        off = offsets[k]
        src, dst = [], []
        for size, o in zip(dims, off):
            if o >= 0:
                src.append(slice(0, size - o))
                dst.append(slice(o, size))
            else:
                src.append(slice(-o, size))
                dst.append(slice(0, size + o))
        u = idx[tuple(src)].reshape(-1)
        v = idx[tuple(dst)].reshape(-1)
        pu.append(u)
        pv.append(v)
        cuv.append(nbr[k][u])
        cvu.append(nbr[k + 1][v])
    cat = lambda xs: np.concatenate(xs) if xs else np.zeros(0, dtype=np.int64)
    return (cat(pu).astype(np.int32), cat(pv).astype(np.int32),
            _c32(cat(cuv)), _c32(cat(cvu)))


def grid_regions(dims, tile):
    """Region id of every vertex for a tiling of the grid into boxes of shape tile
    (the last box along an axis may be partial)."""
    dims = tuple(dims)
    grids = np.meshgrid(*[np.arange(d) // t for d, t in zip(dims, tile)], indexing="ij")
    nt = [-(-d // t) for d, t in zip(dims, tile)]
    rid = np.zeros(dims, dtype=np.int64)
    for ax, g in enumerate(grids):
        rid = rid * nt[ax] + g
    return rid.reshape(-1).astype(np.int32)


def _offsets(inst):
    from synth import offsets_for
    return offsets_for(len(inst.dims), inst.conn)


# ---------------------------------------------------------------------------
# Solvers
# ---------------------------------------------------------------------------

def solve_pairs(n, pu, pv, cuv, cvu, cs, ct, method="pr"):
    lib = _load()
    pu, pv, cuv, cvu, cs, ct = map(_c32, (pu, pv, cuv, cvu, cs, ct))
    m = pu.shape[0]
    r_uv = np.zeros(m, dtype=np.int64)
    r_vu = np.zeros(m, dtype=np.int64)
    rt = np.zeros(n, dtype=np.int64)
    ex = np.zeros(n, dtype=np.int64)
    flow = np.zeros(1, dtype=np.int64)
    smin = np.zeros(n, dtype=np.uint8)
    smax = np.zeros(n, dtype=np.uint8)
    fn = {"pr": lib.orc_pushrelabel, "dinic": lib.orc_dinic}[method]
    rc = fn(n, m, _p(pu), _p(pv), _p(cuv), _p(cvu), _p(cs), _p(ct), _p(r_uv), _p(r_vu),
            _p(rt), _p(ex), _p(flow), _p(smin), _p(smax))
    if rc != 0:
        raise RuntimeError(f"oracle {method} failed with code {rc}")
    return dict(flow=int(flow[0]), smin=smin, smax=smax, r_uv=r_uv, r_vu=r_vu, rt=rt, ex=ex)


def solve_grid(inst, method="pr"):
    pu, pv, cuv, cvu = grid_pairs(inst.dims, inst.nbr, _offsets(inst))
    out = solve_pairs(inst.n, pu, pv, cuv, cvu, inst.cs, inst.ct, method=method)
    out["pairs"] = (pu, pv, cuv, cvu)
    return out


def cuts_of_state(n, pu, pv, r_uv, r_vu, rt, ex):
    lib = _load()
    pu, pv = _c32(pu), _c32(pv)
    r_uv, r_vu, rt, ex = (np.ascontiguousarray(x, dtype=np.int64) for x in (r_uv, r_vu, rt, ex))
    smin = np.zeros(n, dtype=np.uint8)
    smax = np.zeros(n, dtype=np.uint8)
    rc = lib.orc_cuts(n, pu.shape[0], _p(pu), _p(pv), _p(r_uv), _p(r_vu), _p(rt), _p(ex),
                      _p(smin), _p(smax))
    if rc != 0:
        raise RuntimeError(f"orc_cuts failed with code {rc}")
    return smin, smax


def ard_pairs(n, pu, pv, cuv, cvu, cs, ct, region, parallel=True, checks=CHK_ALL,
              max_sweeps=None, partial=False, stop_early=False, boundary_relabel=False):
    """Reference ARD.  With partial=True sweep s runs only the stages k <= s
    (partial discharges, Sec. 6.2): excess may then stay inside a region, so the
    checks that only boundary vertices are active after the first sweep and that
    a discharge leaves no active vertex do not apply and are dropped.  With
    boundary_relabel=True the heuristic of Sec. 6.1 runs after the flow fusion of
    every sweep, before the gap.  With stop_early, reaching max_sweeps returns the
    state after that many sweeps (complete=False) instead of raising."""
    lib = _load()
    if partial:
        checks &= ~(CHK_ACTIVE_B | CHK_DISCHARGE)
    pu, pv, cuv, cvu, cs, ct, region = map(_c32, (pu, pv, cuv, cvu, cs, ct, region))
    m = pu.shape[0]
    r_uv = np.zeros(m, dtype=np.int64)
    r_vu = np.zeros(m, dtype=np.int64)
    rt = np.zeros(n, dtype=np.int64)
    ex = np.zeros(n, dtype=np.int64)
    flow = np.zeros(1, dtype=np.int64)
    smin = np.zeros(n, dtype=np.uint8)
    smax = np.zeros(n, dtype=np.uint8)
    labels = np.zeros(n, dtype=np.int32)
    sweeps = np.zeros(1, dtype=np.int64)
    bsize = np.zeros(1, dtype=np.int64)
    failed = np.zeros(1, dtype=np.int32)
    if max_sweeps is None:
        max_sweeps = (1 << 62)
    rc = lib.orc_ard(n, m, _p(pu), _p(pv), _p(cuv), _p(cvu), _p(cs), _p(ct), _p(region),
                     1 if parallel else 0, (1 if partial else 0) | (2 if boundary_relabel else 0),
                     int(max_sweeps), int(checks),
                     _p(r_uv), _p(r_vu),
                     _p(rt), _p(ex), _p(flow), _p(smin), _p(smax), _p(labels), _p(sweeps),
                     _p(bsize), _p(failed))
    if rc == 3:
        raise AssertionError(f"reference ARD invariant check {int(failed[0])} failed")
    if rc == 4 and stop_early:
        # max_sweeps sweeps ran and active vertices remain: the state at that point, no cuts
        return dict(flow=int(flow[0]), r_uv=r_uv, r_vu=r_vu, rt=rt, ex=ex, labels=labels,
                    sweeps=int(sweeps[0]), bsize=int(bsize[0]), complete=False)
    if rc != 0:
        raise RuntimeError(f"orc_ard failed with code {rc}")
    return dict(flow=int(flow[0]), smin=smin, smax=smax, r_uv=r_uv, r_vu=r_vu, rt=rt, ex=ex,
                labels=labels, sweeps=int(sweeps[0]), bsize=int(bsize[0]), complete=True)


def prd_grid(inst, tile=None, parallel=True, gap=True, checks=CHK_VALID | CHK_MONO,
             max_sweeps=None):
    """Reference P-PRD (parallel=True) or S-PRD: distance labels of Sec. 2
    (d(t) = 0, every arc of length 1, dinf = n), Proc. PRD per region, the
    flow fusion of Alg. 2, the global gap over all labels."""
    lib = _load()
    tile = tuple(tile if tile is not None else inst.tile)
    pu, pv, cuv, cvu = grid_pairs(inst.dims, inst.nbr, _offsets(inst))
    region = grid_regions(inst.dims, tile)
    n = inst.n
    pu, pv, cuv, cvu, cs, ct, region = map(_c32, (pu, pv, cuv, cvu, inst.cs, inst.ct, region))
    m = pu.shape[0]
    r_uv = np.zeros(m, dtype=np.int64)
    r_vu = np.zeros(m, dtype=np.int64)
    rt = np.zeros(n, dtype=np.int64)
    ex = np.zeros(n, dtype=np.int64)
    flow = np.zeros(1, dtype=np.int64)
    smin = np.zeros(n, dtype=np.uint8)
    smax = np.zeros(n, dtype=np.uint8)
    labels = np.zeros(n, dtype=np.int32)
    sweeps = np.zeros(1, dtype=np.int64)
    failed = np.zeros(1, dtype=np.int32)
    if max_sweeps is None:
        max_sweeps = 2 * n * n + 1
    rc = lib.orc_prd(n, m, _p(pu), _p(pv), _p(cuv), _p(cvu), _p(cs), _p(ct), _p(region),
                     1 if parallel else 0, 1 if gap else 0, int(max_sweeps), int(checks),
                     _p(r_uv), _p(r_vu), _p(rt), _p(ex), _p(flow), _p(smin), _p(smax),
                     _p(labels), _p(sweeps), _p(failed))
    if rc == 3:
        raise AssertionError(f"reference PRD invariant check {int(failed[0])} failed")
    if rc != 0:
        raise RuntimeError(f"orc_prd failed with code {rc}")
    return dict(flow=int(flow[0]), smin=smin, smax=smax, r_uv=r_uv, r_vu=r_vu, rt=rt, ex=ex,
                labels=labels, sweeps=int(sweeps[0]), pairs=(pu, pv, cuv, cvu))


def ard_grid(inst, tile=None, parallel=True, checks=CHK_ALL, max_sweeps=None, partial=False,
             stop_early=False, boundary_relabel=False):
    tile = tuple(tile if tile is not None else inst.tile)
    pu, pv, cuv, cvu = grid_pairs(inst.dims, inst.nbr, _offsets(inst))
    region = grid_regions(inst.dims, tile)
    out = ard_pairs(inst.n, pu, pv, cuv, cvu, inst.cs, inst.ct, region, parallel=parallel,
                    checks=checks, max_sweeps=max_sweeps, partial=partial, stop_early=stop_early,
                    boundary_relabel=boundary_relabel)
    out["pairs"] = (pu, pv, cuv, cvu)
    return out


def boundary_relabel_c(n, pu, pv, r_uv, r_vu, region, labels, dinf):
    """The C oracle's boundary relabel (the one orc_ard runs) on a given state."""
    lib = _load()
    pu, pv, r_uv, r_vu, region = map(_c32, (pu, pv, r_uv, r_vu, region))
    out = np.array(labels, dtype=np.int32, copy=True)
    rc = lib.orc_boundary_relabel(int(n), int(pu.shape[0]), _p(pu), _p(pv), _p(r_uv), _p(r_vu),
                                  _p(region), int(dinf), _p(out))
    if rc != 0:
        raise RuntimeError(f"orc_boundary_relabel failed with code {rc}")
    return out


def boundary_relabel(n, pu, pv, r_uv, r_vu, region, labels, dinf, distances=False):
    """Boundary relabel heuristic of Sec. 6.1 on a residual state (pairs form).

    Vertices with a label below dinf are grouped by (region, label); each group
    gets an arc of length 0 to the group of the next larger label of its region
    and the group of u an arc of length 1 to that of w for every residual arc
    (u, w) between regions (r_uv for pu -> pv, r_vu for pv -> pu).  d' is the
    distance from a vertex's group to the nearest group of label 0 (Dijkstra
    over the reversed arcs from all label-0 groups, heapq); the result is
    max(labels, d'), dinf where no label-0 group is reachable.  Interior
    vertices are grouped with the rest (they have no arcs of length 1), so the
    result is a valid labeling of all vertices.  Returns int32 labels, and with
    distances=True also d' itself (int64, -1 where no label-0 group is reached
    or the vertex takes no part)."""
    import heapq
    labels = np.asarray(labels, dtype=np.int64)
    region = np.asarray(region, dtype=np.int64)
    part = np.flatnonzero(labels < dinf)
    groups = {}
    for v in part:
        groups.setdefault((int(region[v]), int(labels[v])), len(groups))
    rev = [[] for _ in range(len(groups))]  # reversed arcs: head group -> (tail group, length)
    by_region = {}
    for (rg, lab), q in groups.items():
        by_region.setdefault(rg, []).append((lab, q))
    for rg, lst in by_region.items():
        lst.sort()
        for (la, qa), (lb, qb) in zip(lst, lst[1:]):
            rev[qb].append((qa, 0))  # arc qa -> qb of length 0
    pu = np.asarray(pu, np.int64)
    pv = np.asarray(pv, np.int64)
    for a, b, r_ab, r_ba in zip(pu, pv, np.asarray(r_uv), np.asarray(r_vu)):
        if region[a] == region[b] or labels[a] >= dinf or labels[b] >= dinf:
            continue
        ga = groups[(int(region[a]), int(labels[a]))]
        gb = groups[(int(region[b]), int(labels[b]))]
        if r_ab > 0:
            rev[gb].append((ga, 1))
        if r_ba > 0:
            rev[ga].append((gb, 1))
    dist = [None] * len(groups)
    heap = [(0, q) for (rg, lab), q in groups.items() if lab == 0]
    heapq.heapify(heap)
    while heap:
        d, q = heapq.heappop(heap)
        if dist[q] is not None:
            continue
        dist[q] = d
        for p, ln in rev[q]:
            if dist[p] is None:
                heapq.heappush(heap, (d + ln, p))
    out = labels.copy()
    dprime = np.full(len(labels), -1, np.int64)
    for v in part:
        dq = dist[groups[(int(region[v]), int(labels[v]))]]
        dp = dinf if dq is None else min(dq, dinf)
        out[v] = max(out[v], dp)
        if dq is not None:
            dprime[v] = dq
    if distances:
        return out.astype(np.int32), dprime
    return out.astype(np.int32)


def region_relabel(n, pu, pv, r_uv, r_vu, rt, region, labels, dinf):
    """Region relabel of Alg. 3 (the ARD variant, Sec. 4.2) of every region on
    a given residual state, with the given labels as the labels d(w) of the
    boundary vertices.  For u in region R: d'(u) = 0 if u reaches, inside R, a
    vertex with a residual t-link; else 1 + min d(w) over the vertices w outside
    R with d(w) < dinf that u reaches through a residual arc (x, w) with x
    reached inside R; else dinf (capped at dinf).  Computed as Alg. 3 steps: a
    backward flood from t inside the regions, then from the boundary seeds x at
    stage d(w) + 1 in increasing stage order, never relabelling a vertex."""
    from collections import deque
    pu = np.asarray(pu, np.int64)
    pv = np.asarray(pv, np.int64)
    r_uv = np.asarray(r_uv)
    r_vu = np.asarray(r_vu)
    region = np.asarray(region)
    labels = np.asarray(labels, np.int64)
    same = region[pu] == region[pv]
    rev = [[] for _ in range(n)]  # y -> x for residual arcs x -> y inside a region
    for a, b in zip(pu[same & (r_uv > 0)], pv[same & (r_uv > 0)]):
        rev[b].append(a)
    for a, b in zip(pv[same & (r_vu > 0)], pu[same & (r_vu > 0)]):
        rev[b].append(a)
    stage = {}
    def seed(x, k):
        stage.setdefault(int(k), []).append(int(x))
    for x in np.flatnonzero(np.asarray(rt) > 0):
        seed(x, 0)
    # boundary seeds: residual arcs leaving a region, to w with d(w) < dinf
    for tail, head, res in ((pu, pv, r_uv), (pv, pu, r_vu)):
        m = ~same & (res > 0)
        for x, w in zip(tail[m], head[m]):
            if labels[w] < dinf:
                seed(x, labels[w] + 1)
    out = np.full(n, dinf, np.int64)
    done = np.zeros(n, bool)
    for k in sorted(stage):
        q = deque()
        for x in stage[k]:
            if not done[x]:
                done[x] = True
                out[x] = min(k, dinf)
                q.append(x)
        while q:
            y = q.popleft()
            for x in rev[y]:
                if not done[x]:
                    done[x] = True
                    out[x] = min(k, dinf)
                    q.append(x)
    return out.astype(np.int32)


REDUCE_STRONG_SOURCE, REDUCE_STRONG_SINK, REDUCE_WEAK_SOURCE, REDUCE_WEAK_SINK = 1, 2, 4, 8


def region_reduction(inst, tile, big=1 << 28, augment="dinic"):
    """Region reduction (Alg. 5, Sec. 8) of every region of a grid instance, as a
    preprocessing of the initial network.  Returns one byte per vertex with the
    bits REDUCE_* of its class.

    The network G^R of region R holds R, its boundary B^R (the vertices outside R
    with a pair to R, without their s- and t-links) and the pairs that touch R,
    in both directions.  Every Augment is a maximum *flow* found by augmenting
    paths (Dinic), so the network after each step is the residual network of a
    true flow (no excess is parked at inner vertices); the s-links are carried
    as their residuals, the unsent supply of each vertex:
      1. Augment(s, t): the s-links of R to the t-links of R;
      2. B^S = boundary vertices reached from s, B^T = boundary vertices that
         reach t (disjoint: s no longer reaches t);
      3. Augment(s, B^S): the remaining supply to B^S, each vertex of B^S
         joined to t without bound;
      4. Augment(B^T, t): paths from B^T, each supplied without bound, to t;
    then in the final residual network, for v in R: s -> v strong source,
    v -> t strong sink, otherwise v -/-> B^R weak source and B^R -/-> v weak
    sink.  Reachability from s starts at the vertices of R with unsent supply
    (the supply of B^T is the auxiliary source of step 4, not s).

    ``augment="pr"`` runs the steps with the push-relabel maximum preflow
    instead; its excess stranded by step 4 is not a flow, and the weak sink
    class then goes wrong (kept only so that the tests can show that)."""
    pu, pv, cuv, cvu = grid_pairs(inst.dims, inst.nbr, _offsets(inst))
    region = grid_regions(inst.dims, tile)
    cls = np.zeros(inst.n, np.uint8)
    cs_all = np.asarray(inst.cs, np.int64)
    ct_all = np.asarray(inst.ct, np.int64)
    for rk in np.unique(region):
        inR = region == rk
        touch = inR[pu] | inR[pv]
        a, b = pu[touch], pv[touch]
        verts = np.unique(np.concatenate([np.flatnonzero(inR), a, b]))
        idx = -np.ones(inst.n, np.int64)
        idx[verts] = np.arange(len(verts))
        la, lb = idx[a], idx[b]
        rin = inR[verts]
        bnd = ~rin
        nl = len(verts)
        zero = np.zeros(nl, np.int64)
        # 1. Augment(s, t)
        s1 = solve_pairs(nl, la, lb, cuv[touch], cvu[touch],
                         np.where(rin, cs_all[verts], 0), np.where(rin, ct_all[verts], 0),
                         method=augment)
        from_s1, not_to_t1 = cuts_of_state(nl, la, lb, s1["r_uv"], s1["r_vu"], s1["rt"], s1["ex"])
        # 2. the source and sink boundary sets
        BS = bnd & (from_s1 == 1)
        BT = bnd & (not_to_t1 == 0)
        assert not (BS & BT).any(), "B^S and B^T intersect"
        # 3. Augment(s, B^S)
        s3 = solve_pairs(nl, la, lb, s1["r_uv"], s1["r_vu"], np.where(rin, s1["ex"], 0),
                         np.where(rin, s1["rt"], np.where(BS, big, 0)), method=augment)
        supply = np.where(rin, s3["ex"], 0)
        # 4. Augment(B^T, t)
        s4 = solve_pairs(nl, la, lb, s3["r_uv"], s3["r_vu"], np.where(BT, big, 0),
                         np.where(rin, s3["rt"], 0), method=augment)
        r_uv, r_vu, rt = s4["r_uv"], s4["r_vu"], np.where(rin, s4["rt"], 0)
        # classification in the final residual network
        from_s, not_to_t = cuts_of_state(nl, la, lb, r_uv, r_vu, rt, supply)
        from_b, _ = cuts_of_state(nl, la, lb, r_uv, r_vu, zero, bnd.astype(np.int64))
        _, not_to_b = cuts_of_state(nl, la, lb, r_uv, r_vu, bnd.astype(np.int64), zero)
        c = np.zeros(nl, np.uint8)
        strong_src = from_s == 1
        strong_snk = not_to_t == 0
        other = ~strong_src & ~strong_snk
        c[strong_src] |= REDUCE_STRONG_SOURCE
        c[strong_snk] |= REDUCE_STRONG_SINK
        c[other & (not_to_b == 1)] |= REDUCE_WEAK_SOURCE
        c[other & (from_b == 0)] |= REDUCE_WEAK_SINK
        cls[verts[rin]] = c[rin]
    return cls


def region_reduction_union(inst, tile):
    """The classes of region_reduction for every region at once, from the two
    auxiliary problems of Sec. 8 (each boundary vertex joined to t, or supplied
    from s, without bound), for large grids.  In the auxiliary problem of region
    R a boundary vertex w is a terminal, so an arc (u, w) leaving R acts as a
    t-link of u of capacity c(u, w) (or an arc (w, u) entering R as an s-link of
    u of capacity c(w, u)); the networks of all regions together are then one
    network with every arc between regions replaced that way, whose components
    are the regions.  Two textbook max flows (push-relabel) give the extremal
    cuts: strong source = minimal source side with boundary sinks, weak source =
    maximal minus minimal there; strong sink = outside the maximal source side
    with boundary sources, weak sink = maximal minus minimal there.  Pinned
    against the steps of Alg. 5 (region_reduction) in the tests."""
    pu, pv, cuv, cvu = grid_pairs(inst.dims, inst.nbr, _offsets(inst))
    region = grid_regions(inst.dims, tile)
    cross = region[pu] != region[pv]
    n = inst.n
    cs = np.asarray(inst.cs, np.int64).copy()
    ct = np.asarray(inst.ct, np.int64).copy()
    out_t = np.zeros(n, np.int64)   # capacity of the arcs leaving each vertex's region
    in_s = np.zeros(n, np.int64)    # capacity of the arcs entering it
    np.add.at(out_t, pu[cross], cuv[cross].astype(np.int64))
    np.add.at(out_t, pv[cross], cvu[cross].astype(np.int64))
    np.add.at(in_s, pu[cross], cvu[cross].astype(np.int64))
    np.add.at(in_s, pv[cross], cuv[cross].astype(np.int64))
    keep = ~cross
    a, b, c1, c2 = pu[keep], pv[keep], cuv[keep], cvu[keep]
    nt = solve_pairs(n, a, b, c1, c2, cs, ct + out_t)
    ns = solve_pairs(n, a, b, c1, c2, cs + in_s, ct)
    cls = np.zeros(n, np.uint8)
    cls[nt["smin"] == 1] |= REDUCE_STRONG_SOURCE
    cls[(nt["smax"] == 1) & (nt["smin"] == 0)] |= REDUCE_WEAK_SOURCE
    cls[ns["smax"] == 0] |= REDUCE_STRONG_SINK
    cls[(ns["smax"] == 1) & (ns["smin"] == 0)] |= REDUCE_WEAK_SINK
    return cls


# ---------------------------------------------------------------------------
# Brute force and certificate
# ---------------------------------------------------------------------------

def cut_cost(side, pu, pv, cuv, cvu, cs, ct):
    """Cost of the cut with source side {v : side[v]} (eq. (1), excess form):
    s-links of sink-side vertices + t-links of source-side vertices + n-links
    from the source side to the sink side.  Works on one mask or a stack."""
    side = np.asarray(side).astype(np.int64)
    cs = np.asarray(cs, dtype=np.int64)
    ct = np.asarray(ct, dtype=np.int64)
    cost = (1 - side) @ cs + side @ ct
    su = side[..., np.asarray(pu, dtype=np.int64)]
    sv = side[..., np.asarray(pv, dtype=np.int64)]
    cost = cost + (su * (1 - sv)) @ np.asarray(cuv, dtype=np.int64) \
        + (sv * (1 - su)) @ np.asarray(cvu, dtype=np.int64)
    return cost


def brute_force(n, pu, pv, cuv, cvu, cs, ct):
    """Enumerate every source side C of V: min cost, and the intersection /
    union of all minimisers (the unique minimal / maximal minimum cuts)."""
    if n > 22:
        raise ValueError("brute force is for tiny networks only")
    masks = np.arange(1 << n, dtype=np.int64)
    bits = ((masks[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1).astype(np.int64)
    cost = cut_cost(bits, pu, pv, cuv, cvu, cs, ct)
    best = int(cost.min())
    arg = bits[cost == best]
    smin = arg.min(axis=0).astype(np.uint8)
    smax = arg.max(axis=0).astype(np.uint8)
    return dict(flow=best, smin=smin, smax=smax)


def certify(n, pu, pv, cuv, cvu, cs, ct, r_uv, r_vu, rt, ex, flow, smin=None, smax=None):
    """Raise AssertionError unless (r, rt, ex) is a feasible preflow state of
    the network with flow value ``flow`` and the given cuts have cost ``flow``."""
    pu = np.asarray(pu, dtype=np.int64)
    pv = np.asarray(pv, dtype=np.int64)
    cuv = np.asarray(cuv, dtype=np.int64)
    cvu = np.asarray(cvu, dtype=np.int64)
    r_uv = np.asarray(r_uv, dtype=np.int64)
    r_vu = np.asarray(r_vu, dtype=np.int64)
    rt = np.asarray(rt, dtype=np.int64)
    ex = np.asarray(ex, dtype=np.int64)
    cs = np.asarray(cs, dtype=np.int64)
    ct = np.asarray(ct, dtype=np.int64)
    assert (r_uv >= 0).all() and (r_vu >= 0).all(), "negative residual"
    assert (r_uv + r_vu == cuv + cvu).all(), "residual pair sum changed"
    assert ((rt >= 0) & (rt <= ct)).all(), "t-link residual out of range"
    assert (ex >= 0).all(), "negative excess"
    f_uv = cuv - r_uv  # net flow pu -> pv
    net_in = np.zeros(n, dtype=np.int64)
    np.add.at(net_in, pv, f_uv)
    np.subtract.at(net_in, pu, f_uv)
    assert (ex == cs - (ct - rt) + net_in).all(), "conservation violated"
    assert int(ex.sum()) + int(flow) == int(cs.sum()), "sum of excess + flow != sum of s-links"
    assert int((ct - rt).sum()) == int(flow), "flow value mismatch"
    for side in (smin, smax):
        if side is not None:
            c = int(cut_cost(side, pu, pv, cuv, cvu, cs, ct))
            assert c == int(flow), f"cut cost {c} != flow {flow}"
    return True
