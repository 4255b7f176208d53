"""Test helpers: turn the solver's row-major state into the oracle's pair form;
build a serpentine single-path instance."""
import numpy as np

import oracle
import synth


def state_to_pairs(inst, state):
    """Residuals (K, n) of the solver -> (r_uv, r_vu) in the order of oracle.grid_pairs."""
    offs = synth.offsets_for(len(inst.dims), inst.conn)
    dims = tuple(inst.dims)
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64).reshape(dims)
    res = state["res"]
    r_uv, r_vu = [], []
    for k in range(0, len(offs), 2):
        src, dst = [], []
        for size, o in zip(dims, offs[k]):
            if o >= 0:
                src.append(slice(0, size - o))
                dst.append(slice(o, size))
            else:
                src.append(slice(-o, size))
                dst.append(slice(0, size + o))
        u = idx[tuple(src)].reshape(-1)
        v = idx[tuple(dst)].reshape(-1)
        r_uv.append(res[k][u])
        r_vu.append(res[k + 1][v])
    return np.concatenate(r_uv).astype(np.int64), np.concatenate(r_vu).astype(np.int64)


def certify_solver_state(inst, out):
    """Feasibility, conservation and duality of a solver result (from the original caps)."""
    pu, pv, cuv, cvu = oracle.grid_pairs(inst.dims, inst.nbr, synth.offsets_for(len(inst.dims), inst.conn))
    r_uv, r_vu = state_to_pairs(inst, out["state"])
    st = out["state"]
    oracle.certify(inst.n, pu, pv, cuv, cvu, inst.cs, inst.ct, r_uv, r_vu, st["rt"], st["ex"],
                   out["flow"], out["smin"], out["smax"])
    # the returned cuts are the extremal cuts of the returned residual state
    smin, smax = oracle.cuts_of_state(inst.n, pu, pv, r_uv, r_vu, st["rt"], st["ex"])
    assert (smin == out["smin"]).all() and (smax == out["smax"]).all()


def serpentine_instance(dims, conn, tile, fwd=50, src=100, sink=30, frac=2 / 3):
    """One residual path in boustrophedon order (x fastest, then y, then z, each
    reversing after the previous axis wraps) through the first frac of the
    vertices: arcs of capacity fwd forward and 0 backward along it, every other
    arc 0, c(s, first) = src, c(last, t) = sink.  With src > sink < fwd the flow
    is sink, the minimal source side is the path (excess stays at the start and
    the forward arcs keep fwd - sink) and the maximal source side is every vertex
    (nothing reaches t once c(last, t) is used up).
    Returns (instance, path as row-major vertex indices)."""
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    offs = synth.offsets_for(nd, conn)
    n = int(np.prod(dims))
    coords = []
    d3 = (1,) * (3 - nd) + dims
    for z in range(d3[0]):
        ys = range(d3[1]) if z % 2 == 0 else range(d3[1] - 1, -1, -1)
        for j, y in enumerate(ys):
            row = z * d3[1] + j  # rows visited so far decide the x direction
            xs = range(d3[2]) if row % 2 == 0 else range(d3[2] - 1, -1, -1)
            for x in xs:
                coords.append((z, y, x))
    coords = coords[:max(2, int(len(coords) * frac))]
    path = [((z * d3[1] + y) * d3[2] + x) for z, y, x in coords]
    nbr = np.zeros((len(offs), n), np.int32)
    for (a, b) in zip(coords, coords[1:]):
        step = tuple(q - p for p, q in zip(a, b))[3 - nd:]
        k = [tuple(o) for o in offs].index(step)
        u = (a[0] * d3[1] + a[1]) * d3[2] + a[2]
        nbr[k, u] = fwd
    cs = np.zeros(n, np.int32)
    ct = np.zeros(n, np.int32)
    cs[path[0]] = src
    ct[path[-1]] = sink
    inst = synth.GridInstance(dims=dims, conn=conn, cs=cs, ct=ct, nbr=nbr, tile=tuple(tile),
                              name=f"serpentine{nd}d{conn}_{'x'.join(map(str, dims))}")
    return inst, np.array(path, np.int64)


def region_chain_instance(L, w, excess=10, big=1000):
    """A 1 x (L w) 4-connected grid cut into L regions of width w: arcs of
    capacity big to the right, excess at the first vertex of every region and
    c(last, t) = big.  After the first P-ARD sweep every region but the last
    is labelled 1 (it reaches only its right neighbour's boundary, labelled 0
    at the start) and the last one 0; the exact region distance of region j is
    L - 1 - j, and the flow is L * excess."""
    inst, _ = serpentine_instance((1, L * w), 4, (1, w), fwd=big, src=excess, sink=big, frac=1.0)
    inst.cs[::w] = excess
    inst.name = f"regionchain_{L}x{w}"
    return inst


def boundary_mask(inst, tile):
    """Geometric boundary set B (Sec. 4.1): vertices with a grid neighbour in
    another region, zero-capacity arcs included."""
    pu, pv, _, _ = oracle.grid_pairs(inst.dims, inst.nbr, synth.offsets_for(len(inst.dims), inst.conn))
    region = oracle.grid_regions(inst.dims, tile)
    cross = region[pu] != region[pv]
    b = np.zeros(inst.n, bool)
    b[pu[cross]] = True
    b[pv[cross]] = True
    return b


def region_distance(n, pu, pv, r_uv, r_vu, region, rt, dinf):
    """Exact d*B (Sec. 4.1), capped at dinf: the distance to t in the residual
    network where an arc between regions has length 1 and an arc inside a
    region length 0.  Shortest paths from t on the reversed residual arcs
    (scipy's Dijkstra), with length-0 arcs given a weight far below 1 / n."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    pu = np.asarray(pu, np.int64)
    pv = np.asarray(pv, np.int64)
    eps = 1e-9
    inter = (np.asarray(region)[pu] != np.asarray(region)[pv])
    w = np.where(inter, 1.0, eps)
    rows, cols, wts = [], [], []
    m = np.asarray(r_uv) > 0          # arc pu -> pv: reversed edge pv -> pu
    rows.append(pv[m]); cols.append(pu[m]); wts.append(w[m])
    m = np.asarray(r_vu) > 0          # arc pv -> pu: reversed edge pu -> pv
    rows.append(pu[m]); cols.append(pv[m]); wts.append(w[m])
    tv = np.flatnonzero(np.asarray(rt) > 0)
    rows.append(np.full(tv.size, n)); cols.append(tv); wts.append(np.full(tv.size, eps))
    A = csr_matrix((np.concatenate(wts), (np.concatenate(rows), np.concatenate(cols))),
                   shape=(n + 1, n + 1))
    d = dijkstra(A, directed=True, indices=n)[:n]
    out = np.full(n, dinf, np.int64)
    fin = np.isfinite(d)
    out[fin] = np.minimum(np.floor(d[fin] + 1e-3).astype(np.int64), dinf)
    return out


def assert_valid_labels(pu, pv, r_uv, r_vu, region, rt, d, bmask, dinf, lifted=False):
    """Validity of Sec. 4.1 on every residual arc (d(u) <= d(v) + length, length
    1 between regions and 0 inside one) and d = 0 wherever r_t > 0.  The solver
    raises only boundary labels in the global gap, and so does the boundary
    relabel (interior labels are recomputed by the region's next discharge
    before anything reads them): an arc from a boundary vertex labelled dinf to
    an interior vertex of its region is not checked, nor, with lifted (the
    boundary relabel on), any arc from a boundary vertex to an interior vertex
    of its region."""
    pu = np.asarray(pu, np.int64)
    pv = np.asarray(pv, np.int64)
    d = np.asarray(d, np.int64)
    ln = (region[pu] != region[pv]).astype(np.int64)
    for tail, head, res in ((pu, pv, r_uv), (pv, pu, r_vu)):
        m = np.asarray(res) > 0
        bad = m & (d[tail] > d[head] + ln)
        into_interior = (ln == 0) & bmask[tail] & ~bmask[head]
        bad &= ~(into_interior & ((d[tail] == dinf) | lifted))
        assert not bad.any(), f"{int(bad.sum())} residual arcs violate d(u) <= d(v) + |(u,v)|"
    assert (d[np.asarray(rt) > 0] == 0).all(), "a vertex with a residual t-link has d > 0"
