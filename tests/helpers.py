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
