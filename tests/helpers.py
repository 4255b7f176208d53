"""Test helpers: turn the solver's row-major state into the oracle's pair form."""
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
