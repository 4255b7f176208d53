"""GPU parity of the labels themselves (Sec. 4), not only of the flow and cuts:
the solver is stopped after s = 1, 2 and 3 sweeps and its own state is read
back (mf_get_state).  On that state:

* validity of Sec. 4.1 on every residual arc and t-link (the global gap
  raises only boundary labels; an arc from a boundary vertex at dinf to an
  interior vertex of its region is the one exemption);
* labels <= min(d*B, dinf), d*B from a separate shortest-path computation;
* after a full sweep only boundary vertices are active (Sec. 4.3-4.4), when
  discharges are not partial;
* the region relabel entry point gives, bit for bit, the labels of Alg. 3
  recomputed by the oracle from the same state and the same halo labels;
* the exact relabel entry point gives min(d*B, dinf) bit for bit (row a6);
* over a whole solve, the per-step label trace never decreases (Sec. 4.2
  monotonicity) and its last entry is the final state's labels.

Every region kernel (wavefront, row-bitmask with 32- and 64-vertex rows, LDS
workgroup, HBM), with and without partial discharges, capped discharge rounds
and the boundary relabel, and the colour phases of Alg. 1."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import assert_valid_labels, boundary_mask, region_distance, state_to_pairs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_1109_1146_amd import mf as _mf
    _mf.load()
    return _mf


# name, dims, conn, tile, kernel, solve options, blob capacities
CASES = [
    ("2d4_wave", (40, 44), 4, (16, 16), "WAVE", {}, False),
    ("2d8_wave_partial", (48, 40), 8, (16, 20), "WAVE", dict(partial=True), True),
    ("2d8_lds_brl", (40, 40), 8, (20, 20), "LDS", dict(boundary_relabel=8), False),
    ("2d4_hbm", (36, 30), 4, (12, 15), "HBM", {}, True),
    ("2d4_wave_colored", (40, 44), 4, (16, 16), "WAVE", dict(schedule=1), False),
    ("3d_rows", (8, 20, 40), 6, (4, 16, 32), "ROWS", {}, False),
    ("3d_rows_partial_brl", (8, 24, 64), 6, (4, 16, 32), "ROWS", dict(partial=True, boundary_relabel=8), True),
    ("3d_lds", (12, 12, 14), 6, (6, 6, 7), "LDS", {}, True),
    ("3d_hbm_partial", (10, 12, 14), 6, (5, 6, 7), "HBM", dict(partial=True), False),
    ("3d_rows64", (64, 64, 100), 6, (64, 64, 64), "ROWS64", {}, True),
    ("3d_rows64_partial_brl", (64, 100, 64), 6, (64, 64, 64), "ROWS64",
     dict(partial=True, boundary_relabel=8), False),
    ("2d8_wave_roundcap", (48, 40), 8, (16, 20), "WAVE", dict(round_cap=1), True),
    ("3d_rows64_roundcap", (64, 64, 100), 6, (64, 64, 64), "ROWS64", dict(round_cap=2), True),
    ("3d_hbm_roundcap", (10, 12, 14), 6, (5, 6, 7), "HBM", dict(round_cap=1), False),
]


def _instance(case):
    name, dims, conn, tile, _, _, blob = case
    seed = 5000 + CASES.index(case)
    if blob:
        return synth.blob_grid(dims, conn, seed, 4, 3.0, 10.0, zero_frac=0.1, tile=tile, name=name)
    return synth.random_grid(dims, conn, seed, tile=tile)


def _kernel(mf, name):
    return getattr(mf, "MF_KERNEL_" + name)


def _geometry(inst, tile):
    pu, pv, _, _ = oracle.grid_pairs(inst.dims, inst.nbr, synth.offsets_for(len(inst.dims), inst.conn))
    return pu, pv, oracle.grid_regions(inst.dims, tile), boundary_mask(inst, tile)


@pytest.mark.parametrize("sweeps", [1, 2, 3])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_labels_after_sweeps(mf, ci, sweeps):
    case = CASES[ci]
    name, dims, conn, tile, kname, kw, _ = case
    inst = _instance(case)
    kernel = _kernel(mf, kname)
    print(f"case {name} dims={dims} tile={tile} kernel={kname} {kw} sweeps={sweeps}", flush=True)
    with mf.Grid(inst.dims, inst.conn, tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        try:
            st = g.solve(max_sweeps=sweeps, check_every=1, region_kernel=kernel, **kw)
            assert st["sweeps"] <= sweeps
        except mf.MFError as e:
            assert e.status == mf.MF_E_SWEEPS
        info = g.info()
        dinf = max(info["boundary_size"], 1)
        state = g.state()
        pu, pv, region, bmask = _geometry(inst, tile)
        r_uv, r_vu = state_to_pairs(inst, state)
        rt, ex, lab = state["rt"], state["ex"], state["labels"].astype(np.int64)
        assert (lab >= 0).all() and (lab <= dinf).all()
        # Sec. 4.1: a valid labeling, below the exact region distance
        assert_valid_labels(pu, pv, r_uv, r_vu, region, rt, lab, bmask, dinf,
                            lifted=bool(kw.get("boundary_relabel")))
        dstar = region_distance(inst.n, pu, pv, r_uv, r_vu, region, rt, dinf)
        assert (lab <= dstar).all(), f"{int((lab > dstar).sum())} labels above d*B"
        # Sec. 4.3-4.4: after a full sweep only boundary vertices are active
        # (partial and capped discharges may leave excess inside a region)
        if not kw.get("partial") and not kw.get("round_cap"):
            active = (ex > 0) & (lab < dinf)
            assert not (active & ~bmask).any(), f"{int((active & ~bmask).sum())} active interior vertices"
        # Alg. 3 on this state, with these labels as the halo labels
        want = oracle.region_relabel(inst.n, pu, pv, r_uv, r_vu, rt, region, lab, dinf)
        g.region_relabel(kernel)
        s2 = g.state()
        assert (s2["res"] == state["res"]).all() and (s2["ex"] == ex).all() and (s2["rt"] == rt).all()
        assert (s2["labels"] == want).all(), f"{int((s2['labels'] != want).sum())} labels differ from Alg. 3"
        # row a6: the exact relabel is min(d*B, dinf)
        g.global_relabel()
        s3 = g.state()
        assert (s3["labels"] == dstar).all(), f"{int((s3['labels'] != dstar).sum())} labels differ from d*B"


@pytest.mark.parametrize("ci", range(len(CASES)))
def test_labels_monotone_over_a_solve(mf, ci):
    torch = pytest.importorskip("torch")
    case = CASES[ci]
    name, dims, conn, tile, kname, kw, _ = case
    inst = _instance(case)
    print(f"case {name} dims={dims} tile={tile} kernel={kname} {kw} (label trace)", flush=True)
    cap = 48
    trace = torch.full((cap, inst.n), -1, dtype=torch.int32, device="cuda")
    with mf.Grid(inst.dims, inst.conn, tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        st = g.solve(region_kernel=_kernel(mf, kname), label_trace=trace, max_sweeps=100000,
                     global_relabel_every=3 if ci % 2 else 0, **kw)
        final = g.state()["labels"]
        ref = oracle.solve_grid(inst)
        assert g.flow_value() == ref["flow"]
    tr = trace.cpu().numpy()
    used = int((tr[:, 0] >= 0).sum())  # every enqueued step up to cap writes its row
    assert used >= 1 and (tr[:used] >= 0).all() and (tr[used:] == -1).all()
    for s in range(1, used):
        dec = tr[s] < tr[s - 1]
        assert not dec.any(), f"step {s}: {int(dec.sum())} labels decreased"
    if used < cap:
        # every step of the solve was recorded: the last one holds the final labels
        assert (tr[used - 1] == final).all()
    assert st["sweeps"] >= 1


def test_max_sweeps_stops_exactly(mf):
    """With the default check interval (8 sweeps), a solve limited to 3 sweeps
    runs exactly 3 (the label trace records every enqueued step) and reports
    MF_E_SWEEPS; its state is the state after those 3 sweeps."""
    torch = pytest.importorskip("torch")
    inst = synth.random_grid((40, 44), 4, 5100, tile=(8, 8))
    trace = torch.full((16, inst.n), -1, dtype=torch.int32, device="cuda")
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        with pytest.raises(mf.MFError) as e:
            g.solve(max_sweeps=3, label_trace=trace)
        assert e.value.status == mf.MF_E_SWEEPS
        lab = g.state()["labels"]
        # the statistics of the three sweeps come with the error
        st = e.value.stats
        assert st is not None and st["sweeps"] == 3 and st["region_discharges"] > 0
    tr = trace.cpu().numpy()
    assert int((tr[:, 0] >= 0).sum()) == 3
    assert (tr[2] == lab).all()
