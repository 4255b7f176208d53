"""GPU parity of the 64-vertex-row discharge kernel (64^3 regions, the tile of
the 464^3 workload) against the CPU oracle: the int64 flow value and both
extremal minimum cuts identical, the residual state certified from the
original capacities, on ragged grids with random and blob capacities, with and
without the exact relabel, partial discharges and the boundary relabel."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import certify_solver_state

pytestmark = pytest.mark.gpu

T64 = (64, 64, 64)


@pytest.fixture(scope="module")
def mf():
    from paper_1109_1146_amd import mf as _mf
    _mf.load()
    return _mf


def _check(mf, inst, certify=True, **kw):
    print(f"case {inst.name} dims={inst.dims} tile={inst.tile} {kw}", flush=True)
    out = mf.solve_instance(inst, tile=T64, max_sweeps=100000, **kw)
    ref = oracle.solve_grid(inst)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all()
    assert (out["smax"] == ref["smax"]).all()
    if certify:
        certify_solver_state(inst, out)
    return out


def test_auto_selects_rows64(mf):
    inst = synth.blob_grid((70, 66, 130), 6, 4100, 6, 6.0, 24.0, zero_frac=0.1, tile=T64,
                           name="blob3d_t64")
    out = _check(mf, inst)
    assert out["stats"]["region_kernel"] == mf.MF_KERNEL_ROWS64
    assert out["stats"]["sweeps"] <= 2 * out["info"]["boundary_size"] ** 2 + 1


CASES = [
    ((64, 64, 64), "random", {}),
    ((65, 70, 128), "random", {}),
    ((128, 64, 70), "blob", {}),
    ((70, 66, 130), "blob", dict(global_relabel_every=4)),
    ((96, 100, 66), "random", dict(global_relabel_every=2)),
    ((66, 128, 64), "blob", dict(partial=True)),
    ((70, 70, 70), "random", dict(partial=True, global_relabel_every=3)),
    ((64, 130, 65), "blob", dict(boundary_relabel=16)),
    ((127, 65, 66), "random", dict(partial=True, boundary_relabel=8)),
    ((100, 70, 64), "blob", dict(schedule=1)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_rows64_exact(mf, case):
    dims, kind, kw = CASES[case]
    if kind == "random":
        inst = synth.random_grid(dims, 6, 4200 + case, tile=T64, cap_hi=20 if case % 2 else 10)
    else:
        inst = synth.blob_grid(dims, 6, 4300 + case, 6, 4.0, 16.0, zero_frac=0.1, tile=T64,
                               name=f"rows64_blob_{case}")
    out = _check(mf, inst, region_kernel=mf.MF_KERNEL_ROWS64, **kw)
    assert out["stats"]["region_kernel"] == mf.MF_KERNEL_ROWS64


def test_rows64_single_region(mf):
    """One 64^3 region: no boundary, d_inf = 1, one sweep is the whole maximum flow."""
    inst = synth.blob_grid((64, 64, 64), 6, 4400, 4, 4.0, 12.0, tile=T64, name="rows64_single")
    out = _check(mf, inst, region_kernel=mf.MF_KERNEL_ROWS64)
    assert out["info"]["boundary_size"] == 0
    assert out["stats"]["sweeps"] <= 1


def test_rows64_selection_errors(mf):
    """ROWS64 needs 3D 6-connected 64^3 tiles."""
    for dims, conn, tile in (((64, 64), 8, (64, 64)), ((40, 40, 70), 6, (32, 32, 32)),
                             ((70, 70, 70), 6, (32, 64, 64))):
        inst = synth.random_grid(dims, conn, 6, tile=tile)
        with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
            g.set_caps(inst.cs, inst.ct, inst.nbr)
            with pytest.raises(mf.MFError) as e:
                g.solve(region_kernel=mf.MF_KERNEL_ROWS64)
            assert e.value.status == mf.MF_E_INVAL



@pytest.mark.parametrize("sweeps", [1, 2, 4])
@pytest.mark.parametrize("kind", ["random", "blob"])
def test_rows64_exact_relabel_is_region_distance(mf, kind, sweeps):
    """Row a6 on 64^3 tiles (the 64-vertex-row relabel kernel): on the solver's
    own state after 1, 2 and 4 sweeps, the exact relabel gives min(d*B, dinf)
    bit for bit, d*B from a separate shortest-path computation; eight regions,
    ragged on every axis, so that seeds cross every face direction."""
    from tests.helpers import region_distance, state_to_pairs
    dims = (100, 128, 90)
    if kind == "random":
        inst = synth.random_grid(dims, 6, 4500 + sweeps, tile=T64, cap_hi=12)
    else:
        inst = synth.blob_grid(dims, 6, 4510 + sweeps, 6, 4.0, 16.0, zero_frac=0.1, tile=T64,
                               name=f"rows64_relabel_{sweeps}")
    print(f"case {inst.name} dims={dims} sweeps={sweeps}", flush=True)
    with mf.Grid(inst.dims, inst.conn, T64) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        try:
            g.solve(max_sweeps=sweeps, check_every=1, region_kernel=mf.MF_KERNEL_ROWS64)
        except mf.MFError as e:
            assert e.status == mf.MF_E_SWEEPS
        dinf = max(g.info()["boundary_size"], 1)
        g.global_relabel()
        state = g.state()
    pu, pv, _, _ = oracle.grid_pairs(inst.dims, inst.nbr, synth.offsets_for(3, 6))
    region = oracle.grid_regions(inst.dims, T64)
    r_uv, r_vu = state_to_pairs(inst, state)
    dstar = region_distance(inst.n, pu, pv, r_uv, r_vu, region, state["rt"], dinf)
    lab = state["labels"].astype(np.int64)
    assert (lab == dstar).all(), f"{int((lab != dstar).sum())} labels differ from d*B"
