"""Push-relabel region discharge on the GPU (Sec. 3, Proc. PRD, under the
parallel driver of Alg. 2): the flow and both extremal cuts are the oracle's,
the final labels are valid distance labels (Sec. 2), and on the same partition
it needs more sweeps than ARD, the paper's comparison."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import certify_solver_state, state_to_pairs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_1109_1146_amd import mf as _mf
    _mf.load()
    return _mf


CASES = [((12, 13), 4, (4, 5)), ((16, 16), 8, (8, 8)), ((6, 7, 8), 6, (3, 4, 4)),
         ((40, 36), 8, (8, 8)), ((9, 10, 11), 6, (4, 4, 4)), ((33, 31), 4, (16, 16)),
         ((70, 90), 8, (32, 32)), ((8, 40, 70), 6, (4, 16, 32))]


def _assert_valid_distance_labels(inst, st, dinf):
    """d(u) <= d(v) + 1 on every residual arc, d(u) <= 1 where c_f(u, t) > 0."""
    pu, pv, _, _ = oracle.grid_pairs(inst.dims, inst.nbr, oracle._offsets(inst))
    r_uv, r_vu = state_to_pairs(inst, st)
    d = np.minimum(st["labels"].astype(np.int64), dinf)
    assert (d[pu][r_uv > 0] <= d[pv][r_uv > 0] + 1).all()
    assert (d[pv][r_vu > 0] <= d[pu][r_vu > 0] + 1).all()
    assert (d[st["rt"] > 0] <= 1).all()


@pytest.mark.parametrize("seed", range(16))
def test_prd_random_grids_exact(mf, seed):
    dims, conn, tile = CASES[seed % len(CASES)]
    inst = (synth.blob_grid(dims, conn, 3300 + seed, 4, 3.0, 9.0, zero_frac=0.1, tile=tile) if seed % 2
            else synth.random_grid(dims, conn, 3300 + seed, tile=tile))
    print(f"case {inst.name} dims={dims} tile={tile}", flush=True)
    ref = oracle.solve_grid(inst)
    out = mf.solve_instance(inst, method=mf.MF_METHOD_PRD, max_sweeps=1000000)
    assert out["stats"]["region_kernel"] == mf.MF_KERNEL_HBM
    assert out["stats"]["d_inf"] == inst.n
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()
    certify_solver_state(inst, out)
    _assert_valid_distance_labels(inst, out["state"], inst.n)
    ard = mf.solve_instance(inst, max_sweeps=1000000)
    print(f"  sweeps: PRD {out['stats']['sweeps']}, ARD {ard['stats']['sweeps']}", flush=True)


def test_prd_needs_more_sweeps_than_ard(mf):
    """The paper's comparison (Tables 1 and 2), summed over a family."""
    prd = ard = 0
    for seed in range(6):
        dims, conn, tile = CASES[seed]
        inst = synth.random_grid(dims, conn, 3400 + seed, tile=tile)
        prd += mf.solve_instance(inst, method=mf.MF_METHOD_PRD, max_sweeps=1000000)["stats"]["sweeps"]
        ard += mf.solve_instance(inst, max_sweeps=1000000)["stats"]["sweeps"]
    print(f"P-PRD {prd} sweeps, P-ARD {ard} sweeps", flush=True)
    assert prd > ard


@pytest.mark.parametrize("case", range(3))
def test_prd_large_regions_and_ragged(mf, case):
    """1024-thread workgroups (regions of 64K vertices) and ragged tiles."""
    cases = [((300, 280), 8, (256, 256)), ((70, 66, 65), 6, (64, 64, 64)), ((37, 45), 4, (8, 16))]
    dims, conn, tile = cases[case]
    inst = synth.blob_grid(dims, conn, 3500 + case, 6, 6.0, 24.0, zero_frac=0.1, tile=tile)
    ref = oracle.solve_grid(inst)
    out = mf.solve_instance(inst, method=mf.MF_METHOD_PRD, max_sweeps=1000000)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()


def test_prd_graph_replay_matches_eager(mf):
    inst = synth.blob_grid((128, 96), 8, 3600, 6, 6.0, 20.0, zero_frac=0.1, tile=(32, 32))
    ref = oracle.solve_grid(inst)
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        eager = g.solve(method=mf.MF_METHOD_PRD, max_sweeps=1000000)
        assert g.flow_value() == ref["flow"]
        for rep in range(3):
            st = g.solve(method=mf.MF_METHOD_PRD, graph=True, check_every=4, max_sweeps=1000000)
            print(f"replay {rep}: sweeps {st['sweeps']} (eager {eager['sweeps']})", flush=True)
            assert g.flow_value() == ref["flow"]
            assert (g.min_cut(mf.MF_CUT_MIN_SOURCE) == ref["smin"]).all()
            g.solve(max_sweeps=100000)  # ARD in between, same handle
            assert g.flow_value() == ref["flow"]


def test_prd_batch_exact(mf):
    insts = synth.config3_instances(24)
    b = mf.load_batch(insts, region_shape=(32, 32))
    try:
        b.solve(method=mf.MF_METHOD_PRD, max_sweeps=1000000)
        flows = b.flow_values()
        for i, inst in enumerate(insts):
            ref = oracle.solve_grid(inst)
            assert flows[i] == ref["flow"], (i, inst.name)
            assert (b.instance_cut(i, mf.MF_CUT_MIN_SOURCE) == ref["smin"]).all(), (i, inst.name)
    finally:
        b.close()


def test_prd_rejected_combinations(mf):
    inst = synth.random_grid((16, 16), 4, 3700, tile=(8, 8))
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        bad = [dict(partial=True), dict(boundary_relabel=4), dict(global_relabel_every=4),
               dict(region_kernel=mf.MF_KERNEL_WAVE), dict(region_kernel=mf.MF_KERNEL_LDS),
               dict(method=7)]
        for kw in bad:
            kw.setdefault("method", mf.MF_METHOD_PRD)
            with pytest.raises(mf.MFError) as e:
                g.solve(**kw)
            assert e.value.status == mf.MF_E_INVAL, kw
        g.solve(method=mf.MF_METHOD_PRD)
        with pytest.raises(mf.MFError) as e:
            g.boundary_relabel()  # a PRD state has no region-distance labels
        assert e.value.status == mf.MF_E_STATE


@pytest.mark.parametrize("case", range(4))
def test_prd_degenerate_inputs(mf, case):
    """One region (plain push-relabel: one sweep), no n-links, no t-links, no s-links."""
    dims, conn, tile = [((20, 18), 8, (20, 18)), ((9, 10, 11), 6, (4, 4, 4)),
                        ((30, 31), 4, (8, 8)), ((15, 16), 8, (4, 4))][case]
    inst = synth.random_grid(dims, conn, 3800 + case, tile=tile)
    if case == 1:
        inst.nbr[:] = 0
    elif case == 2:
        inst.ct[:] = 0
    elif case == 3:
        inst.cs[:] = 0
    ref = oracle.solve_grid(inst)
    out = mf.solve_instance(inst, method=mf.MF_METHOD_PRD, max_sweeps=1000000)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()
    if case == 0:
        assert out["stats"]["sweeps"] == 1


def test_prd_stops_at_max_sweeps(mf):
    inst = synth.random_grid((40, 36), 8, 3900, tile=(8, 8))
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        with pytest.raises(mf.MFError) as e:
            g.solve(method=mf.MF_METHOD_PRD, max_sweeps=2, check_every=1)
        assert e.value.status == mf.MF_E_SWEEPS
        st = g.state()  # the state after two sweeps stays readable
        assert st["labels"].max() <= inst.n


def test_prd_full_size_2048_exact(mf):
    """The 2048^2 workload by push-relabel region discharge: the oracle's flow and cuts."""
    inst = synth.config(1)
    out = mf.solve_instance(inst, method=mf.MF_METHOD_PRD, max_sweeps=1000000)
    ref = oracle.solve_grid(inst)
    print(f"{inst.name}: PRD sweeps {out['stats']['sweeps']}", flush=True)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()
