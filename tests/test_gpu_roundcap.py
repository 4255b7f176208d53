"""GPU parity of capped discharges (mf_solve_opts.round_cap: at most n
search-and-push rounds of a region discharge per sweep, the rest of its excess
carried to the next sweep): the int64 flow and both extremal cuts equal to the
oracle's, the final state certified, on every region kernel, with tiny caps
that force many carries, and combined with partial discharges, the exact and
boundary relabels, the colour phases, captured sweep batches and batches."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import certify_solver_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_1109_1146_amd import mf as _mf
    _mf.load()
    return _mf


CASES = [
    # dims, conn, tile, kernel
    ((64, 72), 8, (16, 16), "WAVE"),
    ((70, 66), 4, (32, 32), "WAVE"),
    ((8, 40, 70), 6, (4, 16, 32), "ROWS"),
    ((64, 70, 66), 6, (64, 64, 64), "ROWS64"),
    ((12, 14, 16), 6, (6, 7, 8), "LDS"),
    ((40, 38), 8, (20, 19), "LDS"),
    ((10, 12, 14), 6, (5, 6, 7), "HBM"),
    ((36, 30), 4, (12, 15), "HBM"),
]


def _instance(case, seed):
    dims, conn, tile, _ = case
    if seed % 2:
        return synth.blob_grid(dims, conn, 9100 + seed, 4, 3.0, 10.0, zero_frac=0.1, tile=tile,
                               name=f"rc_blob_{seed}")
    return synth.random_grid(dims, conn, 9100 + seed, tile=tile)


@pytest.mark.parametrize("cap", [1, 2, 5])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_round_cap_exact_on_every_kernel(mf, ci, cap):
    case = CASES[ci]
    inst = _instance(case, ci * 3 + cap)
    kname = case[3]
    print(f"case {inst.name} dims={inst.dims} tile={inst.tile} kernel={kname} cap={cap}", flush=True)
    out = mf.solve_instance(inst, region_kernel=getattr(mf, "MF_KERNEL_" + kname), round_cap=cap,
                            max_sweeps=1 << 40)
    ref = oracle.solve_grid(inst)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()
    certify_solver_state(inst, out)
    assert out["stats"]["region_kernel"] == getattr(mf, "MF_KERNEL_" + kname)


COMBOS = [
    dict(partial=True), dict(global_relabel_every=3), dict(boundary_relabel=8),
    dict(schedule=1), dict(graph=True, global_relabel_every=4), dict(partial=True, boundary_relabel=4),
]


@pytest.mark.parametrize("k", range(len(COMBOS)))
def test_round_cap_with_other_options(mf, k):
    kw = COMBOS[k]
    for case in (CASES[0], CASES[2], CASES[3]):
        inst = _instance(case, 40 + k)
        print(f"case {inst.name} dims={inst.dims} {kw}", flush=True)
        out = mf.solve_instance(inst, round_cap=2, max_sweeps=1 << 40, **kw)
        ref = oracle.solve_grid(inst)
        assert out["flow"] == ref["flow"]
        assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()


def test_round_cap_batch(mf):
    rng = np.random.default_rng(9)
    insts = [synth.blob_grid((int(rng.integers(20, 120)), int(rng.integers(20, 120))), 4 if i % 2 else 8,
                             9200 + i, 3, 6.0, 6.0) for i in range(12)]
    b = mf.load_batch(insts, region_shape=(32, 32))
    try:
        b.solve(round_cap=3, graph=True, global_relabel_every=4, max_sweeps=1 << 40)
        flows = b.flow_values()
        for i, inst in enumerate(insts):
            ref = oracle.solve_grid(inst)
            assert flows[i] == ref["flow"]
            assert (b.instance_cut(i, mf.MF_CUT_MIN_SOURCE) == ref["smin"]).all()
    finally:
        b.close()


def test_round_cap_rejected_with_prd_and_negative(mf):
    inst = synth.random_grid((16, 16), 4, 9300, tile=(8, 8))
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        for kw in (dict(round_cap=-1), dict(round_cap=2, method=mf.MF_METHOD_PRD)):
            with pytest.raises(mf.MFError) as e:
                g.solve(**kw)
            assert e.value.status == mf.MF_E_INVAL


@pytest.mark.parametrize("dims,conn,tile", [((64, 64), 8, (64, 64)), ((64, 64, 64), 6, (64, 64, 64)),
                                            ((30, 40), 4, (8, 8))])
def test_round_cap_default_guard(mf, dims, conn, tile):
    """With capped rounds the 2|B|^2 + 1 bound of full discharges does not hold
    (a single region, |B| = 0, may need many sweeps for its one discharge), so
    the default guard (max_sweeps = 0) must not stop a capped solve early."""
    inst = synth.blob_grid(dims, conn, 9300 + len(dims), 4, 3.0, 10.0, tile=tile, name="rc_guard")
    print(f"case {inst.name} dims={dims} tile={tile} cap=1 default guard", flush=True)
    out = mf.solve_instance(inst, round_cap=1)
    ref = oracle.solve_grid(inst)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()
