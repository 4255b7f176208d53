"""The sequential driver (Alg. 1) on the GPU as phases of non-interacting
regions (MF_SCHED_COLORED): one colour class per phase, its flow applied before
the next phase, so every region sees the current state of its neighbours.  The
flow and both extremal cuts are the oracle's on every region kernel, with the
exact relabel, captured sweep batches, batches and push-relabel region
discharge (S-PRD); and it needs fewer sweeps than the parallel driver."""
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


CASES = [((12, 13), 4, (4, 5)), ((16, 16), 8, (4, 8)), ((6, 7, 8), 6, (3, 4, 4)),
         ((40, 36), 8, (8, 8)), ((9, 10, 11), 6, (4, 4, 4)), ((33, 31), 4, (16, 16)),
         ((70, 90), 8, (32, 32)), ((8, 40, 70), 6, (4, 16, 32)), ((130, 70), 4, (64, 64))]


@pytest.mark.parametrize("kernel", ["auto", "hbm", "lds"])
@pytest.mark.parametrize("seed", range(9))
def test_colored_exact(mf, seed, kernel):
    dims, conn, tile = CASES[seed]
    inst = (synth.blob_grid(dims, conn, 4000 + seed, 4, 3.0, 9.0, zero_frac=0.1, tile=tile) if seed % 2
            else synth.random_grid(dims, conn, 4000 + seed, tile=tile))
    rk = {"auto": mf.MF_KERNEL_AUTO, "hbm": mf.MF_KERNEL_HBM, "lds": mf.MF_KERNEL_LDS}[kernel]
    ref = oracle.solve_grid(inst)
    for relabel in (0, 3):
        try:
            out = mf.solve_instance(inst, schedule=mf.MF_SCHED_COLORED, region_kernel=rk,
                                    global_relabel_every=relabel, max_sweeps=100000)
        except mf.MFError as e:
            if kernel == "lds" and e.status == mf.MF_E_INVAL:
                pytest.skip("region does not fit the LDS kernel")
            raise
        assert out["flow"] == ref["flow"]
        assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()
        certify_solver_state(inst, out)


def test_colored_needs_fewer_sweeps(mf):
    """Alg. 1 sees its neighbours' new state within a sweep: fewer sweeps than
    Alg. 2 summed over a family (the reference S-ARD shows the same)."""
    col = par = 0
    for seed in range(8):
        dims, conn, tile = CASES[seed]
        inst = synth.blob_grid(dims, conn, 4100 + seed, 4, 3.0, 9.0, zero_frac=0.1, tile=tile)
        col += mf.solve_instance(inst, schedule=mf.MF_SCHED_COLORED, max_sweeps=100000)["stats"]["sweeps"]
        par += mf.solve_instance(inst, max_sweeps=100000)["stats"]["sweeps"]
    print(f"colour phases {col} sweeps, parallel {par} sweeps", flush=True)
    assert col < par


@pytest.mark.parametrize("seed", range(4))
def test_colored_prd_exact(mf, seed):
    """S-PRD: push-relabel region discharge under the colour phases."""
    dims, conn, tile = CASES[seed]
    inst = synth.random_grid(dims, conn, 4200 + seed, tile=tile)
    ref = oracle.solve_grid(inst)
    out = mf.solve_instance(inst, schedule=mf.MF_SCHED_COLORED, method=mf.MF_METHOD_PRD,
                            max_sweeps=1000000)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()


def test_colored_graph_replay_matches_eager(mf):
    inst = synth.blob_grid((256, 192), 8, 4300, 8, 8.0, 30.0, zero_frac=0.1, tile=(32, 32))
    ref = oracle.solve_grid(inst)
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        eager = g.solve(schedule=mf.MF_SCHED_COLORED, max_sweeps=2000)
        assert g.flow_value() == ref["flow"]
        for rep in range(3):
            st = g.solve(schedule=mf.MF_SCHED_COLORED, graph=True, check_every=2, max_sweeps=2000,
                         global_relabel_every=0)
            print(f"replay {rep}: sweeps {st['sweeps']} (eager {eager['sweeps']})", flush=True)
            assert g.flow_value() == ref["flow"]
            assert (g.min_cut(mf.MF_CUT_MIN_SOURCE) == ref["smin"]).all()
            g.solve(max_sweeps=2000)  # the parallel driver in between
            assert g.flow_value() == ref["flow"]


def test_colored_batch_exact(mf):
    insts = synth.config3_instances(32)
    b = mf.load_batch(insts, region_shape=(32, 32))
    try:
        b.solve(schedule=mf.MF_SCHED_COLORED, max_sweeps=100000)
        flows = b.flow_values()
        for i, inst in enumerate(insts):
            ref = oracle.solve_grid(inst)
            assert flows[i] == ref["flow"], (i, inst.name)
            assert (b.instance_cut(i, mf.MF_CUT_MIN_SOURCE) == ref["smin"]).all(), (i, inst.name)
    finally:
        b.close()


def test_colored_full_size_2048_exact(mf):
    inst = synth.config(1)
    out = mf.solve_instance(inst, schedule=mf.MF_SCHED_COLORED, global_relabel_every=10,
                            max_sweeps=100000)
    ref = oracle.solve_grid(inst)
    print(f"{inst.name}: colour-phase sweeps {out['stats']['sweeps']}", flush=True)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()


def test_colored_rejected_combinations(mf):
    inst = synth.random_grid((16, 16), 4, 4400, tile=(8, 8))
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        for kw in (dict(boundary_relabel=4),):
            with pytest.raises(mf.MFError) as e:
                g.solve(schedule=mf.MF_SCHED_COLORED, **kw)
            assert e.value.status == mf.MF_E_INVAL, kw
        st = g.solve(schedule=mf.MF_SCHED_COLORED)
        assert st["sweeps"] >= 1


@pytest.mark.parametrize("seed", range(6))
def test_colored_partial_exact(mf, seed):
    """Partial discharges under the colour phases: sweep s (one phase per colour)
    runs the stages k <= s."""
    cases = [((12, 13), 4, (4, 5)), ((6, 7, 8), 6, (3, 4, 4)), ((40, 36), 8, (8, 8)),
             ((8, 40, 70), 6, (4, 16, 32)), ((70, 90), 8, (32, 32)), ((9, 10, 11), 6, (4, 4, 4))]
    dims, conn, tile = cases[seed]
    inst = synth.blob_grid(dims, conn, 4500 + seed, 4, 3.0, 9.0, zero_frac=0.1, tile=tile)
    ref = oracle.solve_grid(inst)
    for relabel in (0, 4):
        out = mf.solve_instance(inst, schedule=mf.MF_SCHED_COLORED, partial=True,
                                global_relabel_every=relabel, max_sweeps=100000)
        assert out["flow"] == ref["flow"]
        assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()
        certify_solver_state(inst, out)


def test_colored_partial_full_size_256_exact(mf):
    inst = synth.config(2)
    out = mf.solve_instance(inst, schedule=mf.MF_SCHED_COLORED, partial=True,
                            global_relabel_every=4, max_sweeps=100000)
    ref = oracle.solve_grid(inst)
    print(f"{inst.name}: colour-phase sweeps {out['stats']['sweeps']}", flush=True)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()


@pytest.mark.parametrize("defer_mode", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_colored_learned_exact(mf, seed, defer_mode):
    """The learned schedule driving the colour phases (phase order by predicted
    progress, deferrals inside a phase), with an untrained network: arbitrary
    scores, same exact result."""
    cases = [((40, 36), 8, (8, 8)), ((9, 10, 11), 6, (4, 4, 4)), ((8, 40, 70), 6, (4, 16, 32)),
             ((100, 90), 4, (32, 32))]
    dims, conn, tile = cases[seed]
    inst = synth.random_grid(dims, conn, 4600 + seed, tile=tile)
    ref = oracle.solve_grid(inst)
    model = mf.Model(16, seed=seed)
    for partial in (False, True):
        out = mf.solve_instance(inst, schedule=mf.MF_SCHED_LEARNED_COLORED, model=model,
                                defer_threshold=0.6, max_defer=2, defer_mode=defer_mode,
                                partial=partial, max_sweeps=100000)
        assert out["flow"] == ref["flow"]
        assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()


def test_colored_trace_records_sweeps(mf):
    """Per-discharge trace records carry the sweep (one phase per colour), and
    every region is discharged at most once per sweep."""
    import torch
    inst = synth.random_grid((48, 40), 8, 4700, tile=(8, 8))
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        tr = torch.zeros((100000, mf.TRACE_FIELDS), dtype=torch.int32, device="cuda")
        st = g.solve(schedule=mf.MF_SCHED_COLORED, trace=tr, max_sweeps=100000)
        rec = tr[:min(st["trace_records"], tr.shape[0])].cpu().numpy()
        assert rec[:, 0].max() == st["sweeps"] - 1
        pairs = rec[:, 0].astype(np.int64) * 1000003 + rec[:, 1]
        assert len(np.unique(pairs)) == len(pairs)
