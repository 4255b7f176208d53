"""Partial discharges on the GPU (Sec. 6.2: sweep s runs only the stages k <= s
of Proc. ARD): the flow and both extremal cuts stay the oracle's on every region
kernel, schedule and launch mode, and the first sweep augments to the sink only
(checked per discharge from the trace against region-wise textbook max flows)."""
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


def _check(mf, inst, tile=None, **kw):
    tile = tuple(tile if tile is not None else inst.tile)
    print(f"case {inst.name} dims={inst.dims} conn={inst.conn} tile={tile} {kw}", flush=True)
    out = mf.solve_instance(inst, tile=tile, max_sweeps=100000, partial=True, **kw)
    ref = oracle.solve_grid(inst)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all()
    assert (out["smax"] == ref["smax"]).all()
    certify_solver_state(inst, out)
    return out


CASES = [
    ((12, 13), 4, (4, 5)), ((16, 16), 8, (8, 8)), ((9, 20), 4, (3, 7)),
    ((6, 7, 8), 6, (3, 4, 4)), ((33, 31), 8, (16, 16)), ((40, 17), 4, (32, 8)),
    ((5, 9, 13), 6, (5, 4, 6)), ((64, 64), 8, (64, 64)), ((20, 20), 4, (1, 1)),
    ((3, 3, 3), 6, (1, 1, 1)), ((70, 90), 8, (32, 32)), ((130, 70), 4, (64, 64)),
]


@pytest.mark.parametrize("kernel", ["auto", "hbm", "lds"])
@pytest.mark.parametrize("seed", range(24))
def test_partial_random_grids_exact(mf, seed, kernel):
    dims, conn, tile = CASES[seed % len(CASES)]
    inst = synth.random_grid(dims, conn, 900 + seed, tile=tile)
    rk = {"auto": mf.MF_KERNEL_AUTO, "hbm": mf.MF_KERNEL_HBM, "lds": mf.MF_KERNEL_LDS}[kernel]
    _check(mf, inst, region_kernel=rk)


ROWS_TILES = [(2, 32, 32), (4, 16, 32), (8, 8, 32), (32, 2, 32), (4, 32, 32)]


@pytest.mark.parametrize("seed", range(10))
def test_partial_rows_kernel_exact(mf, seed):
    tile = ROWS_TILES[seed % len(ROWS_TILES)]
    dims = tuple(int(t * m + e) for t, m, e in zip(tile, (2, 2, 1), (seed % 3, 1, 7)))
    if seed % 2:
        inst = synth.blob_grid(dims, 6, 950 + seed, 4, 3.0, 8.0, tile=tile)
    else:
        inst = synth.random_grid(dims, 6, 950 + seed, tile=tile)
    out = _check(mf, inst, region_kernel=mf.MF_KERNEL_ROWS)
    assert out["stats"]["region_kernel"] == mf.MF_KERNEL_ROWS


@pytest.mark.parametrize("seed", range(10))
def test_partial_wave_kernel_exact(mf, seed):
    tiles = [(64, 64), (32, 64), (48, 40), (64, 16), (7, 64)]
    tile = tiles[seed % len(tiles)]
    dims = (tile[0] * 3 + seed, tile[1] * 2 + 5)
    conn = 8 if seed % 2 else 4
    inst = synth.blob_grid(dims, conn, 970 + seed, 6, 6.0, 20.0, zero_frac=0.1, tile=tile)
    out = _check(mf, inst, region_kernel=mf.MF_KERNEL_WAVE)
    assert out["stats"]["region_kernel"] == mf.MF_KERNEL_WAVE


def _region_flow_sum(inst, tile):
    """Sum over regions of the max flow of the region alone (inner pairs and its
    t-links, pairs to other regions dropped), by the textbook solver."""
    pu, pv, cuv, cvu = oracle.grid_pairs(inst.dims, inst.nbr, oracle._offsets(inst))
    region = oracle.grid_regions(inst.dims, tile)
    total = 0
    for rk in np.unique(region):
        vs = np.flatnonzero(region == rk)
        idx = -np.ones(inst.n, np.int64)
        idx[vs] = np.arange(len(vs))
        keep = (region[pu] == rk) & (region[pv] == rk)
        total += oracle.solve_pairs(len(vs), idx[pu[keep]], idx[pv[keep]], cuv[keep], cvu[keep],
                                    inst.cs[vs], inst.ct[vs])["flow"]
    return total


# trace record fields (include/mf.h, MF_TR_*)
TR_SWEEP, TR_TO_SINK, TR_TO_BOUNDARY = 0, 7, 8

FIRST_SWEEP_CASES = [
    ("wave", (96, 80), 8, (32, 32)), ("wave", (70, 64), 4, (64, 16)),
    ("rows", (8, 40, 70), 6, (4, 16, 32)), ("lds", (40, 36), 8, (8, 8)),
    ("hbm", (9, 10, 11), 6, (4, 4, 4)), ("hbm", (33, 31), 8, (16, 16)),
]


@pytest.mark.parametrize("case", range(len(FIRST_SWEEP_CASES)))
def test_partial_first_sweep_augments_to_sink_only(mf, case):
    """Sweep 0 with partial discharges: no discharge pushes over a boundary arc,
    and the flow the discharges send to t is the sum of the regions' own max
    flows (textbook solver per region).  Without the cap some flow crosses."""
    import torch
    kname, dims, conn, tile = FIRST_SWEEP_CASES[case]
    rk = {"wave": mf.MF_KERNEL_WAVE, "rows": mf.MF_KERNEL_ROWS, "lds": mf.MF_KERNEL_LDS,
          "hbm": mf.MF_KERNEL_HBM}[kname]
    inst = synth.random_grid(dims, conn, 990 + case, tile=tile)
    want = _region_flow_sum(inst, tile)
    crossed = {}
    with mf.Grid(inst.dims, inst.conn, tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        for partial in (True, False):
            tr = torch.zeros((200000, mf.TRACE_FIELDS), dtype=torch.int32, device="cuda")
            st = g.solve(trace=tr, partial=partial, region_kernel=rk, max_sweeps=100000)
            assert st["region_kernel"] == rk
            rec = tr[:min(st["trace_records"], tr.shape[0])].cpu().numpy().astype(np.int64)
            first = rec[rec[:, TR_SWEEP] == 0]
            crossed[partial] = int(first[:, TR_TO_BOUNDARY].sum())
            if partial:
                assert crossed[True] == 0
                assert int(first[:, TR_TO_SINK].sum()) == want
    assert crossed[False] > 0


@pytest.mark.parametrize("defer_mode", [0, 1])
@pytest.mark.parametrize("seed", range(4))
def test_partial_with_learned_schedule_exact(mf, seed, defer_mode):
    cases = [((40, 36), 8, (8, 8)), ((9, 10, 11), 6, (4, 4, 4)), ((8, 40, 70), 6, (4, 16, 32)),
             ((100, 90), 4, (32, 32))]
    dims, conn, tile = cases[seed]
    inst = synth.random_grid(dims, conn, 1010 + seed, tile=tile)
    model = mf.Model(16, seed=seed)  # untrained: arbitrary scores and deferrals
    _check(mf, inst, schedule=mf.MF_SCHED_LEARNED, model=model, defer_threshold=0.6,
           max_defer=2, defer_mode=defer_mode)


def test_partial_graph_replay_matches_eager(mf):
    """Captured sweep batches read the stage cap from the device sweep counter
    (a cap captured as the launch's sweep index would stay below 4 on every
    replay: flow beyond stage 3 would never move and the sweep limit would end
    the solve with an error)."""
    inst = synth.blob_grid((256, 192), 8, 1020, 8, 8.0, 30.0, zero_frac=0.1, tile=(32, 32))
    ref = oracle.solve_grid(inst)
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        eager = g.solve(partial=True, max_sweeps=2000)
        assert g.flow_value() == ref["flow"]
        for rep in range(3):
            st = g.solve(partial=True, graph=True, check_every=4, max_sweeps=2000)
            print(f"replay {rep}: sweeps {st['sweeps']} (eager {eager['sweeps']})", flush=True)
            assert g.flow_value() == ref["flow"]
            assert (g.min_cut(mf.MF_CUT_MIN_SOURCE) == ref["smin"]).all()
            g.solve(max_sweeps=2000)  # eager, full discharges, in between
            assert g.flow_value() == ref["flow"]


def test_partial_batch_exact(mf):
    insts = synth.config3_instances(40)
    b = mf.load_batch(insts, region_shape=(32, 32))
    try:
        b.solve(partial=True, max_sweeps=100000)
        flows = b.flow_values()
        for i, inst in enumerate(insts):
            ref = oracle.solve_grid(inst)
            assert flows[i] == ref["flow"], (i, inst.name)
            assert (b.instance_cut(i, mf.MF_CUT_MIN_SOURCE) == ref["smin"]).all(), (i, inst.name)
    finally:
        b.close()


@pytest.mark.parametrize("cfg,relabel", [(1, 10), (2, 4)])
def test_full_size_partial_exact(mf, cfg, relabel):
    inst = synth.config(cfg)
    out = mf.solve_instance(inst, max_sweeps=100000, partial=True, global_relabel_every=relabel)
    ref = oracle.solve_grid(inst)
    print(f"{inst.name} partial sweeps {out['stats']['sweeps']} solve_ms {out['stats']['solve_ms']:.1f}",
          flush=True)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()
