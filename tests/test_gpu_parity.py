"""GPU parity: the HIP solver (through the C ABI) against the CPU oracle.

Bar: the int64 flow value and both extremal minimum cuts are identical to the
oracle's on every seeded input; the solver's final residual state is a feasible
preflow whose cuts cost exactly the flow (certificate from the original caps).
"""
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


def _check(mf, inst, tile=None, certify=True, **kw):
    tile = tuple(tile if tile is not None else inst.tile)
    print(f"case {inst.name} dims={inst.dims} conn={inst.conn} tile={tile}", flush=True)
    out = mf.solve_instance(inst, tile=tile, max_sweeps=kw.pop("max_sweeps", 100000), **kw)
    ref = oracle.solve_grid(inst)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all()
    assert (out["smax"] == ref["smax"]).all()
    if certify:
        certify_solver_state(inst, out)
    return out, ref


def test_workload0_exact(mf):
    inst = synth.config(0)
    out, ref = _check(mf, inst)
    assert out["info"]["boundary_size"] == 252
    assert out["stats"]["sweeps"] <= 2 * 252 ** 2 + 1


RANDOM_CASES = [
    ((12, 13), 4, (4, 5)), ((16, 16), 8, (8, 8)), ((9, 20), 4, (3, 7)),
    ((6, 7, 8), 6, (3, 4, 4)), ((33, 31), 8, (16, 16)), ((40, 17), 4, (32, 8)),
    ((5, 9, 13), 6, (5, 4, 6)), ((64, 64), 8, (64, 64)), ((20, 20), 4, (1, 1)),
    ((1, 50), 4, (1, 7)), ((50, 1), 8, (9, 1)), ((3, 3, 3), 6, (1, 1, 1)),
]


@pytest.mark.parametrize("kernel", ["auto", "hbm", "lds"])
@pytest.mark.parametrize("seed", range(48))
def test_random_grids_exact(mf, seed, kernel):
    dims, conn, tile = RANDOM_CASES[seed % len(RANDOM_CASES)]
    inst = synth.random_grid(dims, conn, seed, tile=tile)
    rk = {"auto": mf.MF_KERNEL_AUTO, "hbm": mf.MF_KERNEL_HBM, "lds": mf.MF_KERNEL_LDS}[kernel]
    out, _ = _check(mf, inst, region_kernel=rk)
    B = out["info"]["boundary_size"]
    assert out["stats"]["sweeps"] <= 2 * max(B, 1) ** 2 + 1


@pytest.mark.parametrize("every", [1, 3])
@pytest.mark.parametrize("seed", range(12))
def test_global_relabel_exact(mf, seed, every):
    """Exact region-distance relabels between sweeps change the path, never the result."""
    dims, conn, tile = RANDOM_CASES[seed % len(RANDOM_CASES)]
    inst = synth.random_grid(dims, conn, 500 + seed, tile=tile)
    out, _ = _check(mf, inst, global_relabel_every=every)
    assert out["stats"]["global_relabels"] >= 1


@pytest.mark.parametrize("seed", range(6))
def test_lds_kernel_int32_residuals(mf, seed):
    """Capacities too large for int16 residuals select the int32 LDS layout."""
    inst = synth.random_grid((40, 36), 8 if seed % 2 else 4, 100 + seed, tile=(16, 16))
    inst.nbr = (inst.nbr.astype(np.int64) * 7000).astype(np.int32)
    _check(mf, inst, region_kernel=mf.MF_KERNEL_LDS)


@pytest.mark.parametrize("strength", [5, 40, 150, 400])
def test_paper_synthetic_family_exact(mf, strength):
    for seed in range(2):
        inst = synth.paper_e1_grid((100, 100), 8, seed, strength, tile=(25, 25))
        _check(mf, inst)


def test_partition_invariance(mf):
    inst = synth.blob_grid((96, 80), 8, 7, 4, 6.0, 12.0, zero_frac=0.1)
    outs = []
    for tile in [(96, 80), (32, 32), (16, 40), (7, 9), (64, 1)]:
        o, _ = _check(mf, inst, tile=tile)
        outs.append(o)
    for o in outs[1:]:
        assert o["flow"] == outs[0]["flow"]
        assert (o["smin"] == outs[0]["smin"]).all() and (o["smax"] == outs[0]["smax"]).all()


def test_degenerate_inputs(mf):
    # all capacities zero: flow 0, minimal source side empty, maximal all of V
    z = synth.random_grid((10, 12), 4, 1, tile=(4, 4))
    z.cs[:] = 0
    z.ct[:] = 0
    z.nbr[:] = 0
    out, _ = _check(mf, z)
    assert out["flow"] == 0 and out["smin"].sum() == 0 and out["smax"].all()
    # no n-links: closed form
    nl = synth.config(0)
    nl.nbr[:] = 0
    out, _ = _check(mf, nl)
    assert out["flow"] == int(np.minimum(nl.cs.astype(np.int64), nl.ct).sum())
    # a single vertex
    one = synth.random_grid((1, 1), 4, 2, tile=(1, 1))
    one.cs[:] = 5
    one.ct[:] = 3
    out, _ = _check(mf, one)
    assert out["flow"] == 3
    # only sources / only sinks
    src = synth.random_grid((17, 9), 8, 3, tile=(8, 8))
    src.ct[:] = 0
    out, _ = _check(mf, src)
    assert out["flow"] == 0
    snk = synth.random_grid((17, 9), 8, 4, tile=(8, 8))
    snk.cs[:] = 0
    out, _ = _check(mf, snk)
    assert out["flow"] == 0 and out["smin"].sum() == 0


def test_large_capacities(mf):
    """Capacities near the int32 limits allowed by the overflow rule."""
    inst = synth.random_grid((24, 24), 4, 9, tile=(8, 8), cap_hi=10)
    # c_s(v) + inflow capacity stays below 2^31: 20*20M + 4*10*25M = 1.4e9
    inst.nbr = (inst.nbr.astype(np.int64) * 25_000_000).astype(np.int32)
    inst.cs = (inst.cs.astype(np.int64) * 20_000_000).astype(np.int32)
    inst.ct = (inst.ct.astype(np.int64) * 20_000_000).astype(np.int32)
    _check(mf, inst)


@pytest.mark.parametrize("case", ["u8_limits", "i16_pairs", "i16_inflow"])
def test_wave_kernel_storage_modes(mf, case):
    """The wavefront kernel's LDS widths at their limits: 8-bit residuals with
    16-bit excess (pair sum 255, t-link 255, inflow bound up to 32767, excess
    near the int16 limit), and 16-bit residuals chosen for pair sums above 255
    or inflow bounds above 32767."""
    rng = np.random.default_rng(77)
    dims, tile = (40, 50), (16, 16)
    if case == "u8_limits":
        inst = synth.random_grid(dims, 8, 21, tile=tile, cap_hi=127, tlink_hi=255)
        v = 5 * dims[1] + 7  # one pair with sum exactly 255 (+x arc and its reverse)
        inst.nbr[0][v], inst.nbr[1][v + 1] = 128, 127
        # large source links on a few vertices: c(s,v) + sum_u c(u,v) <= 32767
        # (8 arcs of at most 128 each), so excess gets close to the int16 limit
        pick = rng.choice(inst.n, 12, replace=False)
        inst.cs[pick] = 32767 - 8 * 128
    elif case == "i16_pairs":
        inst = synth.random_grid(dims, 8, 22, tile=tile, cap_hi=1000, tlink_hi=300)
    else:
        inst = synth.random_grid(dims, 8, 23, tile=tile, cap_hi=100, tlink_hi=200)
        inst.cs[rng.choice(inst.n, 20, replace=False)] = 40000
    _check(mf, inst, region_kernel=mf.MF_KERNEL_WAVE)
    _check(mf, inst, region_kernel=mf.MF_KERNEL_WAVE, global_relabel_every=2)


@pytest.mark.parametrize("cfg", [1, 2])
def test_full_size_workloads_exact(mf, cfg):
    inst = synth.config(cfg)
    _check(mf, inst, certify=(cfg == 1))


@pytest.mark.parametrize("kernel", ["hbm", "lds"])
def test_workload1_other_kernels_exact(mf, kernel):
    inst = synth.config(1)
    rk = {"hbm": mf.MF_KERNEL_HBM, "lds": mf.MF_KERNEL_LDS}[kernel]
    _check(mf, inst, certify=False, region_kernel=rk)


@pytest.mark.parametrize("seed", range(16))
def test_wave_kernel_tiles(mf, seed):
    """The wavefront kernel on 2D tiles of every width/height up to 64, ragged grids."""
    rng = np.random.default_rng(seed)
    tile = (int(rng.integers(1, 65)), int(rng.integers(1, 65)))
    dims = (int(rng.integers(1, 3 * tile[0] + 2)), int(rng.integers(1, 3 * tile[1] + 2)))
    conn = 4 if seed % 2 else 8
    inst = synth.random_grid(dims, conn, 900 + seed, tile=tile, cap_hi=30)
    _check(mf, inst, region_kernel=mf.MF_KERNEL_WAVE)


ROWS_TILES = [(2, 32, 32), (4, 16, 32), (8, 8, 32), (16, 4, 32), (32, 2, 32), (32, 32, 32), (4, 32, 32)]


@pytest.mark.parametrize("seed", range(21))
def test_rows_kernel_tiles(mf, seed):
    """The row-bitmask workgroup kernel on 3D tiles with 32-vertex rows and every
    admissible row count, ragged grids, random and blob capacities."""
    rng = np.random.default_rng(seed)
    tile = ROWS_TILES[seed % len(ROWS_TILES)]
    dims = tuple(int(rng.integers(t, 2 * t + 3)) for t in tile)  # tiles are clamped to the grid
    if seed % 3 == 2:
        inst = synth.blob_grid(dims, 6, 1300 + seed, 4, 2.0, 6.0, tile=tile, name=f"rows_blob_{seed}")
    else:
        inst = synth.random_grid(dims, 6, 1200 + seed, tile=tile, cap_hi=20 if seed % 2 else 10)
    out, _ = _check(mf, inst, region_kernel=mf.MF_KERNEL_ROWS)
    B = out["info"]["boundary_size"]
    assert out["stats"]["sweeps"] <= 2 * max(B, 1) ** 2 + 1
    _check(mf, inst, region_kernel=mf.MF_KERNEL_ROWS, global_relabel_every=2)


def test_64_cubed_regions_auto_and_hbm(mf):
    """64^3 regions (the tile of the 464^3 workload): the default picks the
    64-vertex-row kernel; the HBM kernel gives the same result; ragged grid."""
    inst = synth.blob_grid((96, 100, 130), 6, 31, 6, 6.0, 20.0, tile=(64, 64, 64), name="blob3d_t64")
    out, _ = _check(mf, inst, certify=False)
    assert out["stats"]["region_kernel"] == mf.MF_KERNEL_ROWS64
    _check(mf, inst, certify=False, global_relabel_every=4)
    out, _ = _check(mf, inst, certify=False, region_kernel=mf.MF_KERNEL_HBM)
    assert out["stats"]["region_kernel"] == mf.MF_KERNEL_HBM


@pytest.mark.parametrize("case", range(6))
def test_hbm_kernel_large_regions_1024_threads(mf, case):
    """Regions of 8K vertices and more run the HBM kernel with 1024-thread
    workgroups: 2D 128x128 and 256x256, 3D 24^3 and 64^3 tiles, ragged, with
    partial discharges, the exact relabel and the boundary relabel."""
    cases = [((300, 280), 8, (256, 256), {}), ((270, 513), 4, (256, 256), dict(partial=True)),
             ((70, 66, 130), 6, (64, 64, 64), dict(partial=True, global_relabel_every=4)),
             ((65, 128, 64), 6, (64, 64, 64), dict(boundary_relabel=16)),
             ((300, 250), 8, (128, 128), dict(global_relabel_every=6)),
             ((50, 49, 60), 6, (24, 24, 24), dict(partial=True))]
    dims, conn, tile, kw = cases[case]
    inst = synth.blob_grid(dims, conn, 3100 + case, 6, 6.0, 24.0, zero_frac=0.1, tile=tile)
    out, _ = _check(mf, inst, certify=(case < 2), region_kernel=mf.MF_KERNEL_HBM, **kw)
    assert out["stats"]["region_kernel"] == mf.MF_KERNEL_HBM


def test_full_size_464_certified(mf):
    """The 464^3 workload (10^8 vertices, 64^3 regions): the flow and both cuts
    equal the oracle's result on the whole instance (stored: the oracle takes
    minutes and tens of GB for it), and the state is certified at full size from
    the original capacities: residuals feasible, conservation, flow = sum (c_t -
    r_t), both returned cuts of cost equal to the flow (max-flow/min-cut
    duality, Sec. 2), and both cuts equal to the oracle's residual reachability
    on the returned state."""
    import time
    t0 = time.perf_counter()
    inst = synth.config(4)
    out = mf.solve_instance(inst, global_relabel_every=4, max_sweeps=100000)
    print(f"{inst.name}: flow {out['flow']} sweeps {out['stats']['sweeps']} "
          f"({time.perf_counter() - t0:.0f} s with the generator)", flush=True)
    assert out["stats"]["region_kernel"] == mf.MF_KERNEL_ROWS64
    # the oracle's result on the whole instance, stored by tests/golden/make_grid3d6_464.py
    import hashlib
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "grid3d6_464_oracle.json")) as f:
        ref = json.load(f)
    assert out["flow"] == ref["flow"]
    assert hashlib.sha256(out["smin"].astype(np.uint8).tobytes()).hexdigest() == ref["smin_sha256"]
    assert hashlib.sha256(out["smax"].astype(np.uint8).tobytes()).hexdigest() == ref["smax_sha256"]
    certify_solver_state(inst, out)
    print(f"certified ({time.perf_counter() - t0:.0f} s)", flush=True)


def test_workload2_hbm_kernel_exact(mf):
    inst = synth.config(2)
    _check(mf, inst, certify=False, region_kernel=mf.MF_KERNEL_HBM)


def test_rows_kernel_selection(mf):
    """ROWS needs 3D tiles with 32-vertex rows; it is the default where it applies."""
    inst = synth.random_grid((10, 20, 40), 6, 5, tile=(4, 16, 32))
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        g.solve(region_kernel=mf.MF_KERNEL_ROWS)
    for dims, conn, tile in (((64, 64), 8, (32, 32)), ((8, 8, 40), 6, (8, 8, 16)), ((8, 8, 40), 6, (3, 8, 32))):
        inst = synth.random_grid(dims, conn, 6, tile=tile)
        with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
            g.set_caps(inst.cs, inst.ct, inst.nbr)
            with pytest.raises(mf.MFError) as e:
                g.solve(region_kernel=mf.MF_KERNEL_ROWS)
            assert e.value.status == mf.MF_E_INVAL


@pytest.mark.parametrize("cfg", [1, 2])
def test_full_size_global_relabel_exact(mf, cfg):
    inst = synth.config(cfg)
    _check(mf, inst, certify=False, global_relabel_every=4)


def test_region_kernel_selection_errors(mf):
    inst = synth.config(2)  # 32^3 regions do not fit in LDS and are not 2D
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        for rk in (mf.MF_KERNEL_LDS, mf.MF_KERNEL_WAVE):
            with pytest.raises(mf.MFError) as e:
                g.solve(region_kernel=rk)
            assert e.value.status == mf.MF_E_INVAL


def test_resolve_and_device_inputs(mf):
    torch = pytest.importorskip("torch")
    a = synth.random_grid((30, 40), 8, 21, tile=(16, 16))
    b = synth.random_grid((30, 40), 8, 22, tile=(16, 16))
    ra, rb = oracle.solve_grid(a), oracle.solve_grid(b)
    with mf.Grid(a.dims, a.conn, a.tile) as g:
        dev = [torch.from_numpy(x).cuda() for x in (a.cs, a.ct, a.nbr)]
        g.set_caps(*dev)
        g.solve()
        assert g.flow_value() == ra["flow"]
        g.solve()  # solve the same instance again from Init
        assert g.flow_value() == ra["flow"]
        g.set_caps(b.cs, b.ct, b.nbr)
        g.solve()
        assert g.flow_value() == rb["flow"]
        assert (g.min_cut(mf.MF_CUT_MIN_SOURCE) == rb["smin"]).all()
        s = torch.cuda.Stream()
        g.set_caps(*[torch.from_numpy(x).cuda() for x in (a.cs, a.ct, a.nbr)], stream=s.cuda_stream)
        g.solve(stream=s.cuda_stream)
        assert g.flow_value() == ra["flow"]


def test_abi_errors(mf):
    inst = synth.random_grid((8, 8), 4, 0, tile=(4, 4))
    with mf.Grid(inst.dims, 4, (4, 4)) as g:
        with pytest.raises(mf.MFError) as e:
            g.solve()
        assert e.value.status == mf.MF_E_STATE
        with pytest.raises(mf.MFError) as e:
            g.flow_value()
        assert e.value.status == mf.MF_E_STATE
        bad = inst.cs.copy()
        bad[3] = -1
        with pytest.raises(mf.MFError) as e:
            g.set_caps(bad, inst.ct, inst.nbr)
        assert e.value.status == mf.MF_E_INVAL
        nb = inst.nbr.copy()
        nb[0, 7] = 5  # +x arc of the last vertex of row 0 leaves the grid
        with pytest.raises(mf.MFError) as e:
            g.set_caps(inst.cs, inst.ct, nb)
        assert e.value.status == mf.MF_E_INVAL
        with pytest.raises(mf.MFError) as e:
            g.solve()  # a failed set_caps leaves no instance
        assert e.value.status == mf.MF_E_STATE
        ov = inst.nbr.copy()
        ov[0, 0] = 2**31 - 1
        ov[1, 1] = 5
        with pytest.raises(mf.MFError) as e:
            g.set_caps(inst.cs, inst.ct, ov)
        assert e.value.status == mf.MF_E_OVERFLOW
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        g.solve()
        with pytest.raises(mf.MFError) as e:
            g.min_cut(7)
        assert e.value.status == mf.MF_E_INVAL
    with pytest.raises(mf.MFError):
        mf.Grid((8, 8), 6)
    with pytest.raises(mf.MFError):
        mf.Grid((8, 8, 8), 4)


# ---------------------------------------------------------------------------
# Batches (independent instances in one solve)
# ---------------------------------------------------------------------------

def _batch_check(mf, insts, region_shape, **kw):
    b = mf.load_batch(insts, region_shape=region_shape)
    try:
        st = b.solve(max_sweeps=100000, **kw)
        flows = b.flow_values()
        for i, inst in enumerate(insts):
            ref = oracle.solve_grid(inst)
            assert flows[i] == ref["flow"], (i, inst.name)
            assert (b.instance_cut(i, mf.MF_CUT_MIN_SOURCE) == ref["smin"]).all(), (i, inst.name)
            assert (b.instance_cut(i, mf.MF_CUT_MAX_SOURCE) == ref["smax"]).all(), (i, inst.name)
        assert b.flow_value() == int(flows.sum())
    finally:
        b.close()
    return st


@pytest.mark.parametrize("tile", [(16, 16), (32, 32), (64, 64), (24, 40)])
def test_batch_mixed_instances_exact(mf, tile):
    rng = np.random.default_rng(7)
    insts = []
    for i in range(30):
        dims = (int(rng.integers(1, 140)), int(rng.integers(1, 140)))
        if i % 3 == 0:
            insts.append(synth.random_grid(dims, 4 if i % 2 else 8, 2000 + i))
        else:
            insts.append(synth.blob_grid(dims, 4 if i % 2 else 8, 2000 + i, 3, 6.0, 6.0))
    print(f"batch of {len(insts)} tile={tile}", flush=True)
    _batch_check(mf, insts, tile)


def test_batch_graph_replay_matches_eager(mf):
    insts = synth.config3_instances(24)
    b = mf.load_batch(insts, region_shape=(32, 32))
    try:
        b.solve()
        eager = b.flow_values().copy()
        cut = b.instance_cut(5)
        for rep in range(3):  # replays of the captured sweep batches, eager work in between
            b.solve(graph=True, global_relabel_every=2 * rep)
            assert (b.flow_values() == eager).all()
            assert (b.instance_cut(5) == cut).all()
            b.solve()
            assert (b.flow_values() == eager).all()
    finally:
        b.close()


def test_batch_single_connectivity_and_errors(mf):
    insts = [synth.random_grid((9, 13), 4, 30 + i) for i in range(5)]
    _batch_check(mf, insts, (8, 8))
    b = mf.Batch([(9, 13)] * 2, [4, 4], (8, 8))
    try:
        b.set_caps(0, insts[0].cs, insts[0].ct, insts[0].nbr)
        with pytest.raises(mf.MFError) as e:
            b.solve()  # instance 1 not loaded
        assert e.value.status == mf.MF_E_STATE
        bad = insts[1].cs.copy()
        bad[0] = -3
        with pytest.raises(mf.MFError) as e:
            b.set_caps(1, bad, insts[1].ct, insts[1].nbr)
        assert e.value.status == mf.MF_E_INVAL
        with pytest.raises(mf.MFError):
            load = mf.load()
            import ctypes
            rc = load.mf_set_caps(b._h, ctypes.c_void_p(insts[0].cs.ctypes.data),
                                  ctypes.c_void_p(insts[0].ct.ctypes.data),
                                  ctypes.c_void_p(insts[0].nbr.ctypes.data), 0, None)
            mf._check(rc, "mf_set_caps")
    finally:
        b.close()


def test_batch_workload_512_exact(mf):
    """All 512 instances of the batch workload, autotuned, each exact."""
    from paper_1109_1146_amd import autotune
    insts = synth.config3_instances(512)
    tune = autotune.autotune_batch(insts, calib=24, reps=1)
    print("autotuned", tune["region_shape"], tune["relabel_every"], tune["partial"],
          tune["boundary_relabel"], tune["schedule"], tune["region_kernel"], flush=True)
    # every dimension was searched: both schedules and both workgroup shapes were timed
    sub = [t for t in tune["timings"] if t["stage"] == "subset"]
    assert {t["schedule"] for t in sub} == {mf.MF_SCHED_PARD, mf.MF_SCHED_COLORED}
    assert {t["region_kernel"] for t in sub} == {mf.MF_KERNEL_WAVE, mf.MF_KERNEL_LDS}
    assert {t["round_cap"] for t in sub} == {0, 4}
    st = _batch_check(mf, insts, tune["region_shape"], global_relabel_every=tune["relabel_every"],
                      partial=tune["partial"], boundary_relabel=tune["boundary_relabel"],
                      schedule=tune["schedule"], region_kernel=tune["region_kernel"],
                      round_cap=tune["round_cap"], graph=True)
    assert st["sweeps"] > 0
    # the other schedule and workgroup shape are exact too
    other = dict(schedule=mf.MF_SCHED_COLORED if tune["schedule"] == mf.MF_SCHED_PARD else mf.MF_SCHED_PARD,
                 region_kernel=mf.MF_KERNEL_LDS if tune["region_kernel"] == mf.MF_KERNEL_WAVE
                 else mf.MF_KERNEL_WAVE)
    _batch_check(mf, insts[:128], tune["region_shape"], global_relabel_every=tune["relabel_every"],
                 partial=tune["partial"], graph=True, **other)


SERPENTINE_CASES = [
    ((40, 48), 8, (8, 8)),        # wave floods, a path through 30 regions
    ((37, 45), 4, (8, 16)),       # wave floods, ragged tiles
    ((8, 32, 64), 6, (4, 16, 32)),  # rows floods
    ((9, 10, 11), 6, (3, 4, 5)),  # queue floods (k_flood)
]


@pytest.mark.parametrize("case", range(len(SERPENTINE_CASES)))
def test_serpentine_path_many_flood_rounds(mf, case):
    """One residual path snaking across region borders: the flow has to cross
    every border along it, and the cut floods need one round per crossing."""
    from tests.helpers import serpentine_instance
    dims, conn, tile = SERPENTINE_CASES[case]
    inst, path = serpentine_instance(dims, conn, tile)
    out, ref = _check(mf, inst, certify=False)
    want = np.zeros(inst.n, np.uint8)
    want[path] = 1
    assert out["flow"] == 30 and (out["smin"] == want).all() and (out["smax"] == 1).all()
