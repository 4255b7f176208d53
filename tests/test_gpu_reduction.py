"""GPU parity of region reduction (Alg. 5, Sec. 8): the four class bits of every
vertex, byte for byte against the oracle, on random tilings in 2D and 3D with
every region kernel (against the oracle's Alg. 5 steps) and on the full-size
workloads 0-2 and a grid of 64^3 regions (against the oracle's all-regions
form of the same classes, which the CPU tests pin to Alg. 5)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_1109_1146_amd import mf as _mf
    _mf.load()
    return _mf


SMALL = [
    ((12, 13), 4, (4, 5), "AUTO"), ((16, 16), 8, (8, 8), "WAVE"), ((9, 20), 4, (3, 7), "HBM"),
    ((6, 7, 8), 6, (3, 4, 4), "LDS"), ((33, 31), 8, (16, 16), "LDS"), ((40, 17), 4, (32, 8), "AUTO"),
    ((5, 9, 13), 6, (5, 4, 6), "HBM"), ((8, 20, 40), 6, (4, 16, 32), "ROWS"),
    ((20, 20), 4, (20, 20), "AUTO"), ((64, 48), 8, (64, 16), "WAVE"), ((6, 6, 6), 6, (2, 2, 2), "LDS"),
    ((8, 24, 64), 6, (4, 16, 32), "ROWS"),
]


@pytest.mark.parametrize("seed", range(36))
def test_reduction_random_tilings(mf, seed):
    dims, conn, tile, kname = SMALL[seed % len(SMALL)]
    inst = (synth.blob_grid(dims, conn, 6000 + seed, 3, 2.0, 6.0, zero_frac=0.1, tile=tile)
            if seed % 3 == 2 else synth.random_grid(dims, conn, 6000 + seed, tile=tile))
    print(f"case {inst.name} dims={dims} tile={tile} kernel={kname}", flush=True)
    want = oracle.region_reduction(inst, tile)
    with mf.Grid(inst.dims, inst.conn, tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        got = g.region_reduction(getattr(mf, "MF_KERNEL_" + kname))
        # the reduction overwrote the solver state; a solve afterwards is exact
        with pytest.raises(mf.MFError) as e:
            g.flow_value()
        assert e.value.status == mf.MF_E_STATE
        g.solve()
        assert g.flow_value() == oracle.solve_grid(inst)["flow"]
    assert (got == want).all(), f"{int((got != want).sum())} vertices classified differently"


@pytest.mark.parametrize("cfg", [0, 1, 2])
def test_reduction_full_size_workloads(mf, cfg):
    inst = synth.config(cfg)
    print(f"case {inst.name} dims={inst.dims} tile={inst.tile}", flush=True)
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        got = g.region_reduction()
    want = oracle.region_reduction_union(inst, inst.tile)
    assert (got == want).all(), f"{int((got != want).sum())} vertices classified differently"
    if cfg == 0:
        assert (got == oracle.region_reduction(inst, inst.tile)).all()
    # the paper's measure of the reduction: decided = strong sink or weak source
    decided = ((got & (mf.MF_REDUCE_STRONG_SINK | mf.MF_REDUCE_WEAK_SOURCE)) > 0).mean()
    print(f"decided {100 * decided:.1f}%", flush=True)


def test_reduction_64_cubed_regions(mf):
    inst = synth.blob_grid((64, 64, 100), 6, 6100, 4, 4.0, 12.0, zero_frac=0.1, tile=(64, 64, 64))
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        got = g.region_reduction(mf.MF_KERNEL_ROWS64)
        got_hbm = g.region_reduction(mf.MF_KERNEL_HBM)
    want = oracle.region_reduction_union(inst, inst.tile)
    assert (got == want).all() and (got_hbm == want).all()
