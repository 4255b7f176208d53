"""Learned region scheduler on the GPU: gradient check of the HIP training
kernels against the FP64 CPU reference, BF16 inference against a bfloat16
reference at float32 tolerance, training
progress, and exactness of solves under learned (or arbitrary) scores."""
import numpy as np
import pytest

import oracle
import synth
from oracle import cnn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mf():
    from paper_1109_1146_amd import mf as _mf
    _mf.load()
    return _mf


def _rand_problem(rng, dims, C=16):
    p = rng.normal(scale=0.3, size=cnn.num_params(C)).astype(np.float32)
    x = rng.normal(size=dims + (6,)).astype(np.float32)
    t = (rng.uniform(size=dims) < 0.4).astype(np.float32)
    m = (rng.uniform(size=dims) < 0.7).astype(np.float32)
    return p, x, t, m


@pytest.mark.parametrize("dims", [(1, 32, 32), (8, 8, 8), (2, 5, 7)])
def test_gpu_gradients_match_fp64_reference(mf, dims):
    import torch
    rng = np.random.default_rng(3)
    p, x, t, m = _rand_problem(rng, dims)
    model = mf.Model(16)
    model.set_params(p)
    X = torch.from_numpy(x.reshape(-1, 6)).cuda()
    loss, g = model.loss_grad(X, torch.from_numpy(t.reshape(-1)).cuda(),
                              torch.from_numpy(m.reshape(-1)).cuda(), dims, want_grads=True)
    rl, rg = cnn.loss_and_grad(p.astype(np.float64), x.astype(np.float64), t, m, 16)
    assert abs(loss - rl) <= 1e-4 * max(1.0, abs(rl))
    scale = np.abs(rg).max()
    np.testing.assert_allclose(g, rg, rtol=0, atol=2e-4 * scale)


def test_gpu_forward_fp32_and_bf16(mf):
    import torch
    rng = np.random.default_rng(4)
    dims = (8, 8, 8)
    p, x, _, _ = _rand_problem(rng, dims)
    model = mf.Model(16)
    model.set_params(p)
    X = torch.from_numpy(x.reshape(-1, 6)).cuda()
    z32 = model.forward(X, dims, bf16=False).cpu().numpy()
    z16 = model.forward(X, dims, bf16=True).cpu().numpy()
    ref, _ = cnn.forward(p.astype(np.float64), x.astype(np.float64), 16)
    ref = ref.reshape(-1)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(z32, ref, rtol=0, atol=1e-4 * scale)
    # bf16: against the reference that rounds inputs, weights and every layer's
    # output to bfloat16 and sums in float32 (bias, taps, channels); products of
    # bfloat16 values are exact in float32, so only float32 rounding may differ
    ref16 = cnn.forward_bf16(p, x, 16).reshape(-1)
    np.testing.assert_allclose(z16, ref16, rtol=2e-6, atol=2e-6 * scale)
    print(f"bf16 logits equal to the reference: {int((z16 == ref16).sum())} of {z16.size}", flush=True)
    # and the bf16 path stays near the FP64 logits (8 significand bits, 3 layers)
    np.testing.assert_allclose(z16, ref, rtol=0, atol=5e-2 * scale)


def test_training_reduces_loss(mf):
    import torch
    rng = np.random.default_rng(5)
    dims = (1, 16, 16)
    x = rng.normal(size=dims + (6,)).astype(np.float32)
    t = (x[..., 0] + 0.5 * x[..., 2] > 0).astype(np.float32)  # a learnable rule
    m = np.ones(dims, np.float32)
    X = torch.from_numpy(x.reshape(-1, 6)).cuda()
    T = torch.from_numpy(t.reshape(-1)).cuda()
    M = torch.from_numpy(m.reshape(-1)).cuda()
    model = mf.Model(16, seed=1)
    first, _ = model.loss_grad(X, T, M, dims)
    for _ in range(150):
        loss, _ = model.loss_grad(X, T, M, dims)
        model.adam_step(3e-3)
    assert loss < 0.5 * first


def _exact(mf, inst, **kw):
    out = mf.solve_instance(inst, max_sweeps=100000, **kw)
    ref = oracle.solve_grid(inst)
    assert out["flow"] == ref["flow"]
    assert (out["smin"] == ref["smin"]).all() and (out["smax"] == ref["smax"]).all()
    return out


@pytest.mark.parametrize("threshold,max_defer", [(0.5, 2), (0.95, 1), (0.99, 4)])
@pytest.mark.parametrize("seed", range(6))
def test_learned_schedule_exact_with_arbitrary_scores(mf, seed, threshold, max_defer):
    """Whatever the network says, the flow and cuts are the oracle's."""
    cases = [((40, 36), 8, (8, 8)), ((30, 50), 4, (10, 16)), ((9, 10, 11), 6, (4, 4, 4)),
             ((8, 40, 70), 6, (4, 16, 32))]  # the last one runs the row-bitmask 3D kernel
    dims, conn, tile = cases[seed % len(cases)]
    inst = synth.random_grid(dims, conn, 700 + seed, tile=tile)
    model = mf.Model(16, seed=seed)  # untrained: arbitrary scores
    _exact(mf, inst, schedule=mf.MF_SCHED_LEARNED, model=model, defer_threshold=threshold,
           max_defer=max_defer)


def test_learned_schedule_needs_model(mf):
    inst = synth.random_grid((8, 8), 4, 1, tile=(4, 4))
    with mf.Grid(inst.dims, 4, (4, 4)) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        with pytest.raises(mf.MFError) as e:
            g.solve(schedule=mf.MF_SCHED_LEARNED)
        assert e.value.status == mf.MF_E_INVAL


def test_trained_network_gain_over_skeleton(mf):
    """Ablation: the same learned-schedule skeleton driven by the trained network
    vs by an untrained network (random weights), and plain P-ARD.  All three give
    the oracle's flow; the trained network defers fewer useful discharges than
    random scores (so it needs no more sweeps) and skips discharges plain P-ARD does."""
    from paper_1109_1146_amd import learned
    inst = synth.blob_grid((1024, 1024), 8, 7, 24, 10.0, 60.0, zero_frac=0.1, tile=(64, 64))
    ref = oracle.solve_grid(inst)
    trained = learned.load_model()
    untrained = mf.Model(16, seed=123)
    res = {}
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        for name, kw in (("plain", {}),
                         ("trained", dict(schedule=mf.MF_SCHED_LEARNED, model=trained)),
                         ("untrained", dict(schedule=mf.MF_SCHED_LEARNED, model=untrained))):
            if "model" in kw:
                kw.update(defer_threshold=learned.DEFAULT_THRESHOLD, max_defer=learned.DEFAULT_MAX_DEFER)
            st = g.solve(global_relabel_every=8, **kw)
            assert g.flow_value() == ref["flow"]
            res[name] = (st["sweeps"], st["region_discharges"])
    print("ablation (sweeps, region discharges):", res, flush=True)
    assert res["trained"][0] <= res["untrained"][0]
    assert res["trained"][1] < res["plain"][1]


def _features_sweep0_reference(inst, tile):
    """Region features at the start of sweep 0 (after Init: excess = c(s,v), all labels 0)."""
    dims = tuple(inst.dims)
    nd = len(dims)
    t3 = (1,) * (3 - nd) + tuple(tile)
    d3 = (1,) * (3 - nd) + dims
    offs = synth.offsets_for(nd, inst.conn)
    offs3 = [(0,) * (3 - nd) + tuple(o) for o in offs]
    rg = tuple(-(-d // t) for d, t in zip(d3, t3))
    cs = inst.cs.reshape(d3).astype(np.float64)
    nbr = [inst.nbr[k].reshape(d3) for k in range(len(offs))]
    out = np.zeros(rg + (6,))
    for rz in range(rg[0]):
        for ry in range(rg[1]):
            for rx in range(rg[2]):
                o = (rz * t3[0], ry * t3[1], rx * t3[2])
                ex = 0.0
                arcs = opened = 0
                for lz in range(t3[0]):
                    for ly in range(t3[1]):
                        for lx in range(t3[2]):
                            g = (o[0] + lz, o[1] + ly, o[2] + lx)
                            real = all(a < b for a, b in zip(g, d3))
                            if real and cs[g] > 0:
                                ex += cs[g]
                            for k, (dz, dy, dx) in enumerate(offs3):
                                l2 = (lz + dz, ly + dy, lx + dx)
                                if all(0 <= a < b for a, b in zip(l2, t3)):
                                    continue  # stays in the tile
                                r2 = tuple(r + (a < 0) * -1 + (a >= b) * 1 for r, a, b in zip((rz, ry, rx), l2, t3))
                                if not all(0 <= a < b for a, b in zip(r2, rg)):
                                    continue  # no region there
                                arcs += 1
                                opened += int(real and nbr[k][g] > 0)
                out[rz, ry, rx] = (np.log1p(ex) / 8, 0.0, opened / arcs if arcs else 0.0, float(ex > 0), 0.0, ex)
    return out.reshape(-1, 6)


@pytest.mark.parametrize("case", ["2d", "3d_rows"])
def test_region_features_sweep0(mf, case):
    """Region features (the scheduler's input) at sweep 0 against a NumPy recomputation."""
    import torch
    if case == "2d":
        inst = synth.random_grid((70, 90), 8, 41, tile=(32, 32))
    else:
        inst = synth.random_grid((6, 20, 45), 6, 42, tile=(4, 16, 32))
    tile = inst.tile
    ref = _features_sweep0_reference(inst, tile)
    with mf.Grid(inst.dims, inst.conn, tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        R = ref.shape[0]
        ft = torch.zeros((64, R, mf.FEATURES), dtype=torch.float32, device="cuda")
        g.solve(features=ft)
        f0 = ft[0].cpu().numpy()
    np.testing.assert_allclose(f0, ref, rtol=1e-5, atol=1e-5)


def test_learned_schedule_many_regions(mf):
    """More than 16384 regions (tiny tiles): the scheduler's queue and the CNN
    cover the whole region grid; the result is the oracle's."""
    inst = synth.random_grid((300, 300), 4, 77, tile=(2, 2))
    model = mf.Model(16, seed=2)
    _exact(mf, inst, schedule=mf.MF_SCHED_LEARNED, model=model, defer_threshold=0.5, max_defer=1)
