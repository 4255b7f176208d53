"""Learned region scheduler: trace collection, GPU training, evaluation.

The scheduler CNN (``mf.Model``, kernels in ``csrc/mf_sched.hip``) reads three
features per region at the start of a sweep (active excess, boundary label
level, residual degree of the boundary) and predicts whether discharging the
region in this sweep makes progress: it sends flow to the sink, or the excess
it pushes out does not come back (a bounce is a discharge whose region holds
at least 90% of the same excess at its next discharge, with nothing sent to the
sink).  ``train --slow-bounce`` marks only the bounces among the slower half of
their sweep's discharges (a sweep lasts as long as its slowest region).
``MF_SCHED_LEARNED`` defers active regions whose probability is below a
threshold (at most ``max_defer`` sweeps in a row, never in the first sweep) and
queues the others longest previous discharge first.  The exact result never
depends on the scores.

Training data are plain P-ARD solves (the fallback schedule, relabel every 8
sweeps, or the bench intervals with ``--slow-bounce``) of instances from the generator families of the 2048^2
8-connected and 256^3 6-connected workloads, with training seeds (100-105)
disjoint from the validation seeds of ``tune`` (110, 111) and the bench seeds.  Training
runs on the GPU with the library's own forward, backward and Adam kernels.

    python -m paper_1109_1146_amd.learned train      # writes models/sched_cnn16.npy
    python -m paper_1109_1146_amd.learned train --slow-bounce [path]
    python -m paper_1109_1146_amd.learned tune       # deferral threshold on validation instances
    python -m paper_1109_1146_amd.learned evaluate   # plain vs learned on the workloads
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import mf

PKG = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(PKG, "models", "sched_cnn16.npy")
CHANNELS = 16
TRAIN_SEEDS_2D = (100, 101, 102, 103)
TRAIN_SEEDS_3D = (104, 105)


def train_instance(kind, seed):
    import synth
    if kind == "2d":
        return synth.blob_grid((2048, 2048), 8, seed, 64, 10.0, 80.0, zero_frac=0.1, tile=(64, 64),
                               name=f"train2d_{seed}")
    return synth.blob_grid((256, 256, 256), 6, seed, 32, 8.0, 32.0, tile=(32, 32, 32),
                           name=f"train3d_{seed}")


def region_dims(inst, tile=None):
    tile = tuple(tile or inst.tile)
    d = tuple(int(x) for x in inst.dims)
    if len(d) == 2:
        d, tile = (1,) + d, (1,) + tile
    return tuple(-(-a // b) for a, b in zip(d, tile))


def progress_targets(rec, bounce=0.9, slow_q=None):
    """1 for a discharge that sent flow to the sink or whose excess did not come
    back by the region's next discharge; 0 for a bounce.  With slow_q, only the
    bounces at or above the slow_q quantile of their sweep's discharge times are
    0 (a sweep lasts as long as its slowest discharge)."""
    s, r = rec[:, 0], rec[:, 1]
    ex_in = rec[:, 6].astype(np.float64)
    to_sink = rec[:, 7]
    y = np.ones(len(rec), np.float32)
    order = np.lexsort((s, r))
    for a, b in zip(order[:-1], order[1:]):
        if r[a] == r[b] and to_sink[a] == 0 and ex_in[b] >= bounce * ex_in[a]:
            y[a] = 0.0
    if slow_q is not None:
        ticks = rec[:, 5].astype(np.float64)
        for sw in np.unique(s):
            m = s == sw
            cut = np.quantile(ticks[m], slow_q)
            y[m & (ticks < cut)] = 1.0
    return y


# relabel intervals the solves use (those of the bench workloads)
RELABEL = {"2d": 10, "3d": 4}
SLOW_Q = 0.5


def collect(inst, relabel_every=8, max_sweeps=256, trace_cap=500000, target="progress"):
    """Plain P-ARD solve with per-sweep features and per-discharge traces.
    Returns a list of (features [R, 6], target [R], mask [R], dims) CUDA tensors,
    one per sweep after the first (deferral never applies to the first)."""
    import torch
    rd = region_dims(inst)
    R = int(np.prod(rd))
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        tr = torch.zeros((trace_cap, mf.TRACE_FIELDS), dtype=torch.int32, device="cuda")
        ft = torch.zeros((max_sweeps, R, mf.FEATURES), dtype=torch.float32, device="cuda")
        st = g.solve(trace=tr, features=ft, global_relabel_every=relabel_every)
    n = min(st["trace_records"], trace_cap)
    rec = tr[:n].cpu().numpy()
    S = min(st["sweeps"], max_sweeps)
    if target == "progress":
        y = progress_targets(rec)
    elif target == "slow_bounce":
        y = progress_targets(rec, slow_q=SLOW_Q)
    else:
        y = (rec[:, 7] > 0).astype(np.float32)
    out = []
    for s in range(1, S):
        m = rec[:, 0] == s
        target = np.zeros(R, np.float32)
        mask = np.zeros(R, np.float32)
        regs = rec[m, 1]
        mask[regs] = 1.0
        target[regs] = y[m]
        if mask.sum() == 0:
            continue
        out.append((ft[s].clone(), torch.from_numpy(target).cuda(), torch.from_numpy(mask).cuda(), rd))
    return out, st


def train(examples, epochs=60, lr=3e-3, seed=0, log=print):
    model = mf.Model(CHANNELS, seed=seed)
    rng = np.random.default_rng(seed)
    for ep in range(epochs):
        tot = 0.0
        for i in rng.permutation(len(examples)):
            x, t, m, rd = examples[i]
            loss, _ = model.loss_grad(x, t, m, rd)
            model.adam_step(lr)
            tot += loss
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"epoch {ep} mean loss {tot / len(examples):.4f}")
    return model


def accuracy(model, examples, threshold=0.5):
    import torch
    hit, cnt = 0.0, 0.0
    for x, t, m, rd in examples:
        z = model.forward(x, rd, bf16=True)
        p = (torch.sigmoid(z) >= threshold).float()
        hit += float(((p == t).float() * m).sum())
        cnt += float(m.sum())
    return hit / max(cnt, 1.0)


def save(model, path=MODEL_PATH):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, model.get_params())


def load_model(path=MODEL_PATH):
    p = np.load(path, allow_pickle=False)
    m = mf.Model(CHANNELS)
    m.set_params(p)
    return m


DEFAULT_THRESHOLD = 0.1
DEFAULT_MAX_DEFER = 1


def compare(inst, model, relabel_every=8, threshold=DEFAULT_THRESHOLD, max_defer=DEFAULT_MAX_DEFER,
            reps=3):
    """Plain P-ARD vs the learned schedule on one instance (same exact flow)."""
    out = {}
    with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
        g.set_caps(inst.cs, inst.ct, inst.nbr)
        for name, kw in (("plain", {}),
                         ("learned", dict(schedule=mf.MF_SCHED_LEARNED, model=model,
                                          defer_threshold=threshold, max_defer=max_defer))):
            g.solve(global_relabel_every=relabel_every, **kw)
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                st = g.solve(global_relabel_every=relabel_every, **kw)
                times.append((time.perf_counter() - t0) * 1e3)
            out[name] = dict(ms=float(np.median(times)), sweeps=st["sweeps"],
                             region_discharges=st["region_discharges"], flow=g.flow_value())
    return out


def main(argv):
    cmd = argv[1] if len(argv) > 1 else "train"
    mf.load()
    if cmd == "train":
        slow = "--slow-bounce" in argv
        argv = [a for a in argv if a != "--slow-bounce"]
        examples = []
        for kind, seeds in (("2d", TRAIN_SEEDS_2D), ("3d", TRAIN_SEEDS_3D)):
            for seed in seeds:
                inst = train_instance(kind, seed)
                if slow:
                    ex, st = collect(inst, relabel_every=RELABEL[kind], target="slow_bounce")
                else:
                    ex, st = collect(inst)
                print(f"traces {inst.name}: {len(ex)} sweeps, {st['region_discharges']} discharges",
                      flush=True)
                examples += ex
        model = train(examples)
        print(json.dumps({"train_accuracy_bf16": accuracy(model, examples)}), flush=True)
        path = argv[2] if len(argv) > 2 else MODEL_PATH
        save(model, path)
        print(f"saved {path}", flush=True)
    elif cmd == "evaluate":
        import synth
        model = load_model(argv[3] if len(argv) > 3 else MODEL_PATH)
        for cfg in [int(c) for c in (argv[2] if len(argv) > 2 else "1,2").split(",")]:
            inst = synth.config(cfg)
            rel = RELABEL["2d" if len(inst.dims) == 2 else "3d"]
            print(json.dumps({"workload": inst.name, **compare(inst, model, relabel_every=rel)}), flush=True)
    elif cmd == "tune":
        # deferral threshold and limit, chosen on validation instances (seeds
        # disjoint from the training and bench instances)
        model = load_model(argv[2] if len(argv) > 2 else MODEL_PATH)
        for kind, seed in (("2d", 110), ("3d", 111)):
            inst = train_instance(kind, seed)
            rel = RELABEL[kind]
            with mf.Grid(inst.dims, inst.conn, inst.tile) as g:
                g.set_caps(inst.cs, inst.ct, inst.nbr)
                runs = [("plain", {})] + [(f"t{t}_d{d}_m{mode}", dict(schedule=mf.MF_SCHED_LEARNED, model=model,
                                                                      defer_threshold=t, max_defer=d,
                                                                      defer_mode=mode))
                                          for mode in (0, 1) for t in (0.1, 0.3, 0.5) for d in (1, 2)]
                for name, kw in runs:
                    g.solve(global_relabel_every=rel, **kw)
                    times = []
                    for _ in range(2):
                        t0 = time.perf_counter()
                        st = g.solve(global_relabel_every=rel, **kw)
                        times.append((time.perf_counter() - t0) * 1e3)
                    print(json.dumps({"instance": inst.name, "run": name, "ms": round(min(times), 2),
                                      "sweeps": st["sweeps"], "discharges": st["region_discharges"],
                                      "relabel_only": st["relabel_only"], "flow": g.flow_value()}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
