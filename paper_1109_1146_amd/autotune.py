"""Autotuner for batched solves: region shape, relabel interval and partial
discharges (Sec. 6.2).

It only calls the C ABI (through the binding): it builds a batch of a
calibration subset for each candidate region shape, solves it with each relabel
interval after a warm-up solve, and keeps the fastest.  Every candidate gives
the same exact result; only the time differs.
"""
from __future__ import annotations

import json
import time

import numpy as np

from . import mf

TILES = ((16, 16), (32, 32), (64, 64))
RELABEL = (0, 4, 8)
PARTIAL = (False, True)


def calibration_subset(instances, size=48, seed=0):
    """A size-stratified sample of the batch (sorted by area, evenly spaced)."""
    if len(instances) <= size:
        return list(instances)
    order = np.argsort([inst.n for inst in instances], kind="stable")
    picks = np.linspace(0, len(instances) - 1, size).round().astype(int)
    return [instances[int(order[p])] for p in picks]


def autotune_batch(instances, tiles=TILES, relabel=RELABEL, partial=PARTIAL, calib=48, reps=2,
                   graph=True):
    """Return dict(region_shape, relabel_every, partial, timings) for this batch."""
    sample = calibration_subset(instances, calib)
    timings = []
    for tile in tiles:
        b = mf.load_batch(sample, region_shape=tile)
        try:
            for ev in relabel:
                for pd in partial:
                    kw = dict(global_relabel_every=ev, graph=graph, partial=pd)
                    b.solve(**kw)  # warm-up, graph capture
                    best = float("inf")
                    for _ in range(reps):
                        t0 = time.perf_counter()
                        b.solve(**kw)
                        best = min(best, time.perf_counter() - t0)
                    timings.append(dict(region_shape=list(tile), relabel_every=ev, partial=pd,
                                        ms=best * 1e3))
        finally:
            b.close()
    win = min(timings, key=lambda t: t["ms"])
    return dict(region_shape=tuple(win["region_shape"]), relabel_every=win["relabel_every"],
                partial=win["partial"], timings=timings)


def solve_batch(instances, region_shape=None, relabel_every=None, graph=True, tune=None,
                partial=None):
    """Solve all instances in one batch; returns (flows, batch handle, tuning)."""
    if region_shape is None or relabel_every is None or partial is None:
        tune = tune or autotune_batch(instances, graph=graph)
        region_shape = region_shape or tune["region_shape"]
        relabel_every = tune["relabel_every"] if relabel_every is None else relabel_every
        partial = tune["partial"] if partial is None else partial
    b = mf.load_batch(instances, region_shape=region_shape)
    st = b.solve(global_relabel_every=relabel_every, graph=graph, partial=partial)
    return b.flow_values(), b, dict(region_shape=tuple(region_shape), relabel_every=relabel_every,
                                    partial=partial, stats=st, tune=tune)


if __name__ == "__main__":
    import sys
    import synth
    count = int(sys.argv[1]) if len(sys.argv) > 1 else 64
    insts = synth.config3_instances(count)
    print(json.dumps(autotune_batch(insts), default=str))
