"""Autotuner for batched solves: region shape, relabel interval, partial
discharges (Sec. 6.2), the cap on search-and-push rounds of a region discharge
per sweep, the boundary relabel heuristic (Sec. 6.1), the schedule
(P-ARD of Alg. 2 or the colour phases of Alg. 1) and the workgroup shape of a
region discharge (the region kernel: one 64-lane wavefront per region, or a
512-thread workgroup with the region in LDS).

It only calls the C ABI (through the binding): it builds a batch of a
calibration subset for each candidate region shape and solves it with each
relabel interval, partial setting, schedule and region kernel after a warm-up
solve (combinations the handle rejects, such as a kernel whose region does not
fit, are skipped).  The fastest few settings are then timed again on the whole
batch, each with and without the boundary relabel (P-ARD only: the colour
phases do not run it), and the fastest of those wins: the subset's small
instances overstate the heuristic's fixed per-sweep launch cost, and its
timings are close enough that noise decides between neighbours.  Every
candidate gives the same exact result; only the time differs.
"""
from __future__ import annotations

import json
import time

import numpy as np

from . import mf

TILES = ((16, 16), (32, 32), (64, 64))
RELABEL = (0, 4, 8)
PARTIAL = (False, True)
BRL = (0, 8)  # boundary relabel after every sweep: off, or at most 8 levels
SCHEDULES = (mf.MF_SCHED_PARD, mf.MF_SCHED_COLORED)
KERNELS = (mf.MF_KERNEL_WAVE, mf.MF_KERNEL_LDS)  # 64-lane wavefront, 512-thread workgroup
ROUND_CAPS = (0, 4)  # rounds of a region discharge per sweep: no cap, or 4


def calibration_subset(instances, size=48, seed=0):
    """A size-stratified sample of the batch (sorted by area, evenly spaced)."""
    if len(instances) <= size:
        return list(instances)
    order = np.argsort([inst.n for inst in instances], kind="stable")
    picks = np.linspace(0, len(instances) - 1, size).round().astype(int)
    return [instances[int(order[p])] for p in picks]


def autotune_batch(instances, tiles=TILES, relabel=RELABEL, partial=PARTIAL, calib=48, reps=2,
                   graph=True, brl=BRL, finalists=3, schedules=SCHEDULES, kernels=KERNELS,
                   round_caps=ROUND_CAPS):
    """Return dict(region_shape, relabel_every, partial, boundary_relabel,
    schedule, region_kernel, round_cap, timings) for this batch."""
    sample = calibration_subset(instances, calib)

    def timed(b, kw):
        b.solve(**kw)  # warm-up, graph capture
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            b.solve(**kw)
            best = min(best, time.perf_counter() - t0)
        return best * 1e3

    timings = []
    for tile in tiles:
        b = mf.load_batch(sample, region_shape=tile)
        try:
            for ev in relabel:
                for pd in partial:
                    for sch in schedules:
                        for ker in kernels:
                            for rc in round_caps:
                                kw = dict(global_relabel_every=ev, graph=graph, partial=pd, schedule=sch,
                                          region_kernel=ker, round_cap=rc)
                                try:
                                    ms = timed(b, kw)
                                except mf.MFError as e:
                                    if e.status != mf.MF_E_INVAL:
                                        raise
                                    continue  # not applicable to this region shape
                                timings.append(dict(stage="subset", region_shape=list(tile), relabel_every=ev,
                                                    partial=pd, boundary_relabel=0, schedule=sch,
                                                    region_kernel=ker, round_cap=rc, ms=ms))
        finally:
            b.close()
    best = sorted(timings, key=lambda t: t["ms"])[:max(1, finalists)]
    full = []
    for tile in sorted({tuple(t["region_shape"]) for t in best}):
        b = mf.load_batch(instances, region_shape=tile)
        try:
            for cand in best:
                if tuple(cand["region_shape"]) != tile:
                    continue
                for br in brl:
                    if br and cand["schedule"] != mf.MF_SCHED_PARD:
                        continue
                    kw = dict(global_relabel_every=cand["relabel_every"], graph=graph,
                              partial=cand["partial"], boundary_relabel=br, schedule=cand["schedule"],
                              region_kernel=cand["region_kernel"], round_cap=cand["round_cap"])
                    full.append(dict(cand, stage="full", boundary_relabel=br, ms=timed(b, kw)))
        finally:
            b.close()
    timings += full
    win = min(full, key=lambda t: t["ms"])
    return dict(region_shape=tuple(win["region_shape"]), relabel_every=win["relabel_every"],
                partial=win["partial"], boundary_relabel=win["boundary_relabel"],
                schedule=win["schedule"], region_kernel=win["region_kernel"], round_cap=win["round_cap"],
                timings=timings)


def solve_batch(instances, region_shape=None, relabel_every=None, graph=True, tune=None,
                partial=None, boundary_relabel=None, schedule=None, region_kernel=None, round_cap=None):
    """Solve all instances in one batch; returns (flows, batch handle, tuning)."""
    if (region_shape is None or relabel_every is None or partial is None or boundary_relabel is None
            or schedule is None or region_kernel is None or round_cap is None):
        tune = tune or autotune_batch(instances, graph=graph)
        region_shape = region_shape or tune["region_shape"]
        relabel_every = tune["relabel_every"] if relabel_every is None else relabel_every
        partial = tune["partial"] if partial is None else partial
        boundary_relabel = tune["boundary_relabel"] if boundary_relabel is None else boundary_relabel
        schedule = tune["schedule"] if schedule is None else schedule
        region_kernel = tune["region_kernel"] if region_kernel is None else region_kernel
        round_cap = tune["round_cap"] if round_cap is None else round_cap
    b = mf.load_batch(instances, region_shape=region_shape)
    st = b.solve(global_relabel_every=relabel_every, graph=graph, partial=partial,
                 boundary_relabel=boundary_relabel, schedule=schedule, region_kernel=region_kernel,
                 round_cap=round_cap)
    return b.flow_values(), b, dict(region_shape=tuple(region_shape), relabel_every=relabel_every,
                                    partial=partial, boundary_relabel=boundary_relabel, schedule=schedule,
                                    region_kernel=region_kernel, round_cap=round_cap, stats=st, tune=tune)


if __name__ == "__main__":
    import sys
    import synth
    count = int(sys.argv[1]) if len(sys.argv) > 1 else 64
    insts = synth.config3_instances(count)
    print(json.dumps(autotune_batch(insts), default=str))
