"""Benchmark: exact max-flow by P-ARD region discharge on one MI355X.

One step = one full solve of the workload from Init to a maximum preflow plus
the minimal minimum cut (mf_solve + mf_min_cut), with the capacities already
resident in HBM.  Prints ONE JSON line (rank 0).

Default workload: the 2048 x 2048 8-connected blob grid with 64 x 64 regions
(seed 1); ``--workload 3d`` selects the 256^3 6-connected grid with 32^3 regions.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def measured_traffic(kernel_src, summary, config=None):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated), or None when
    the summary is missing, the kernel source changed since it was taken, or
    (with config) it was taken with other solve settings."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    src = os.path.join(ROOT, kernel_src)
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if rec.get("source_sha256") != sha:
        return None
    if config is not None and rec.get("config") != config:
        return None
    return float(rec["traffic_bytes_per_launch"])

WORKLOADS = {
    "2d": dict(cfg=1, tag="grid2d8_2048", relabel=10, partial=False, desc="2048x2048 2D 8-connected blob grid, 64 blobs, 10% n-links zeroed, "
                           "64x64 regions (1024), seed 1"),
    "3d": dict(cfg=2, tag="grid3d6_256", relabel=4, partial=True, desc="256^3 3D 6-connected blob grid, 32 blobs, 32^3 regions (512), seed 2"),
    "batch": dict(cfg=3, tag="batch512", relabel=None, partial=None, desc="512 independent 2D blob grids, sides log-uniform in [32,512], "
                              "half 4- and half 8-connected, seeds 3000+i, one batched solve"),
    # the learned scheduler's workload: one solve takes seconds, run it with --steps 1 --warmup 0
    "464": dict(cfg=4, tag="grid3d6_464", relabel=4, partial=False, crop=(160, 160, 160),
                desc="464^3 3D 6-connected blob grid, 256 blobs, 64^3 regions (512), seed 4"),
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", choices=sorted(WORKLOADS), default="2d",
                   help="2d, 3d, batch, or 464 (the learned scheduler's workload: use --steps 1 "
                        "--warmup 0; its oracle baseline runs on a 160^3 corner block)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-learned", action="store_true",
                   help="skip the learned-schedule comparison solves (profiling runs)")
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="CPU work budget of the oracle baseline sample")
    p.add_argument("--relabel-every", type=int, default=None,
                   help="exact region-distance relabel every N sweeps (0 = off; default: the "
                        "workload's tuned interval)")
    p.add_argument("--partial", choices=("auto", "on", "off"), default="auto",
                   help="partial discharges (sweep s runs only the stages k <= s of ARD); auto: "
                        "the workload's tuned setting (the autotuner's for the batch)")
    p.add_argument("--boundary-relabel", type=int, default=None, metavar="N",
                   help="boundary relabel heuristic after every sweep with at most N levels "
                        "(0 = off); default: off for the single grids, the autotuner's choice "
                        "for the batch")
    p.add_argument("--schedule", choices=("parallel", "colored"), default="parallel",
                   help="sweep driver: parallel (Alg. 2, all regions at once) or colored (Alg. 1 "
                        "as phases of non-interacting regions)")
    p.add_argument("--method", choices=("ard", "prd"), default="ard",
                   help="region discharge: ard (augmented paths, Sec. 4) or prd (push-relabel, "
                        "Sec. 3; no exact relabel, partial discharges or boundary relabel, and no "
                        "learned comparison)")
    p.add_argument("--region-shape", type=int, nargs=2, default=None, metavar=("H", "W"),
                   help="batch only: solve with this region shape and the given relabel, "
                        "partial and boundary-relabel settings instead of autotuning "
                        "(defaults: no relabel, full discharges, no boundary relabel)")
    p.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                   help="only run a device-to-device copy of MIB MiB (HBM counter calibration)")
    return p.parse_args()


def calibrate_copy(mib):
    """A plain copy kernel of known size: reads and writes mib MiB once each, so
    that a hardware-counter run can relate FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": n * 4}), flush=True)


def crop_instance(inst, shape):
    """The corner block [0, shape) of a grid instance, arcs leaving it dropped:
    a bounded sample of a workload too large for the oracle."""
    import numpy as np
    import synth
    dims = tuple(inst.dims)
    sl = tuple(slice(0, c) for c in shape)
    nbr = []
    for k, off in enumerate(synth.offsets_for(len(dims), inst.conn)):
        a = np.array(inst.nbr[k].reshape(dims)[sl])
        for ax, o in enumerate(off):
            if o > 0:
                a[(slice(None),) * ax + (slice(shape[ax] - o, None),)] = 0
        nbr.append(a.reshape(-1))
    return synth.GridInstance(dims=tuple(shape), conn=inst.conn,
                              cs=np.ascontiguousarray(inst.cs.reshape(dims)[sl]).reshape(-1),
                              ct=np.ascontiguousarray(inst.ct.reshape(dims)[sl]).reshape(-1),
                              nbr=np.stack(nbr), tile=inst.tile,
                              name=f"{inst.name}_corner{'x'.join(map(str, shape))}")


def cpu_baseline(inst, budget_s):
    """The oracle (single-thread push-relabel) on whole copies of the same
    instance, repeated until the budget is used (at least once)."""
    import oracle
    oracle.build(force=False)
    reps, t_total, ref = 0, 0.0, None
    while True:
        t0 = time.perf_counter()
        ref = oracle.solve_grid(inst, method="pr")
        t_total += time.perf_counter() - t0
        reps += 1
        if t_total >= budget_s or reps >= 3:
            break
    mvs = inst.n * reps / t_total / 1e6
    return ref, dict(value=round(mvs, 4), unit="Mvertices/s", cores=1, kind="oracle",
                     sample=f"{reps} full solve(s) of the same instance, {t_total:.1f} s total, "
                            f"highest-label push-relabel, 1 thread")


def bench_batch(args):
    """Batched workload: autotune (region shape, relabel interval) on a
    calibration subset, then time whole-batch solves (captured sweep batches)."""
    import torch
    import synth
    from paper_1109_1146_amd import autotune, mf

    mf.load()
    insts = synth.config3_instances(512)
    total_n = sum(inst.n for inst in insts)
    forced = {"on": (True,), "off": (False,)}.get(args.partial, autotune.PARTIAL)
    brl = autotune.BRL if args.boundary_relabel is None else (args.boundary_relabel,)
    if args.region_shape:
        # fixed settings (profiling runs): no tuning solves
        tune = dict(region_shape=tuple(args.region_shape), relabel_every=args.relabel_every or 0,
                    partial=args.partial == "on", boundary_relabel=args.boundary_relabel or 0,
                    timings=[])
    else:
        tune = autotune.autotune_batch(insts, calib=48, reps=1, partial=forced, brl=brl)
    args.partial = tune["partial"]
    args.boundary_relabel = tune["boundary_relabel"]
    b = mf.load_batch(insts, region_shape=tune["region_shape"])
    stream = torch.cuda.Stream()

    def step(profile):
        st = b.solve(global_relabel_every=tune["relabel_every"], graph=not profile,
                     profile=profile, stream=stream.cuda_stream, partial=args.partial,
                     boundary_relabel=args.boundary_relabel)
        flows = b.flow_values()
        cut = b.min_cut(mf.MF_CUT_MIN_SOURCE)
        return st, flows, cut

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, flows, _ = step(False)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pst, _, _ = step(True)  # one profiled solve for the kernel average (events need eager launches)
    ms = elapsed * 1e3 / args.steps
    d_ms, d_launch, d_bytes = pst["discharge_ms"], pst["discharge_launches"], pst["discharge_bytes"]
    achieved = d_bytes / (d_ms / 1e3) / 1e9 if d_ms > 0 else 0.0
    traffic = measured_traffic("paper_1109_1146_amd/csrc/mf_discharge_wave.hip",
                               "k_discharge_wave_batch512_traffic.json",
                               config=dict(region_shape=list(tune["region_shape"]),
                                           relabel_every=tune["relabel_every"],
                                           partial=bool(args.partial),
                                           boundary_relabel=args.boundary_relabel))
    rec = {
        "metric": "exact-maxflow solve throughput (batched plain P-ARD), % HBM peak",
        "value": round(total_n / (ms / 1e3) / 1e6, 3), "unit": "Mvertices/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["batch"]["desc"], "instances": len(insts), "n": total_n,
                   "canvas": list(b.dims), "region_shape": list(tune["region_shape"]),
                   "global_relabel_every": tune["relabel_every"], "graph": True,
                   "partial_discharges": args.partial, "boundary_relabel": args.boundary_relabel},
        "instances_per_s": round(len(insts) / (ms / 1e3), 1),
        "sweeps": st["sweeps"], "region_discharges": st["region_discharges"],
        "flow": int(flows.sum()),
        "autotune": tune["timings"],
        "roofline": {"bound": "hbm", "kernel": "k_discharge_wave", "achieved": round(achieved, 3),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                     "traffic": traffic, "avg_launch_ms": round(d_ms / max(d_launch, 1), 4),
                     "algorithmic_bytes_per_launch": round(d_bytes / max(d_launch, 1), 1)},
    }
    # the learned schedule on the same batch (not in value): sweeps, discharges, time
    if not args.no_learned:
        try:
            from paper_1109_1146_amd import learned
            model = learned.load_model()
            lkw = dict(schedule=mf.MF_SCHED_LEARNED, model=model, defer_threshold=learned.DEFAULT_THRESHOLD,
                       max_defer=learned.DEFAULT_MAX_DEFER, global_relabel_every=tune["relabel_every"],
                       stream=stream.cuda_stream, partial=args.partial,
                       boundary_relabel=args.boundary_relabel)
            b.solve(**lkw)
            lt = []
            for _ in range(max(1, min(args.steps, 3))):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                lst = b.solve(**lkw)
                lt.append((time.perf_counter() - t1) * 1e3)
            lflows = b.flow_values()
            rec["learned"] = {"solve_ms": round(float(sorted(lt)[len(lt) // 2]), 3), "sweeps": lst["sweeps"],
                              "region_discharges": lst["region_discharges"],
                              "flow_equal": bool((lflows == flows).all()), "plain_ms_per_step": round(ms, 3),
                              "plain_sweeps": st["sweeps"], "plain_region_discharges": st["region_discharges"]}
        except (OSError, ValueError, mf.MFError) as e:  # no trained model, or a schedule limit
            rec["learned"] = {"error": str(e)}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        t_cpu, done, exact = 0.0, 0, True
        for i, inst in enumerate(insts):
            t1 = time.perf_counter()
            ref = oracle.solve_grid(inst)
            t_cpu += time.perf_counter() - t1
            exact = exact and ref["flow"] == int(flows[i])
            done += inst.n
            if t_cpu > args.cpu_seconds:
                break
        rec["cpu_baseline"] = dict(value=round(done / t_cpu / 1e6, 4), unit="Mvertices/s", cores=1,
                                   kind="oracle", sample=f"first {i + 1} instances of the batch, "
                                   f"{t_cpu:.1f} s, highest-label push-relabel, 1 thread")
        rec["exact_sample"] = bool(exact)
    b.close()
    print(json.dumps(rec), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; multi-GPU runs are not supported, --gpus must be 1"}))
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.workload == "batch":
        bench_batch(args)
        return
    import numpy as np
    import torch
    import synth
    from paper_1109_1146_amd import mf

    mf.load()
    wl = WORKLOADS[args.workload]
    if args.relabel_every is None:
        args.relabel_every = wl["relabel"]
    args.partial = {"on": True, "off": False}.get(args.partial, wl["partial"])
    if args.boundary_relabel is None:
        args.boundary_relabel = 0
    method = mf.MF_METHOD_PRD if args.method == "prd" else mf.MF_METHOD_ARD
    schedule = mf.MF_SCHED_COLORED if args.schedule == "colored" else mf.MF_SCHED_PARD
    if args.schedule == "colored":
        args.boundary_relabel, args.no_learned = 0, True
    if args.method == "prd":
        # the exact relabel and the heuristics are those of region distances
        args.relabel_every, args.partial, args.boundary_relabel, args.no_learned = 0, False, 0, True
    inst = synth.config(wl["cfg"])
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    cs = torch.from_numpy(inst.cs).to(dev)
    ct = torch.from_numpy(inst.ct).to(dev)
    nbr = torch.from_numpy(np.ascontiguousarray(inst.nbr)).to(dev)
    torch.cuda.synchronize()

    g = mf.Grid(inst.dims, inst.conn, inst.tile)
    g.set_caps(cs, ct, nbr, stream=stream.cuda_stream)
    info = g.info()

    def step(profile):
        st = g.solve(stream=stream.cuda_stream, profile=profile,
                     global_relabel_every=args.relabel_every, partial=args.partial,
                     boundary_relabel=args.boundary_relabel, method=method,
                     schedule=schedule, max_sweeps=1 << 40)
        cut = g.min_cut(mf.MF_CUT_MIN_SOURCE)
        return st, cut

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, cut = step(True)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    flow = g.flow_value()
    smax = g.min_cut(mf.MF_CUT_MAX_SOURCE)

    ms_per_step = elapsed * 1e3 / args.steps
    value = inst.n / (ms_per_step / 1e3) / 1e6
    d_ms = sum(s["discharge_ms"] for s in stats)
    d_launch = sum(s["discharge_launches"] for s in stats)
    d_bytes = sum(s["discharge_bytes"] for s in stats)
    achieved = d_bytes / (d_ms / 1e3) / 1e9 if d_ms > 0 else 0.0
    # the region kernel that ran, its source and the counter summary of this workload
    kname, ksrc = {mf.MF_KERNEL_WAVE: ("k_discharge_wave", "mf_discharge_wave.hip"),
                   mf.MF_KERNEL_ROWS: ("k_discharge_rows", "mf_discharge_rows.hip"),
                   mf.MF_KERNEL_LDS: ("k_discharge_lds", "mf_discharge_lds.hip"),
                   mf.MF_KERNEL_HBM: ("k_discharge", "mf_kernels.hip")}[stats[-1]["region_kernel"]]
    # the committed counter summaries cover the parallel ARD solves
    traffic = (None if args.method == "prd" or args.schedule == "colored" else
               measured_traffic("paper_1109_1146_amd/csrc/" + ksrc, f"{kname}_{wl['tag']}_traffic.json"))
    rec = {
        "metric": "exact-maxflow solve throughput (plain %s-%s), sweeps, %% HBM peak" % (
            "S" if args.schedule == "colored" else "P", args.method.upper()),
        "value": round(value, 3),
        "unit": "Mvertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": inst.n, "regions": info["regions"],
                   "region_shape": list(info["region_shape"]), "boundary_size": info["boundary_size"],
                   "schedule": ("S-" if args.schedule == "colored" else "P-") + args.method.upper()
                               + (" (colour phases)" if args.schedule == "colored" else "")
                               + (", partial discharges" if args.partial else "")
                               + (", boundary relabel" if args.boundary_relabel else ""),
                   "connectivity": inst.conn,
                   "global_relabel_every": args.relabel_every, "partial_discharges": args.partial,
                   "boundary_relabel": args.boundary_relabel},
        "sweeps": stats[-1]["sweeps"],
        "region_discharges": stats[-1]["region_discharges"],
        "flow": flow,
        "solve_ms": round(sum(s["solve_ms"] for s in stats) / len(stats), 3),
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": round(achieved, 3),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 6),
            "traffic": traffic,
            "avg_launch_ms": round(d_ms / max(d_launch, 1), 4),
            "algorithmic_bytes_per_launch": round(d_bytes / max(d_launch, 1), 1),
        },
    }
    # the learned-ordered schedule on the same input (untimed in value): sweeps,
    # discharges and wall time next to plain P-ARD, same exact flow
    try:
        if args.no_learned:
            raise ValueError("skipped (--no-learned)")
        from paper_1109_1146_amd import learned
        model = learned.load_model()
        lkw = dict(schedule=mf.MF_SCHED_LEARNED, model=model, defer_threshold=learned.DEFAULT_THRESHOLD,
                   max_defer=learned.DEFAULT_MAX_DEFER, global_relabel_every=args.relabel_every,
                   stream=stream.cuda_stream, partial=args.partial,
                   boundary_relabel=args.boundary_relabel)
        g.solve(**lkw)
        times = []
        for _ in range(max(1, min(args.steps, 3))):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            lst = g.solve(**lkw)
            times.append((time.perf_counter() - t1) * 1e3)
        rec["learned"] = {"solve_ms": round(float(np.median(times)), 3), "sweeps": lst["sweeps"],
                          "region_discharges": lst["region_discharges"],
                          "flow_equal": g.flow_value() == flow,
                          "plain_solve_ms": rec["solve_ms"], "plain_sweeps": rec["sweeps"],
                          "plain_region_discharges": rec["region_discharges"]}
    except (OSError, ValueError) as e:  # no trained model in the tree
        rec["learned"] = {"error": str(e)}
    # the learned schedule driving the colour phases of Alg. 1 (phase order by
    # the network, no deferral), and the same phases in fixed order (ablation)
    if not args.no_learned:
        try:
            from paper_1109_1146_amd import learned
            model = learned.load_model()
            variants = (("learned_colored", dict(schedule=mf.MF_SCHED_LEARNED_COLORED, model=model,
                                                 defer_threshold=1e-9, max_defer=1)),
                        ("colored_fixed_order", dict(schedule=mf.MF_SCHED_COLORED)))
            for key, kw in variants:
                kw.update(global_relabel_every=args.relabel_every, stream=stream.cuda_stream,
                          partial=args.partial)
                g.solve(**kw)
                times = []
                for _ in range(max(1, min(args.steps, 3))):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    vst = g.solve(**kw)
                    times.append((time.perf_counter() - t1) * 1e3)
                rec[key] = {"solve_ms": round(float(np.median(times)), 3), "sweeps": vst["sweeps"],
                            "region_discharges": vst["region_discharges"],
                            "flow_equal": g.flow_value() == flow}
        except (OSError, ValueError, mf.MFError) as e:
            rec["learned_colored"] = {"error": str(e)}
    if not args.no_cpu_baseline and "crop" in wl:
        # too large for the oracle within the bench: time it on a corner block
        sample = crop_instance(inst, wl["crop"])
        _, cb = cpu_baseline(sample, args.cpu_seconds)
        cb["sample"] = (f"a {'x'.join(map(str, wl['crop']))} corner block of the instance (arcs leaving "
                        f"it dropped): " + cb["sample"])
        rec["cpu_baseline"] = cb
        rec["exact"] = None  # the full-size flow is not checked against the oracle here
    elif not args.no_cpu_baseline:
        ref, cb = cpu_baseline(inst, args.cpu_seconds)
        rec["cpu_baseline"] = cb
        rec["exact"] = bool(ref["flow"] == flow and (ref["smin"] == cut).all()
                            and (ref["smax"] == smax).all())
    g.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
