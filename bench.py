"""Benchmark: exact max-flow by P-ARD region discharge on one MI355X.

One step = one full solve of the workload from Init to a maximum preflow plus
the minimal minimum cut (mf_solve + mf_min_cut), with the capacities already
resident in HBM.  Prints ONE JSON line (rank 0).

Default workload: the 464^3 6-connected blob grid with 64^3 regions (seed 4),
plain P-ARD timed, the learned-ordered schedules and the fixed-order colour
phases solved on the same input beside it, the oracle on the whole instance as
the CPU baseline and exactness check, and nested in the same line the
roofline record of the 256^3 grid with 32^3 regions and the general-network
record (a 128^3 volume with the 26-neighbourhood in region pages, resident and
streamed).  ``--workload 2d`` / ``3d`` / ``batch`` / ``graph`` select the
2048^2 8-connected grid, the 256^3 grid, the 512-instance batch or the
general network alone.
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
    "2d": dict(cfg=1, tag="grid2d8_2048", relabel=10, partial=False, round_cap=3, desc="2048x2048 2D 8-connected blob grid, 64 blobs, 10% n-links zeroed, "
                           "64x64 regions (1024), seed 1"),
    "3d": dict(cfg=2, tag="grid3d6_256", relabel=4, partial=True, round_cap=4,
               desc="256^3 3D 6-connected blob grid, 32 blobs, 32^3 regions (512), seed 2"),
    "batch": dict(cfg=3, tag="batch512", relabel=None, partial=None, desc="512 independent 2D blob grids, sides log-uniform in [32,512], "
                              "half 4- and half 8-connected, seeds 3000+i, one batched solve"),
    # the headline workload: plain vs learned-ordered ARD
    "464": dict(cfg=4, tag="grid3d6_464", relabel=3, partial=True, round_cap=16, crop=(192, 192, 192),
                reference="grid3d6_464_oracle.json",
                desc="464^3 3D 6-connected blob grid, 256 blobs, 64^3 regions (512; last layer 16 thick), seed 4"),
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", choices=sorted(WORKLOADS) + ["graph"], default="464",
                   help="464 (default: the headline 464^3 grid, with the 256^3 roofline record "
                        "and the general-network record nested), 3d (256^3), 2d (2048^2), batch "
                        "(512 instances) or graph (128^3 26-connected volume in region pages)")
    p.add_argument("--no-nested", action="store_true",
                   help="464 only: skip the nested 256^3 and general-network records")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-stream", action="store_true",
                   help="graph only: skip the streamed-pages solves (profiling runs)")
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
    p.add_argument("--round-cap", type=int, default=None, metavar="N",
                   help="at most N search-and-push rounds per region discharge and sweep (0 = off; "
                        "default: the workload's tuned setting)")
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
    a bounded sample of a workload too large to time the oracle on whole."""
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


def stored_reference(name):
    """The oracle's result on a workload too large for the oracle inside the
    bench, written by the committed script beside it (tests/golden/make_*.py,
    oracle and generator only)."""
    path = os.path.join(ROOT, "tests", "golden", name)
    with open(path) as f:
        return json.load(f), os.path.relpath(path, ROOT)


def host_cpu():
    """Model name of the host CPU and the logical CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return model, nproc


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
    model, nproc = host_cpu()
    return ref, dict(value=round(mvs, 4), unit="Mvertices/s", cores=1, kind="oracle",
                     sample=f"{reps} full solve(s) of the same instance, {t_total:.1f} s total, "
                            f"highest-label push-relabel, 1 thread",
                     cpu_model=model, nproc=nproc)


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
                    schedule=mf.MF_SCHED_PARD, region_kernel=mf.MF_KERNEL_AUTO,
                    round_cap=args.round_cap or 0, timings=[])
    else:
        tune = autotune.autotune_batch(insts, calib=48, reps=1, partial=forced, brl=brl)
    args.partial = tune["partial"]
    args.boundary_relabel = tune["boundary_relabel"]
    b = mf.load_batch(insts, region_shape=tune["region_shape"])
    stream = torch.cuda.Stream()

    def step(profile):
        st = b.solve(global_relabel_every=tune["relabel_every"], graph=not profile,
                     profile=profile, stream=stream.cuda_stream, partial=args.partial,
                     boundary_relabel=args.boundary_relabel, schedule=tune["schedule"],
                     region_kernel=tune["region_kernel"], round_cap=tune["round_cap"])
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
    kname, ksrc = kernel_of(mf, pst["region_kernel"])
    traffic = measured_traffic(f"paper_1109_1146_amd/csrc/{ksrc}",
                               f"{kname}_batch512_traffic.json",
                               config=dict(region_shape=list(tune["region_shape"]),
                                           relabel_every=tune["relabel_every"],
                                           partial=bool(args.partial),
                                           boundary_relabel=args.boundary_relabel,
                                           round_cap=tune["round_cap"]))
    rec = {
        "metric": "exact-maxflow solve throughput (batched plain P-ARD), % HBM peak",
        "value": round(total_n / (ms / 1e3) / 1e6, 3), "unit": "Mvertices/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["batch"]["desc"], "instances": len(insts), "n": total_n,
                   "canvas": list(b.dims), "region_shape": list(tune["region_shape"]),
                   "global_relabel_every": tune["relabel_every"], "graph": True,
                   "partial_discharges": args.partial, "boundary_relabel": args.boundary_relabel,
                   "schedule": "colour phases (Alg. 1)" if tune["schedule"] == mf.MF_SCHED_COLORED
                   else "P-ARD (Alg. 2)", "region_kernel": kname, "round_cap": tune["round_cap"]},
        "instances_per_s": round(len(insts) / (ms / 1e3), 1),
        "sweeps": st["sweeps"], "region_discharges": st["region_discharges"],
        "flow": int(flows.sum()),
        "autotune": tune["timings"],
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 3),
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
                       boundary_relabel=args.boundary_relabel, round_cap=tune["round_cap"])
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




GRAPH = dict(dims=(128, 128, 128), seed=9000, tile=(16, 16, 16), pages=64, round_cap=2,
             desc="128^3 volume with the 26-neighbourhood (26.8 M pairs, capacities <= 100), "
                  "4 blobs with sharp borders, 16^3 box regions (512), seed 9000")


def bench_graph(args, steps, warmup, cpu):
    """The general-network path (region pages, Sec. 5.3) on a 26-connected
    volume: `steps` solves + both cuts with every page resident in HBM (a fresh
    handle per step, built before the timed region), then the same with the
    pages streamed from pinned host memory through 64 device page slots (the
    PCIe transfers are part of that path).  Flow and both cuts compared with
    the oracle on the whole instance, which is also the CPU baseline."""
    import torch
    import synth
    from paper_1109_1146_amd import mf

    mf.load()
    inst = synth.grid26_graph(GRAPH["dims"], GRAPH["seed"])
    reg = synth.block_regions(GRAPH["dims"], GRAPH["tile"])

    def run(pages, nsteps, nwarm):
        times, out = [], None
        for i in range(nwarm + nsteps):
            g = mf.Graph(inst.n, *inst.arrays(), region=reg, device_pages=pages)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = g.solve(round_cap=GRAPH["round_cap"])
                smin = g.min_cut(mf.MF_CUT_MIN_SOURCE)
                smax = g.min_cut(mf.MF_CUT_MAX_SOURCE)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                if i >= nwarm:
                    times.append(dt)
                out = dict(flow=g.flow_value(), smin=smin, smax=smax, stats=st, info=g.info())
            finally:
                g.close()
        return sum(times) / len(times), out

    ms_res, res = run(0, steps, warmup)
    stream = not getattr(args, "no_stream", False)
    ms_str, stre = run(GRAPH["pages"], max(1, steps // 2), 0) if stream else (None, None)
    # one profiled solve: the discharge launches timed by HIP events on the solve stream
    g = mf.Graph(inst.n, *inst.arrays(), region=reg)
    try:
        pst = g.solve(profile=True, round_cap=GRAPH["round_cap"])
    finally:
        g.close()
    D, V, A = pst["discharges"], pst["discharged_vertices"], pst["discharged_arcs"]
    d_bytes = mf.graph_discharge_bytes(V, A) + 4 * (D - 1) if D else 0
    d_ms, d_launch = pst["discharge_ms"], max(pst["discharge_launches"], 1)
    achieved = d_bytes / (d_ms / 1e3) / 1e9 if d_ms > 0 else 0.0
    rec = {"workload": GRAPH["desc"], "n": inst.n, "pairs": inst.npairs, "steps": steps, "warmup": warmup,
           "ms_per_step": round(ms_res * 1e3, 3), "value": round(inst.n / ms_res / 1e6, 3),
           "unit": "Mvertices/s", "round_cap": GRAPH["round_cap"], "sweeps": res["stats"]["sweeps"],
           "region_discharges": res["stats"]["discharges"], "boundary_size": res["info"]["boundary_size"],
           "push_rounds_per_discharge": round(res["stats"]["push_rounds"] / max(res["stats"]["discharges"], 1), 2),
           "search_levels_per_discharge": round(res["stats"]["search_steps"] / max(res["stats"]["discharges"], 1), 1),
           "flow": res["flow"],
           "streamed": None if not stream else {
               "device_pages": GRAPH["pages"], "regions": res["info"]["regions"],
               "ms_per_step": round(ms_str * 1e3, 3), "value": round(inst.n / ms_str / 1e6, 3),
               "unit": "Mvertices/s (PCIe transfers included)",
               "sweeps": stre["stats"]["sweeps"], "pages_in": stre["stats"]["pages_in"],
               "pages_out": stre["stats"]["pages_out"],
               "bytes_h2d": stre["stats"]["bytes_h2d"], "bytes_d2h": stre["stats"]["bytes_d2h"],
               "same_result": bool(stre["flow"] == res["flow"] and (stre["smin"] == res["smin"]).all()
                                   and (stre["smax"] == res["smax"]).all())},
           "roofline": {"bound": "hbm", "kernel": "k_gdischarge", "achieved": round(achieved, 3),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                        "traffic": measured_traffic("paper_1109_1146_amd/csrc/mf_graph.hip",
                                                    "k_gdischarge_graph26_128_traffic.json"),
                        "avg_launch_ms": round(d_ms / d_launch, 4),
                        "algorithmic_bytes_per_launch": round(d_bytes / d_launch, 1)}}
    if cpu:
        import oracle
        oracle.build(force=False)
        t0 = time.perf_counter()
        ref = oracle.solve_pairs(inst.n, *inst.arrays())
        t_cpu = time.perf_counter() - t0
        model, nproc = host_cpu()
        rec["exact"] = bool(ref["flow"] == res["flow"] and (ref["smin"] == res["smin"]).all()
                            and (ref["smax"] == res["smax"]).all())
        rec["cpu_baseline"] = dict(value=round(inst.n / t_cpu / 1e6, 4), unit="Mvertices/s", cores=1,
                                   kind="oracle", sample=f"1 full solve of the same instance, {t_cpu:.1f} s, "
                                                         "highest-label push-relabel, 1 thread",
                                   cpu_model=model, nproc=nproc)
    return rec


def kernel_of(mf, kid):
    return {mf.MF_KERNEL_WAVE: ("k_discharge_wave", "mf_discharge_wave.hip"),
            mf.MF_KERNEL_ROWS: ("k_discharge_rows", "mf_discharge_rows.hip"),
            mf.MF_KERNEL_ROWS64: ("k_discharge_rows64", "mf_discharge_rows64.hip"),
            mf.MF_KERNEL_LDS: ("k_discharge_lds", "mf_discharge_lds.hip"),
            mf.MF_KERNEL_HBM: ("k_discharge", "mf_kernels.hip")}[kid]


def bench_grid(args, wl, steps, warmup, compare, cpu):
    """Time `steps` solves + minimal cuts of one grid workload (after `warmup`),
    with every discharge launch timed by HIP events on the solve stream.  With
    compare, solve the same input with the learned-ordered schedules and the
    fixed-order colour phases beside it; with cpu, run the oracle on the whole
    instance (CPU baseline and exactness of the flow and both cuts)."""
    import numpy as np
    import torch
    import synth
    from paper_1109_1146_amd import mf

    method = mf.MF_METHOD_PRD if args.method == "prd" else mf.MF_METHOD_ARD
    schedule = mf.MF_SCHED_COLORED if args.schedule == "colored" else mf.MF_SCHED_PARD
    t_gen = time.perf_counter()
    inst = synth.config(wl["cfg"])
    t_gen = time.perf_counter() - t_gen
    print(f"bench: {inst.name} generated in {t_gen:.1f} s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    cs = torch.from_numpy(inst.cs).to(dev)
    ct = torch.from_numpy(inst.ct).to(dev)
    nbr = torch.from_numpy(np.ascontiguousarray(inst.nbr)).to(dev)
    torch.cuda.synchronize()

    g = mf.Grid(inst.dims, inst.conn, inst.tile)
    g.set_caps(cs, ct, nbr, stream=stream.cuda_stream)
    del cs, ct, nbr
    info = g.info()
    relabel, partial, brl = args.relabel_every, args.partial, args.boundary_relabel
    rcap = args.round_cap

    def step(profile):
        st = g.solve(stream=stream.cuda_stream, profile=profile, global_relabel_every=relabel,
                     partial=partial, boundary_relabel=brl, method=method, schedule=schedule,
                     round_cap=rcap,
                     max_sweeps=1 << 40)
        cut = g.min_cut(mf.MF_CUT_MIN_SOURCE)
        return st, cut

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        st, cut = step(True)
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    flow = g.flow_value()
    smax = g.min_cut(mf.MF_CUT_MAX_SOURCE)
    print(f"bench: {steps} timed steps in {elapsed:.1f} s", file=sys.stderr, flush=True)

    ms_per_step = elapsed * 1e3 / steps
    d_ms = sum(s["discharge_ms"] for s in stats)
    d_launch = sum(s["discharge_launches"] for s in stats)
    d_bytes = sum(s["discharge_bytes"] for s in stats)
    achieved = d_bytes / (d_ms / 1e3) / 1e9 if d_ms > 0 else 0.0
    kname, ksrc = kernel_of(mf, stats[-1]["region_kernel"])
    # the committed counter summaries cover the parallel ARD solves
    traffic = (None if args.method == "prd" or args.schedule == "colored" else
               measured_traffic("paper_1109_1146_amd/csrc/" + ksrc, f"{kname}_{wl['tag']}_traffic.json"))
    rec = {
        "ms_per_step": round(ms_per_step, 3),
        "value": round(inst.n / (ms_per_step / 1e3) / 1e6, 3),
        "config": {"workload": wl["desc"], "n": inst.n, "regions": info["regions"],
                   "region_shape": list(info["region_shape"]), "boundary_size": info["boundary_size"],
                   "schedule": ("S-" if args.schedule == "colored" else "P-") + args.method.upper()
                               + (" (colour phases)" if args.schedule == "colored" else "")
                               + (", partial discharges" if partial else "")
                               + (", boundary relabel" if brl else "")
                               + (f", at most {rcap} rounds per discharge and sweep" if rcap else ""),
                   "connectivity": inst.conn,
                   "global_relabel_every": relabel, "partial_discharges": partial,
                   "boundary_relabel": brl, "round_cap": rcap},
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

    def timed_solves(kw):
        g.solve(**kw)
        times = []
        for _ in range(max(1, min(steps, 3))):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            vst = g.solve(**kw)
            times.append((time.perf_counter() - t1) * 1e3)
        return vst, float(np.median(times))

    if compare:
        # the learned-ordered schedules on the same input (not in value):
        # sweeps, discharges and solve time next to plain P-ARD, same exact
        # flow; and the colour phases in fixed order, the learned colour
        # schedule's skeleton without the network
        base = dict(global_relabel_every=relabel, stream=stream.cuda_stream, partial=partial, round_cap=rcap)
        try:
            from paper_1109_1146_amd import learned
            model = learned.load_model()
            variants = (("learned", dict(schedule=mf.MF_SCHED_LEARNED, model=model,
                                         defer_threshold=learned.DEFAULT_THRESHOLD,
                                         max_defer=learned.DEFAULT_MAX_DEFER, boundary_relabel=brl)),
                        ("learned_colored", dict(schedule=mf.MF_SCHED_LEARNED_COLORED, model=model,
                                                 defer_threshold=1e-9, max_defer=1)),
                        ("colored_fixed_order", dict(schedule=mf.MF_SCHED_COLORED)))
        except (OSError, ValueError) as e:  # no trained model in the tree
            rec["learned"] = {"error": str(e)}
            variants = (("colored_fixed_order", dict(schedule=mf.MF_SCHED_COLORED)),)
        for key, kw in variants:
            try:
                vst, vms = timed_solves(dict(base, **kw))
                rec[key] = {"solve_ms": round(vms, 3), "sweeps": vst["sweeps"],
                            "region_discharges": vst["region_discharges"],
                            "flow_equal": g.flow_value() == flow}
            except mf.MFError as e:
                rec[key] = {"error": str(e)}
            print(f"bench: {key} done", file=sys.stderr, flush=True)
        plain = {"solve_ms": rec["solve_ms"], "sweeps": rec["sweeps"],
                 "region_discharges": rec["region_discharges"]}
        rec["plain"] = plain
        for key in ("learned", "learned_colored"):
            v = rec.get(key, {})
            if "sweeps" in v:
                v["fewer_sweeps_and_less_time_than_plain"] = bool(
                    v["flow_equal"] and v["sweeps"] < plain["sweeps"] and v["solve_ms"] < plain["solve_ms"])
        fixed = rec.get("colored_fixed_order", {})
        if "sweeps" in rec.get("learned_colored", {}) and "sweeps" in fixed:
            rec["learned_colored"]["fewer_sweeps_and_less_time_than_fixed_order"] = bool(
                rec["learned_colored"]["sweeps"] < fixed["sweeps"]
                and rec["learned_colored"]["solve_ms"] < fixed["solve_ms"])
    g.close()
    if cpu and "reference" in wl:
        # the whole instance is beyond the oracle within the bench's time: the
        # oracle is timed on a corner block, and the result is compared with the
        # oracle's stored result on the whole instance
        import hashlib
        sample = crop_instance(inst, wl["crop"])
        _, cb = cpu_baseline(sample, args.cpu_seconds)
        cb["sample"] = (f"a {'x'.join(map(str, wl['crop']))} corner block of the instance (arcs leaving "
                        f"it dropped): " + cb["sample"])
        rec["cpu_baseline"] = cb
        want, path = stored_reference(wl["reference"])
        got_min = hashlib.sha256(np.ascontiguousarray(cut, np.uint8).tobytes()).hexdigest()
        got_max = hashlib.sha256(np.ascontiguousarray(smax, np.uint8).tobytes()).hexdigest()
        rec["exact"] = bool(want["flow"] == flow and want["smin_sha256"] == got_min
                            and want["smax_sha256"] == got_max)
        rec["exact_reference"] = (f"{path}: the oracle on the whole instance "
                                  f"({want['oracle_seconds']} s, 1 thread, when stored)")
        print(f"bench: oracle sample done", file=sys.stderr, flush=True)
    elif cpu:
        ref, cb = cpu_baseline(inst, args.cpu_seconds)
        rec["cpu_baseline"] = cb
        rec["exact"] = bool(ref["flow"] == flow and (ref["smin"] == cut).all()
                            and (ref["smax"] == smax).all())
        print(f"bench: oracle done", file=sys.stderr, flush=True)
    return rec


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
    if args.workload == "graph":
        sub = bench_graph(args, args.steps, args.warmup, cpu=not args.no_cpu_baseline)
        rec = {"metric": "exact-maxflow solve throughput, general network in region pages (P-ARD)",
               "value": sub.pop("value"), "unit": sub.pop("unit"), "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": sub.pop("ms_per_step"), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
               "config": {"workload": sub.pop("workload")}}
        rec.update(sub)
        print(json.dumps(rec), flush=True)
        return
    from paper_1109_1146_amd import mf

    mf.load()
    wl = WORKLOADS[args.workload]
    if args.relabel_every is None:
        args.relabel_every = wl["relabel"]
    args.partial = {"on": True, "off": False}.get(args.partial, wl["partial"])
    if args.boundary_relabel is None:
        args.boundary_relabel = 0
    if args.round_cap is None:
        args.round_cap = wl.get("round_cap", 0)
    if args.schedule == "colored":
        args.boundary_relabel, args.no_learned = 0, True
    if args.method == "prd":
        # the exact relabel and the heuristics are those of region distances
        args.relabel_every, args.partial, args.boundary_relabel, args.no_learned = 0, False, 0, True
        args.round_cap = 0
    headline = args.workload == "464"
    sub = bench_grid(args, wl, args.steps, args.warmup, compare=not args.no_learned,
                     cpu=not args.no_cpu_baseline)
    rec = {
        "metric": ("exact-maxflow solve time + sweeps, plain vs learned-ordered ARD; % HBM peak"
                   if headline else
                   "exact-maxflow solve throughput (plain %s-%s), sweeps, %% HBM peak" % (
                       "S" if args.schedule == "colored" else "P", args.method.upper())),
        "value": sub.pop("value"),
        "unit": "Mvertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sub.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
    }
    rec.update(sub)
    if headline and not args.no_nested:
        # the HBM-roofline configuration: 256^3 with 32^3 regions, its tuned
        # settings, a few timed steps (roofline only: no comparison, no oracle)
        w3 = WORKLOADS["3d"]
        a3 = argparse.Namespace(**vars(args))
        a3.relabel_every, a3.partial = w3["relabel"], w3["partial"]
        a3.round_cap = w3.get("round_cap", 0)
        n3 = bench_grid(a3, w3, 3, 1, compare=False, cpu=False)
        rec["grid3d6_256"] = {"workload": n3["config"]["workload"], "steps": 3, "warmup": 1,
                              "ms_per_step": n3["ms_per_step"], "value": n3["value"],
                              "unit": "Mvertices/s", "sweeps": n3["sweeps"],
                              "region_discharges": n3["region_discharges"],
                              "global_relabel_every": w3["relabel"],
                              "partial_discharges": w3["partial"], "round_cap": a3.round_cap,
                              "roofline": n3["roofline"]}
        # the general-network path (region pages) on a 26-connected volume
        rec["graph26_128"] = bench_graph(args, 2, 1, cpu=not args.no_cpu_baseline)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
