#!/usr/bin/env python3
"""Benchmark of the Z4c hot path on one MI355X.

Workload (a "step"): one classic RK4 step of an uneven MeshBlock level set,
1,024 blocks of 8^3/16^3/24^3/32^3 interior points (410/307/205/102) with 4
ghost points, 6th-order finite differences, Kreiss-Oliger 0.5, 1+log lapse,
Gamma-driver shift, flat space + U(-1e-8, 1e-8) noise; each of the 4 stages
is one fused RHS + Runge-Kutta launch,
the whole step captured in one HIP graph and replayed.  Ghost points are
read through the periodic rule inside the stage kernels (no separate
refresh pass; the stored ghosts are not rewritten).

Metric: interior grid-point stage updates per second (one point through one
RHS evaluation and Runge-Kutta combination), FP64.  The same step with
FP32 arithmetic (FP64 storage and accumulation) is reported beside it.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Z4c RHS+RK grid-point updates/sec (FP64 vs FP32, batched) + % FP64/HBM roofline"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# FP64 operations executed per interior point and RK stage by the stage
# kernel in the tuned launch configuration (rocprofv3
# SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 of one RK4 stage-2 launch times 64
# lanes over the interior points, every lane active; an FMA counts two)
FLOP_PER_PT_STAGE = 1798 + 870 + 2 * 1313 + 6
FP32_PEAK_TFLOPS = 157.3
# Relative L2 difference of the Hamiltonian constraint between the FP32 and the
# FP64 runs of the precision study that the FP32 form must stay within.
FP32_H_TOLERANCE = 1e-5
# Algorithmic HBM bytes per interior point for each RK4 stage (22 FP64 fields,
# each value moved once): stage 1 reads u0, writes u1 and u0'; stages 2-3 read
# u0, u1, u2 and write u1, u0'; stage 4 reads u0, u1 and writes u0'.
STAGE_BYTES = [3 * 176, 5 * 176, 5 * 176, 3 * 176]
# HBM traffic of one RK4 stage-2 launch (the dominant launch: stages 2 and 3
# move the most data), from rocprofv3 counter runs of `bench.py --profile`
# with the committed autotuning cache: FETCH_SIZE and WRITE_SIZE summed over
# the launch's dispatches (mean of 3 launches), each scaled by what the
# counter reads for a device copy of 1 GiB (FETCH_SIZE reads half the bytes,
# WRITE_SIZE all of them).  Valid only for the launch configuration it was
# taken with (size class -> tile shape, persistent workgroups, waves per
# SIMD); otherwise the benchmark reports null.
PROFILED_STAGE2 = {
    "tiles": {8: ((8, 8, 4), 256, 1), 16: ((8, 8, 4), 256, 1), 24: ((8, 8, 4), 256, 1),
              32: ((8, 8, 4), 256, 1)},
    "fetch_kib": 3850980.8, "fetch_scale": 2.0,
    "write_kib": 2656116.1, "write_scale": 1.0,
}


# The launch shapes the autotuner chose on an MI355X for the benchmark's size
# classes, kept so that every run times (and every profile counts) the same
# launch configuration; classes missing from it are timed and added.
TUNE_CACHE = os.path.join(ROOT, "paper_2311_04989_amd", "tune_gfx950.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the FP32-vs-FP64 constraint study on 8 x 128^3 blocks")
    ap.add_argument("--precision-steps", type=int, default=100)
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuning cache file (launch shapes per size class); '' for none")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--no-matter", action="store_true",
                    help="skip the matter-coupling kernels (metric to cells, ADM sources, "
                         "sources to vertices)")
    ap.add_argument("--no-lopsided", action="store_true",
                    help="skip the lopsided-advection stage timing")
    ap.add_argument("--no-sommerfeld", action="store_true",
                    help="skip the radiative outer boundary timing on 8 x 128^3 blocks")
    ap.add_argument("--no-intergrid", action="store_true",
                    help="skip the transfers between refinement levels")
    ap.add_argument("--intergrid-only", action="store_true",
                    help="only the transfers between refinement levels (one JSON line)")
    ap.add_argument("--profile", action="store_true",
                    help="counter-collection run: a 1 GiB device copy (calibration), then "
                         "--steps launches of RK4 stage 2 in the autotuned configuration")
    ap.add_argument("--profile-arith", choices=("fp64", "fp32"), default="fp64",
                    help="arithmetic of the --profile launches")
    ap.add_argument("--cpu-sample-blocks", type=int, default=0,
                    help="oracle sample size (0: the whole level set)")
    ap.add_argument("--matter-only", action="store_true",
                    help="only the matter-coupling and primitive-recovery kernels (one JSON line)")
    ap.add_argument("--table", action="store_true",
                    help="instead of the benchmark line: GPU FP64 / FP32 throughput of every "
                         "workload configuration and the oracle on 1 and on all host threads "
                         "(configurations 2-4), one JSON line")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "design is described but not built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2311_04989_amd import workloads as W
    from paper_2311_04989_amd import z4c as Z

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    Z.set_tune_cache(args.tune_cache or None)
    if args.profile:
        profile_run(args.steps, stream, args.profile_arith)
        return
    if args.matter_only:
        print(json.dumps(matter_coupling(stream, args.steps)), flush=True)
        return
    if args.intergrid_only:
        print(json.dumps(intergrid_transfers(stream, args.steps)), flush=True)
        return
    if args.table:
        print(json.dumps(config_table(stream, max(args.steps, 20), args.warmup)), flush=True)
        return

    t0 = time.time()
    bt = W.config4()
    log(f"[bench] generated {bt.name}: {bt.ninterior} interior / {bt.nstored} stored points "
        f"in {time.time() - t0:.1f}s")
    n_int = bt.ninterior
    nstages = 4

    def to_dev(a):
        return torch.from_numpy(a).to("cuda:0")

    y0 = to_dev(bt.u)
    results = {}
    for arith, label in ((Z.ARITH_FP64, "fp64"), (Z.ARITH_FP32, "fp32")):
        if label == "fp32" and args.no_fp32:
            continue
        plan = Z.plan_for(bt, arith)
        regs = [y0.clone(), y0.clone(), y0.clone(), torch.zeros_like(y0)]
        plan.ghost_fill(Z.GHOST_PERIODIC, regs[0], stream=stream)
        plan.set_halo(Z.GHOST_PERIODIC)   # stage launches outside the step read the same way
        default_ms = None
        if not args.no_autotune:
            if label == "fp64":
                default_ms = step_time(plan, regs, bt, stream, args.warmup, args.steps)
            plan.autotune(regs[0], regs[1], regs[3], None, reps=3, stream=stream)
        launches = {s: plan.get_launch(s, s, s) for s in (8, 16, 24, 32)}
        torch.cuda.synchronize()
        log(f"[bench] {label}: launch shapes {launches}")
        # warm-up (captures the graph on the first call)
        for _ in range(args.warmup):
            r = plan.step(regs, None, Z.RK4, bt.dt, Z.GHOST_PERIODIC, graph=True, stream=stream,
                          flags=Z.STEP_NO_FINAL_FILL)
            assert r == 0
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.steps):
            plan.step(regs, None, Z.RK4, bt.dt, Z.GHOST_PERIODIC, graph=True, stream=stream,
                      flags=Z.STEP_NO_FINAL_FILL)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        log(f"[bench] {label}: {ms:.3f} ms per RK4 step (graph replay)")
        # stage-kernel durations: the same step eager, an event pair around
        # each fused stage launch on the launch stream
        stage_ms = np.zeros(nstages)
        reps = max(3, args.steps // 2)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * nstages)]
        sched_in, sched_out = [0, 1, 2, 1], [1, 2, 1, 0]
        tab = Z.RK4
        for _ in range(reps):
            for s in range(nstages):
                evs[2 * s].record(stream)
                plan.rk_stage(regs[sched_in[s]], regs[sched_out[s]], regs[3], regs[0], None,
                              tab[s], bt.dt, stream=stream)
                evs[2 * s + 1].record(stream)
            torch.cuda.synchronize()
            for s in range(nstages):
                stage_ms[s] += evs[2 * s].elapsed_time(evs[2 * s + 1])
        stage_ms /= reps
        mon = monitor_timing(plan, regs, bt, stream, reps) if label == "fp64" else None
        # a stored-ghost refresh, timed alone for reference (not part of the step)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.ghost_fill(Z.GHOST_PERIODIC, regs[1], stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ghost_ms = e0.elapsed_time(e1)
        nonfinite = plan.check_finite(regs[0], stream=stream)
        queue = None
        if label == "fp64" and not args.no_autotune:
            # the tuned shapes once more as persistent work-queue launches
            ncu = torch.cuda.get_device_properties(0).multi_processor_count
            grid_l = {n: plan.get_launch(n, n, n) for n in (8, 16, 24, 32)}
            timings = {}
            for mode in ("grid", "persistent"):
                for n, (tile, pers, waves) in grid_l.items():
                    plan.set_launch(n, n, n, tile, 0 if mode == "grid" else ncu, waves)
                timings[mode] = stage2_time(plan, regs, bt, stream, reps)
            for n, (tile, pers, waves) in grid_l.items():
                plan.set_launch(n, n, n, tile, pers, waves)
            queue = {"grid_stage2_ms": timings["grid"], "persistent_stage2_ms": timings["persistent"],
                     "persistent_workgroups": ncu,
                     "persistent_le_grid": bool(timings["persistent"] <= 1.01 * timings["grid"])}
        results[label] = dict(ms=ms, stage_ms=stage_ms, ghost_ms=ghost_ms, launches=launches,
                              nonfinite=nonfinite, monitor=mon, default_ms=default_ms,
                              queue=queue)
        log(f"[bench] {label}: stage kernels {np.round(stage_ms, 3).tolist()} ms, "
            f"(a separate ghost refresh would cost {ghost_ms:.3f} ms), non-finite values "
            f"{nonfinite}")
        del regs
        plan.close()

    # measured device-to-device copy of 1 GiB (what HBM sustains in practice)
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cms = []
    for _ in range(10):
        e0.record(stream)
        b.copy_(a)
        e1.record(stream)
        torch.cuda.synchronize()
        cms.append(e0.elapsed_time(e1))
    copy_gbs = 2.0 * a.numel() * 8 / (float(np.median(cms)) * 1e-3) / 1e9
    del a, b

    r64 = results["fp64"]
    value = n_int * nstages / (r64["ms"] * 1e-3)
    # roofline of the dominant launch, a fused RHS + RK4 stage-2 launch:
    # algorithmic bytes (u0, u1, u2 read; u1, u0' written) over its duration
    achieved_gbs = n_int * STAGE_BYTES[1] / (r64["stage_ms"][1] * 1e-3) / 1e9
    step_gbs = n_int * sum(STAGE_BYTES) / (r64["stage_ms"].sum() * 1e-3) / 1e9
    traffic = None
    if {s: tuple(v) for s, v in r64["launches"].items()} == PROFILED_STAGE2["tiles"]:
        traffic = 1024.0 * (PROFILED_STAGE2["fetch_kib"] * PROFILED_STAGE2["fetch_scale"]
                            + PROFILED_STAGE2["write_kib"] * PROFILED_STAGE2["write_scale"])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pt-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "uneven AMR level set: 1024 MeshBlocks 8^3/16^3/24^3/32^3 "
                        "(410/307/205/102) + 4 ghosts, 6th-order FD, KO 0.5, flat space + "
                        "1e-8 noise, one RK4 step = 4 fused RHS+RK stages reading ghosts "
                        "through the periodic rule, in one HIP graph",
            "interior_points": n_int,
            "stored_points": bt.nstored,
            "stages_per_step": nstages,
            "launch_shapes": {str(k): v for k, v in r64["launches"].items()},
        },
        "zone_cycles_per_s": n_int / (r64["ms"] * 1e-3),
        "stage_kernel_ms": r64["stage_ms"].round(4).tolist(),
        "separate_ghost_refresh_ms": round(r64["ghost_ms"], 4),
        "constraint_monitor": r64["monitor"],
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": traffic,
            "launch": "one fused RHS+RK4 stage-2 launch over all 1024 blocks, "
                      f"{STAGE_BYTES[1]} algorithmic B per interior point",
        },
        "step_roofline_frac": step_gbs / HBM_PEAK_GBS,
        "hbm_copy_gbs": copy_gbs,
        "autotune": None if r64["default_ms"] is None else {
            "default_launch": "8x8x8 tiles, two waves per SIMD, grid launch (the plan's default)",
            "default_ms_per_step": r64["default_ms"], "tuned_ms_per_step": r64["ms"],
            "tuned_ge_default": bool(r64["ms"] <= r64["default_ms"]),
            "persistent_vs_grid": r64["queue"]},
        "fp64_flop_per_pt_stage": FLOP_PER_PT_STAGE,
        "fp64_alu_frac": value * FLOP_PER_PT_STAGE / (FP64_PEAK_TFLOPS * 1e12),
    }
    if "fp32" in results:
        r32 = results["fp32"]
        v32 = n_int * nstages / (r32["ms"] * 1e-3)
        out["fp32"] = {"value": v32, "unit": "pt-stage/s", "ms_per_step": r32["ms"],
                       "speedup_vs_fp64": v32 / value,
                       "stage_kernel_ms": r32["stage_ms"].round(4).tolist()}
        if not args.no_precision:
            out["fp32"]["precision_study"] = precision_leg(args.precision_steps)
            out["fp32"]["constraint_error"] = out["fp32"]["precision_study"]["constraint_error"]
            out["fp32"]["constraint_tolerance"] = FP32_H_TOLERANCE
    if not args.no_batching:
        out["batching"] = batching(stream, args.steps)
    if not args.no_lopsided:
        out["lopsided_advection"] = lopsided_timing(bt, stream, max(3, args.steps // 2),
                                                    r64["stage_ms"][1])
    if not args.no_sommerfeld:
        out["sommerfeld"] = sommerfeld_timing(stream, max(5, args.steps // 2))
    if not args.no_matter:
        out["matter_coupling"] = matter_coupling(stream, args.steps)
    if not args.no_intergrid:
        out["intergrid"] = intergrid_transfers(stream, args.steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(bt, args.cpu_sample_blocks)
    print(json.dumps(out), flush=True)


def step_time(plan, regs, bt, stream, warmup, steps):
    """ms per RK4 step of `plan` (graph replay), on copies of the registers."""
    import torch

    from paper_2311_04989_amd import z4c as Z

    r = [x.clone() for x in regs]
    for _ in range(max(1, warmup)):
        plan.step(r, None, Z.RK4, bt.dt, Z.GHOST_PERIODIC, graph=True, stream=stream,
                  flags=Z.STEP_NO_FINAL_FILL)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan.step(r, None, Z.RK4, bt.dt, Z.GHOST_PERIODIC, graph=True, stream=stream,
                  flags=Z.STEP_NO_FINAL_FILL)
    e1.record(stream)
    torch.cuda.synchronize()
    del r
    return e0.elapsed_time(e1) / steps


def stage2_time(plan, regs, bt, stream, reps):
    """Median ms of an RK4 stage-2 launch of `plan`."""
    import numpy as np
    import torch

    from paper_2311_04989_amd import z4c as Z

    out = torch.empty_like(regs[0])
    plan.rk_stage(regs[1], out, regs[3], regs[0], None, Z.RK4[1], bt.dt, stream=stream)
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.rk_stage(regs[1], out, regs[3], regs[0], None, Z.RK4[1], bt.dt, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del out
    return float(np.median(ms))


def lopsided_timing(bt, stream, reps, centred_ms):
    """RK4 stage 2 of the level set with lopsided advection stencils (its own
    plan, autotuned), against the centred stage of the main run."""
    import dataclasses

    import numpy as np
    import torch

    from paper_2311_04989_amd import z4c as Z

    params = dataclasses.replace(bt.params, advection=Z.ADVECT_LOPSIDED)
    plan = Z.Plan(Z.make_params(params), Z.make_blocks(bt.block_table()))
    u0 = torch.from_numpy(bt.u).to("cuda:0")
    plan.ghost_fill(Z.GHOST_PERIODIC, u0, stream=stream)
    plan.set_halo(Z.GHOST_PERIODIC)
    out, u1 = u0.clone(), torch.zeros_like(u0)
    plan.autotune(u0, out, u1, None, reps=3, stream=stream)
    fn = lambda: plan.rk_stage(u0, out, u1, u0, None, Z.RK4[1], bt.dt, stream=stream)  # noqa: E731
    fn()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    med = float(np.median(ms))
    res = {"stage_ms": med, "centred_stage_ms": centred_ms, "ratio": med / centred_ms,
           "launch_shapes": {str(k): plan.get_launch(k, k, k) for k in (8, 16, 24, 32)},
           "achieved_gbs": bt.ninterior * STAGE_BYTES[1] / (med * 1e-3) / 1e9}
    plan.close()
    log(f"[bench] lopsided advection: {res}")
    return res


def sommerfeld_timing(stream, reps):
    """The radiative outer boundary on the star level set (8 blocks of 128^3
    + 4 ghosts tiling [-16, 16]^3): one radiative stage of the outer ghost
    points (RK4 stage 2: reads u0, u1, u2, writes u1, u0', 880 algorithmic B
    per point) against the fused interior stage of the same plan, medians
    over `reps` launches."""
    import numpy as np
    import torch

    from paper_2311_04989_amd import workloads as W
    from paper_2311_04989_amd import z4c as Z

    bt = W.config5()
    bt.frozen = None
    bt.sommerfeld = True
    nbr = np.asarray(bt.neighbours)
    outer = 0
    for b, blk in enumerate(bt.blocks):
        for d in range(27):
            if d == 13 or nbr[b, d] >= 0:
                continue
            o = (d % 3 - 1, (d // 3) % 3 - 1, d // 9 - 1)
            n = (blk.nx, blk.ny, blk.nz)
            outer += int(np.prod([blk.ng if o[a] else n[a] for a in range(3)]))
    plan = Z.plan_for(bt)
    plan.set_halo(Z.GHOST_NEIGHBOUR)
    u0 = torch.from_numpy(bt.u).to("cuda:0")
    m = torch.from_numpy(bt.matter).to("cuda:0")
    out, u1 = u0.clone(), u0.clone()
    calls = {
        "radiative_stage_ms": lambda: plan.sommerfeld_stage(u0, out, u1, u0, Z.RK4[1], bt.dt,
                                                            stream=stream),
        "interior_stage_ms": lambda: plan.rk_stage(u0, out, u1, u0, m, Z.RK4[1], bt.dt,
                                                   stream=stream),
    }
    res = {"workload": "star level set 8 x 128^3 + 4 ghosts tiling [-16, 16]^3, radiative "
                       "outer ghosts (every ghost region without a neighbour), RK4 stage 2",
           "outer_points": outer, "interior_points": bt.ninterior}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        res[name] = float(np.median(ms))
    res["algorithmic_bytes"] = outer * STAGE_BYTES[1]
    res["achieved_gbs"] = res["algorithmic_bytes"] / (res["radiative_stage_ms"] * 1e-3) / 1e9
    res["hbm_frac"] = res["achieved_gbs"] / HBM_PEAK_GBS
    res["cost_vs_interior_stage"] = res["radiative_stage_ms"] / res["interior_stage_ms"]
    plan.close()
    del u0, m, out, u1
    torch.cuda.empty_cache()
    log(f"[bench] radiative outer boundary: {res}")
    return res


def monitor_timing(plan, regs, bt, stream, reps):
    """RK4 stage 2 of the level set in the tuned shapes: plain, with the
    constraint monitor fused (constraint fields + per-block norms), and the
    separate constraint pass it replaces; medians over `reps`."""
    import numpy as np
    import torch

    from paper_2311_04989_amd import z4c as Z

    nb = len(bt.blocks)
    cons = torch.zeros(bt.total_c, dtype=torch.float64, device="cuda:0")
    norms = torch.zeros(16 * nb, dtype=torch.float64, device="cuda:0")
    calls = {
        "stage_ms": lambda: plan.rk_stage(regs[1], regs[2], regs[3], regs[0], None, Z.RK4[1],
                                          bt.dt, stream=stream),
        "stage_with_monitor_ms": lambda: plan.rk_stage_monitor(
            regs[1], regs[2], regs[3], regs[0], None, Z.RK4[1], bt.dt, cons, norms,
            stream=stream),
        "separate_constraints_ms": lambda: plan.constraints(regs[1], None, cons, norms,
                                                            stream=stream),
    }
    out = {}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        out[name] = float(np.median(ms))
    out["monitor_cost_ms"] = out["stage_with_monitor_ms"] - out["stage_ms"]
    out["monitor_cost_vs_separate_pass"] = out["monitor_cost_ms"] / out["separate_constraints_ms"]
    log(f"[bench] constraint monitor: {out}")
    return out


def profile_run(launches, stream, arith="fp64"):
    """What the committed counter profiles ran: a device copy of 2^27 doubles
    (1 GiB read, 1 GiB written) to calibrate FETCH_SIZE / WRITE_SIZE, then RK4
    stage 2 (reads u0, u1, u2; writes u1, u0') of the uneven level set with
    ghosts read through the periodic rule, in the autotuned launch shapes, with
    FP64 or FP32 arithmetic."""
    import torch

    from paper_2311_04989_amd import workloads as W
    from paper_2311_04989_amd import z4c as Z

    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    bt = W.config4()
    plan = Z.plan_for(bt, Z.ARITH_FP32 if arith == "fp32" else Z.ARITH_FP64)
    u = torch.from_numpy(bt.u).to("cuda:0")
    regs = [u.clone(), u.clone(), u.clone(), u.clone()]
    plan.ghost_fill(Z.GHOST_PERIODIC, regs[0], stream=stream)
    plan.set_halo(Z.GHOST_PERIODIC)
    plan.autotune(regs[0], regs[1], regs[3], None, reps=3, stream=stream)
    torch.cuda.synchronize()
    shapes = {s: plan.get_launch(s, s, s) for s in (8, 16, 24, 32)}
    log(f"[profile] {arith}: launch shapes {shapes}; {launches} launches of RK4 stage 2")
    for _ in range(launches):
        plan.rk_stage(regs[0], regs[1], regs[3], regs[2], None, Z.RK4[1], bt.dt, stream=stream)
    torch.cuda.synchronize()
    log("[profile] done")


def batching(stream, reps):
    """One fused RK4 stage of 512 MeshBlocks of 16^3 (4 ghosts, 6th order,
    gauge wave + noise): 512 per-block launches (one plan per block, the
    same arrays) vs one grid launch of all tiles vs one persistent launch."""
    import numpy as np
    import torch

    from paper_2311_04989_amd import workloads as W
    from paper_2311_04989_amd import z4c as Z

    bt = W.config3()
    n_int = bt.ninterior
    u = torch.from_numpy(bt.u).to("cuda:0")
    out = torch.empty_like(u)
    u1 = torch.zeros_like(u)
    c = Z.RK4[0]
    plan = Z.plan_for(bt)
    params = Z.make_params(bt.params, Z.ARITH_FP64)
    tab = bt.block_table()
    singles = [Z.Plan(params, Z.make_blocks(tab[i:i + 1])) for i in range(len(bt.blocks))]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms)), float(np.min(ms))

    def per_block():
        for p in singles:
            p.rk_stage(u, out, u1, u, None, c, bt.dt, stream=stream)

    def whole():
        plan.rk_stage(u, out, u1, u, None, c, bt.dt, stream=stream)

    res = {"workload": "512 MeshBlocks 16^3 + 4 ghosts, 6th-order FD, gauge wave + 1e-10 noise, "
                       "one fused RHS+RK4 stage (stored ghosts)",
           "interior_points": n_int}
    log("[bench] batching: 512 per-block launches")
    res["per_block_launches_ms"] = timed(per_block)
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    # every launch shape as a grid launch and as a persistent (work-queue)
    # launch of one and two workgroups per CU
    shapes = {}
    for tile, waves in (((8, 8, 8), 2), ((8, 8, 4), 2), ((8, 8, 4), 1), ((8, 4, 8), 1)):
        row = {}
        for pers in (0, ncu, 2 * ncu):
            plan.set_launch(16, 16, 16, tile, pers, waves)
            row["grid" if pers == 0 else f"persistent_{pers}"] = timed(whole)
        shapes["x".join(map(str, tile)) + f"_w{waves}"] = row
    best_key = min(shapes, key=lambda k: shapes[k]["grid"][0])
    best = shapes[best_key]
    pers_best = min((v for k, v in best.items() if k != "grid"), key=lambda v: v[0])
    res["launch_shapes_ms"] = shapes
    res["grid_launch_ms"] = best["grid"]
    res["persistent_launch_ms"] = pers_best
    res["best_shape"] = best_key
    res["persistent_le_grid"] = bool(pers_best[0] <= best["grid"][0] * 1.01)
    res["note"] = ("(median, min) over the timed repetitions, ms per stage; grid and "
                   "persistent compared in the shape whose grid launch is fastest; "
                   "persistent_le_grid allows 1 % timing noise")
    res["pt_stage_per_s"] = {k[:-3]: n_int / (res[k][0] * 1e-3)
                             for k in ("per_block_launches_ms", "grid_launch_ms",
                                       "persistent_launch_ms")}
    log(f"[bench] batching: {res}")
    for p in singles:
        p.close()
    plan.close()
    return res


def matter_coupling(stream, reps):
    """The matter coupling on the level set of 8 blocks of 128^3 cells (129^3
    vertices, 4 ghost vertices, 3 ghost cells): chi and gt_ij to the cells and
    their three ghost layers (order 4), GRMHD ADM sources there, sources back
    to the vertices (order 6).  Each launch timed alone (median, min of
    `reps`), and the three in sequence; HBM roofline of each from its
    algorithmic bytes (every input value read once, every output written
    once)."""
    import numpy as np
    import torch

    from paper_2311_04989_amd import workloads as W
    from paper_2311_04989_amd import z4c as Z

    t0 = time.time()
    mb = W.matter_level_set()
    log(f"[bench] matter coupling: generated {mb.name} in {time.time() - t0:.1f}s")
    plan = Z.mplan_for(mb)
    dev = lambda a: torch.from_numpy(a).to("cuda:0")   # noqa: E731
    u, prim = dev(mb.u), dev(mb.prim)
    geom, adm = torch.zeros(mb.geom.size, dtype=torch.float64, device="cuda:0"), \
        torch.zeros(mb.adm.size, dtype=torch.float64, device="cuda:0")
    matter = torch.zeros(mb.matter.size, dtype=torch.float64, device="cuda:0")
    calls = {
        "metric_to_cc": lambda: plan.metric_to_cc(4, 3, u, geom, stream=stream),
        "adm_sources": lambda: plan.adm_sources(1, 2.0, 1e-6, 3, geom, prim, adm, stream=stream),
        "sources_to_vc": lambda: plan.sources_to_vc(6, adm, matter, stream=stream),
    }
    nvs = sum(int(np.prod(b.vshape)) for b in mb.blocks)              # stored vertices
    ncs = sum(int(np.prod(b.cshape)) for b in mb.blocks)              # stored cells
    nv = mb.nvertices
    algo = {"metric_to_cc": 8 * (7 * nvs + 7 * ncs),                  # every stored vertex read
            "adm_sources": 8 * (7 + 8 + 10) * ncs,
            "sources_to_vc": 8 * (10 * ncs + 10 * nv)}
    res = {"workload": mb.name + "; metric order 4 to the cells and 3 ghost layers, GRMHD "
                                 "sources (Gamma = 2), sources order 6 to the vertices; "
                                 "primitive recovery (ideal gas, Gamma = 2) on the same cells",
           "cells": mb.ncells, "vertices": nv}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms)), float(np.min(ms))

    for name, fn in calls.items():
        med, mn = timed(fn)
        gbs = algo[name] / (med * 1e-3) / 1e9
        res[name] = {"ms": (med, mn), "algorithmic_bytes": algo[name], "achieved_gbs": gbs,
                     "hbm_frac": gbs / HBM_PEAK_GBS}
    med, mn = timed(lambda: [fn() for fn in calls.values()])
    res["chain"] = {"ms": (med, mn), "vertices_per_s": nv / (med * 1e-3),
                    "hbm_frac": sum(algo.values()) / (med * 1e-3) / 1e9 / HBM_PEAK_GBS}
    # primitive recovery at the cells and their 3 ghost layers: conservatives
    # of the level set's primitives (z4c_p2c), then z4c_c2p (the generator's
    # vacuum cells become atmosphere on the first call; repeated calls find
    # the same state)
    c = Z.c2p_params(mhd=1, gamma_ad=2.0, rho_atm=1e-12)
    cons = torch.zeros(mb.cons.size, dtype=torch.float64, device="cuda:0")
    out = torch.zeros(mb.prim.size, dtype=torch.float64, device="cuda:0")
    status = torch.zeros(mb.status.size, dtype=torch.int32, device="cuda:0")
    algo_p2c = 8 * (7 + 8 + 8) * ncs
    algo_c2p = (8 * (7 + 8 + 8) + 4) * ncs
    for name, fn, nb in (("p2c", lambda: plan.p2c(c, 3, geom, prim, cons, stream=stream), algo_p2c),
                         ("c2p", lambda: plan.c2p(c, 3, geom, cons, out, status, stream=stream),
                          algo_c2p)):
        med, mn = timed(fn)
        gbs = nb / (med * 1e-3) / 1e9
        res[name] = {"ms": (med, mn), "algorithmic_bytes": nb, "achieved_gbs": gbs,
                     "hbm_frac": gbs / HBM_PEAK_GBS, "cells_per_s": ncs / (med * 1e-3)}
    st = status.cpu().numpy()
    res["c2p"]["status_counts"] = {str(k): int(v) for k, v in zip(*np.unique(st, return_counts=True))}
    log(f"[bench] matter coupling: {res}")
    plan.close()
    return res


def _footprint(t, order, prolong):
    """Stored source points one transfer reads (the product over directions of
    the index range its destination box reaches)."""
    n = 1
    for d in range(3):
        idx = set()
        for i in range(t["lo"][d], t["hi"][d]):
            if not prolong:
                idx.add(2 * (i - t["c0"][d]))
            elif i % 2 == 0:
                idx.add(t["c0"][d] + i // 2)
            else:
                left = t["c0"][d] + (i - 1) // 2
                idx.update(range(left - (order // 2 - 1), left + order // 2 + 1))
        n *= len(idx)
    return n


def intergrid_transfers(stream, reps, order=6):
    """Transfers of a level jump at scale (64 coarse and 512 fine blocks of
    16^3 + 4 ghosts): prolongation (order 6) of the six face slabs of every
    fine block, restriction (injection) of every fine block into its octant.
    Algorithmic bytes of a transfer: its destination box written once and
    the source points its box reaches read once (22 fields, FP64)."""
    import numpy as np
    import torch

    from paper_2311_04989_amd import workloads as W
    from paper_2311_04989_amd import z4c as Z

    t0 = time.time()
    bt, pro, res = W.level_jump()
    log(f"[bench] intergrid: generated {bt.name} in {time.time() - t0:.1f}s")
    plan = Z.plan_for(bt)
    xp = Z.XPlan(plan, pro, res, order)
    u = torch.from_numpy(bt.u).to("cuda:0")
    box = lambda t: int(np.prod([h - l for l, h in zip(t["lo"], t["hi"])]))   # noqa: E731
    npro = sum(box(t) for t in pro)
    nres = sum(box(t) for t in res)
    algo = {"prolongate": 8 * 22 * (npro + sum(_footprint(t, order, True) for t in pro)),
            "restrict": 8 * 22 * (nres + sum(_footprint(t, order, False) for t in res))}
    calls = {"prolongate": lambda: xp.prolongate(u, stream=stream),
             "restrict": lambda: xp.restrict(u, stream=stream)}
    out = {"workload": bt.name + f"; prolongation order {order}, restriction by injection",
           "prolongated_points": npro, "restricted_points": nres}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        med = float(np.median(ms))
        gbs = algo[name] / (med * 1e-3) / 1e9
        out[name] = {"ms": (med, float(np.min(ms))), "algorithmic_bytes": algo[name],
                     "achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    log(f"[bench] intergrid: {out}")
    xp.close()
    plan.close()
    return out


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def config_table(stream, reps, warmup):
    """Every workload configuration on the GPU, FP64 and FP32 arithmetic,
    (median, min) ms over `reps` timed repetitions after `warmup`:
    1: one RK4 step (4 fused stages + periodic ghost refreshes) in a graph;
    2: one RHS and one RK4 stage-2 launch (reads u0, u1, u2);
    3: one RK4 stage-2 launch over the 512 blocks;
    4: one RK4 step, ghosts read through the periodic rule, in a graph;
    5: one RK4 step (neighbour copies + frozen outer ghosts) in a graph.
    The oracle (FP64, host) times one RK4 stage 2 on configurations 2-4,
    on one thread (a seeded sample of blocks for 3 and 4) and on all threads."""
    import numpy as np
    import torch

    import oracle as O
    from paper_2311_04989_amd import workloads as W
    from paper_2311_04989_amd import z4c as Z

    def dev(a):
        return None if a is None else torch.from_numpy(a).to("cuda:0")

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms)), float(np.min(ms))

    rows = {}
    nall = None
    for c in (1, 2, 3, 4, 5):
        t0 = time.time()
        bt = W.CONFIGS[c]()
        log(f"[table] config {c}: {bt.name}, {bt.ninterior} interior points "
            f"(generated in {time.time() - t0:.1f} s)")
        row = {"workload": bt.name, "interior_points": bt.ninterior}
        u, m, fz = dev(bt.u), dev(bt.matter), dev(bt.frozen)
        for arith, label in ((Z.ARITH_FP64, "fp64"), (Z.ARITH_FP32, "fp32")):
            plan = Z.plan_for(bt, arith)
            regs = [u.clone(), u.clone(), u.clone(), torch.zeros_like(u)]
            if c == 4:
                plan.ghost_fill(Z.GHOST_PERIODIC, regs[0], stream=stream)
                plan.set_halo(Z.GHOST_PERIODIC)
            plan.autotune(regs[0], regs[1], regs[3], m, reps=3, stream=stream)
            if c in (1, 4, 5):
                flags = Z.STEP_NO_FINAL_FILL if c == 4 else 0

                def step():
                    plan.step(regs, m, Z.RK4, bt.dt, bt.ghost, fz, stream=stream, graph=True,
                              flags=flags)
                med, mn = timed(step)
                row[label] = {"what": "RK4 step", "ms": (med, mn),
                              "pt_stage_per_s": 4 * bt.ninterior / (med * 1e-3)}
            else:
                def stage():
                    plan.rk_stage(regs[0], regs[1], regs[3], regs[2], m, Z.RK4[1], bt.dt,
                                  stream=stream)
                med, mn = timed(stage)
                row[label] = {"what": "RK4 stage 2", "ms": (med, mn),
                              "pt_stage_per_s": bt.ninterior / (med * 1e-3)}
                if c == 2:
                    out = torch.zeros_like(u)
                    rmed, rmn = timed(lambda: plan.rhs(regs[0], m, out, stream=stream))
                    row[label]["rhs_ms"] = (rmed, rmn)
                    row[label]["rhs_pt_per_s"] = bt.ninterior / (rmed * 1e-3)
            row[label]["nonfinite"] = plan.check_finite(regs[0], stream=stream)
            log(f"[table] config {c} {label}: {row[label]}")
            del regs
            plan.close()
        del u, m, fz
        torch.cuda.empty_cache()
        if c in (2, 3, 4):
            O.build(force=False)
            if nall is None:
                nall = O.max_threads()   # before any call sets a thread count
            row["oracle"] = {}
            rng = np.random.default_rng(11)
            for nthr, key in ((1, "1_thread"), (0, "all_threads")):
                if nthr == 1 and len(bt.blocks) > 1:
                    # a seeded sample of about 1/16 of the blocks, every size class
                    sizes = np.array([b.nx for b in bt.blocks])
                    idx = np.concatenate([
                        rng.choice(np.nonzero(sizes == s)[0],
                                   size=max(1, np.count_nonzero(sizes == s) // 16), replace=False)
                        for s in np.unique(sizes)])
                    sub = bt.subset(idx)
                else:
                    sub = bt
                y = sub.u.copy()
                u1 = sub.u.copy()
                out = sub.u.copy()
                t0 = time.time()
                O.rk_stage(sub, sub.u, out, u1, y, O.RK4[1], sub.dt, nthreads=nthr)
                dt = time.time() - t0
                row["oracle"][key] = {"pt_stage_per_s": sub.ninterior / dt, "seconds": dt,
                                      "interior_points": sub.ninterior,
                                      "threads": 1 if nthr == 1 else nall}
            log(f"[table] config {c} oracle: {row['oracle']}")
        rows[str(c)] = row
        del bt
    return {"table": "per-configuration throughput, pt-stage/s", "host": host_info(),
            "configs": rows}


def cpu_baseline(bt, nsample):
    """The FP64 oracle on the host cores: one RK4 step (4 stages + ghost
    refresh) of a seeded sample of the same level set's blocks."""
    import numpy as np

    import oracle as O

    O.build(force=False)
    rng = np.random.default_rng(7)
    sizes = np.array([b.nx for b in bt.blocks])
    if nsample <= 0 or nsample >= len(bt.blocks):
        idx = np.arange(len(bt.blocks))
    else:
        # the same share of every size class
        idx = np.concatenate([rng.choice(np.nonzero(sizes == s)[0],
                                         size=max(1, round(nsample * np.count_nonzero(sizes == s)
                                                           / len(bt.blocks))), replace=False)
                              for s in (8, 16, 24, 32)])
    sub = bt.subset(idx)
    O.ghost_fill(sub, sub.u)
    cores = O.max_threads()
    t0 = time.time()
    O.rk_step(sub, sub.u, dt=bt.dt)
    dt = time.time() - t0
    pts = sub.ninterior * 4
    # one thread, on a sixteenth of the sample (the same share of every size)
    idx1 = np.concatenate([rng.choice(np.nonzero(sizes == s)[0],
                                      size=max(1, np.count_nonzero(sizes[idx] == s) // 16),
                                      replace=False) for s in (8, 16, 24, 32)])
    sub1 = bt.subset(idx1)
    O.ghost_fill(sub1, sub1.u)
    t1 = time.time()
    O.rk_step(sub1, sub1.u, dt=bt.dt, nthreads=1)
    dt1 = time.time() - t1
    host = host_info()
    return {"value": pts / dt, "unit": "pt-stage/s", "cores": cores, "kind": "oracle",
            "cpu_model": host["cpu_model"], "nproc": host["nproc"],
            "value_1thread": sub1.ninterior * 4 / dt1,
            "sample": f"one RK4 step (4 stages + periodic ghost refresh) of {len(idx)} of the "
                      f"{len(bt.blocks)} blocks ({sub.ninterior} interior points) of the same "
                      f"level set, {dt:.1f} s on all threads; 1 thread: {len(idx1)} blocks "
                      f"({sub1.ninterior} interior points), {dt1:.1f} s"}


def precision_leg(steps):
    """The FP32 form against FP64 on the precision-study level set (8 blocks
    of 128^3, star metric with matter and 1e-6 noise, neighbour and frozen
    ghosts): `steps` RK4 steps of each; the relative L2 difference of their
    Hamiltonian-constraint fields at the end, against the stated tolerance."""
    import torch

    from paper_2311_04989_amd import precision_study as PS
    from paper_2311_04989_amd import workloads as W
    from paper_2311_04989_amd import z4c as Z

    stream = torch.cuda.current_stream()
    t0 = time.time()
    bt = W.config5()
    log(f"[bench] precision study level set generated in {time.time() - t0:.1f}s")
    every = max(1, steps // 4)
    r64, _, h64 = PS.evolve(bt, Z.ARITH_FP64, steps, every, stream)
    r32, _, _ = PS.evolve(bt, Z.ARITH_FP32, steps, every, stream, h_ref=h64)
    del h64
    end32, end64 = r32["history"][-1], r64["history"][-1]
    err = end32["dH_L2"] / end64["H_L2"]
    return {"workload": "8 MeshBlocks 128^3 + 4 ghosts tiling [-16,16]^3, star metric + matter "
                        "blobs + 1e-6 noise, neighbour + frozen outer ghosts, 6th-order FD, "
                        f"KO 0.5, {steps} RK4 steps of dt = dx/4, FP32 arithmetic vs FP64",
            "steps": steps,
            "constraint_error": err,
            "constraint_error_def": "||H_fp32 - H_fp64||_2 / ||H_fp64||_2 after the last step",
            "tolerance": FP32_H_TOLERANCE,
            "within_tolerance": bool(err <= FP32_H_TOLERANCE),
            "H_L2_fp64": [r64["history"][0]["H_L2"], end64["H_L2"]],
            "H_L2_fp32": [r32["history"][0]["H_L2"], end32["H_L2"]],
            "fp64_ms_per_step": r64["ms_per_step"], "fp32_ms_per_step": r32["ms_per_step"],
            "speedup_vs_fp64": r64["ms_per_step"] / r32["ms_per_step"],
            "nonfinite": [r64["nonfinite"], r32["nonfinite"]]}


if __name__ == "__main__":
    main()
