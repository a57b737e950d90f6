"""Throughput benchmark of the star-stencil hot path on one MI355X.

One bench step = the whole workload once: 2D star stencils of radius
1, 2, 3 and 4 (seeded per-point coefficients summing to 1, clamp boundary)
on a 16384 x 16384 FP32 grid of U[0,1) values, 1000 time steps per radius,
each radius with its plan's temporal degree K.  Inputs are resident in HBM
before timing starts.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-tune] [--no-3d]

Each plan is autotuned (every feasible kernel configuration timed at the
real shape) before the timed region.  A secondary leg measures the 3D
workload (512^3, radius 1..4, 200 steps each) the same way and reports it
under "extra".

value: whole-job cell updates per second (GCell/s, Eq. (3) of the paper read
as cells*iterations/time), summed over the four radii.
roofline: the dominant kernel (the radius whose passes take longest),
measured with HIP events on the launch stream: algorithmic HBM bytes (8 per
cell per pass) or FLOP (8r+1 per cell update, Table I) per launch over the
average launch duration, against MI355X peaks.
cpu_baseline: the FP64 CPU oracle on a bounded sample (2 steps per radius on
the same grid), on the host's cores.
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

METRIC = "GCell/s & GFLOP/s, 2D/3D star r=1–4, FP32 vs FP16-store, % HBM roofline"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
SIDE = 16384
TIME_STEPS = 1000
RADII = (1, 2, 3, 4)


def flop_per_cell(ndim: int, radius: int) -> int:
    return 8 * radius + 1 if ndim == 2 else 12 * radius + 1


def cpu_baseline(f0, coeffs_by_r, sample_steps: int = 2):
    """The FP64 oracle, unchanged, timed on the host: sample_steps steps per
    radius on the full grid."""
    from oracle import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    f64 = f0.astype("float64")
    cells = f0.size
    t = 0.0
    for r, c in coeffs_by_r.items():
        t0 = time.perf_counter()
        oracle.star_run_f64(f64, c, r, sample_steps, threads=threads)
        t += time.perf_counter() - t0
    updates = cells * sample_steps * len(coeffs_by_r)
    return {"value": round(updates / t / 1e9, 4), "unit": "GCell/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"FP64 oracle, {sample_steps} steps at each radius "
                      f"{list(coeffs_by_r)} on the full {SIDE}x{SIDE} grid "
                      f"({updates:.3e} cell updates in {t:.1f} s)"}


def bench_3d(stencil, synth, torch, dev, side=512, time_steps=200, reps=2, tune=True):
    """3D star stencils r=1..4 on side^3 FP32 (U[0,1)), time_steps steps each."""
    shape = (side, side, side)
    x = torch.from_numpy(synth.grid_uniform(2, shape)).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)
    rows, tot_ms = [], 0.0
    for r in RADII:
        p = stencil.Plan(shape, r, synth.coefficients(2000 + r, 3, r))
        if tune:
            p.autotune(x, y, stream=stream)
        p.run(x, y, time_steps, stream=stream)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(dev)
        a.record(stream)
        for _ in range(reps):
            p.run(x, y, time_steps, stream=stream)
        b.record(stream)
        torch.cuda.synchronize(dev)
        ms = a.elapsed_time(b) / reps
        tot_ms += ms
        gc = x.numel() * time_steps / (ms / 1e3) / 1e9
        rows.append({"radius": r, "ms": round(ms, 3), "GCell/s": round(gc, 1),
                     "GFLOP/s": round(gc * flop_per_cell(3, r), 1),
                     "pct_hbm_roofline": round(100 * gc * 8 / PEAK_HBM_GBS, 1),
                     "config": p.describe()})
        p.close()
    total = x.numel() * time_steps * len(RADII) / (tot_ms / 1e3) / 1e9
    return {"workload": f"3D star stencils r=1..4, {side}^3 FP32 U[0,1), {time_steps} steps per "
                        f"radius, clamp", "GCell/s": round(total, 1), "per_radius": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="use the plans' default configurations")
    ap.add_argument("--no-3d", action="store_true", help="skip the secondary 3D leg")
    ap.add_argument("--side", type=int, default=SIDE, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2002_05983_amd import stencil, synth

    dev = torch.device("cuda:0")
    side = args.side
    shape = (side, side)
    f0 = synth.grid_uniform(1, shape)
    coeffs = {r: synth.coefficients(1000 + r, 2, r) for r in RADII}
    x = torch.from_numpy(f0).to(dev)
    y = torch.empty_like(x)
    plans = {r: stencil.Plan(shape, r, coeffs[r]) for r in RADII}
    stream = torch.cuda.current_stream(dev)
    if not args.no_tune:
        for r in RADII:
            plans[r].autotune(x, y, stream=stream)

    def one_step(record=None):
        for r in RADII:
            if record is not None:
                record[r][0].record(stream)
            plans[r].run(x, y, TIME_STEPS, stream=stream)
            if record is not None:
                record[r][1].record(stream)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize(dev)

    events = [{r: (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for r in RADII} for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    t_start.record(stream)
    for k in range(args.steps):
        one_step(events[k])
    t_end.record(stream)
    torch.cuda.synchronize(dev)
    total_ms = t_start.elapsed_time(t_end)
    ms_per_step = total_ms / args.steps
    cells = side * side
    updates_per_step = cells * TIME_STEPS * len(RADII)
    value = updates_per_step * args.steps / (total_ms / 1e3) / 1e9

    per_radius = []
    dominant = None
    for r in RADII:
        ms = sum(ev[r][0].elapsed_time(ev[r][1]) for ev in events) / args.steps
        q = plans[r].query()
        K = q["K"]
        npass = -(-TIME_STEPS // K)
        gc = cells * TIME_STEPS / (ms / 1e3) / 1e9
        row = {"radius": r, "K": K, "tile": q["tile"][:2], "ms": round(ms, 3),
               "GCell/s": round(gc, 1), "GFLOP/s": round(gc * flop_per_cell(2, r), 1),
               "eff_GB/s": round(gc * 8, 1), "pct_hbm_roofline": round(100 * gc * 8 / PEAK_HBM_GBS, 1),
               "passes": npass, "ms_per_pass": round(ms / npass, 4),
               "config": plans[r].describe()}
        per_radius.append(row)
        if dominant is None or ms > dominant["ms"]:
            dominant = row
    # roofline of the dominant kernel: one launch = one pass of K steps
    r, K, launch_s = dominant["radius"], dominant["K"], dominant["ms_per_pass"] / 1e3
    hbm_gbs = cells * 8 / launch_s / 1e9
    alu_tflops = cells * K * flop_per_cell(2, r) / launch_s / 1e12
    hbm_frac, alu_frac = hbm_gbs / PEAK_HBM_GBS, alu_tflops / PEAK_FP32_TFLOPS
    if hbm_frac >= alu_frac:
        roofline = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(hbm_frac, 4), "traffic": None}
    else:
        roofline = {"bound": "alu", "achieved": round(alu_tflops, 2), "peak": PEAK_FP32_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(alu_frac, 4), "traffic": None}
    roofline["kernel"] = f"star2d_stream R={r} K={K}"
    roofline["other"] = {"hbm_GB/s": round(hbm_gbs, 1), "hbm_frac": round(hbm_frac, 4),
                         "alu_TFLOP/s": round(alu_tflops, 2), "alu_frac": round(alu_frac, 4)}

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GCell/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D star stencils r=1..4, {side}x{side} FP32 grid U[0,1), "
                               f"seeded coefficients summing to 1, clamp boundary, "
                               f"{TIME_STEPS} steps per radius, temporal degree per plan",
                   "radii": list(RADII), "grid": [side, side], "time_steps": TIME_STEPS},
        "gflops": round(sum(p["GFLOP/s"] * p["ms"] for p in per_radius) /
                        sum(p["ms"] for p in per_radius), 1),
        "per_radius": per_radius,
        "roofline": roofline,
    }
    for p in plans.values():
        p.close()
    del x, y
    torch.cuda.empty_cache()
    if not args.no_3d:
        out["extra"] = {"3d": bench_3d(stencil, synth, torch, dev, tune=not args.no_tune)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(f0, coeffs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
