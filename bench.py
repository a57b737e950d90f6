"""Throughput benchmark of the star-stencil hot path on one MI355X.

One bench step = the whole workload once: 2D star stencils of radius
1, 2, 3 and 4 (seeded per-point coefficients summing to 1, clamp boundary)
on a 16384 x 16384 FP32 grid of U[0,1) values, 1000 time steps per radius,
each radius with its plan's temporal degree K.  Inputs are resident in HBM
before timing starts.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-tune] [--no-3d]
                  [--no-single] [--no-high] [--no-precision] [--no-batch]

Each plan is autotuned (every feasible kernel configuration timed at the
real shape) before the timed region.  Secondary legs, reported under
"extra": plain single-step (K=1) sweeps of the 2D grid and a 512^3 grid
against the HBM peak and a device copy; 2D radius 5..8 on the same grid
(200 steps each) and 3D radius 5..8 on 512^3 (50 steps each); the 3D workload
(512^3, radius 1..4, 200 steps each) measured the same way; the precision form (768^3 radius 4, 1000 steps, FP32 against
FP16/BF16 storage re-anchored every 10 or 50 steps, with errors); and the
batched form (256 mixed 2D/3D grids, 100 steps, one captured batch against
256 single-grid runs).

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
# FP32 vector peaks: 157.3 TFLOP/s is the published figure, reached only by
# packed (two-wide) FP32 instructions, which this library does not emit; its
# kernels issue plain v_fma_f32: 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x
# 2.4 GHz = 78.6 TFLOP/s, the ceiling the ALU roofline is measured against.
PEAK_FP32_PACKED_TFLOPS = 157.3
PEAK_FMA_TFLOPS = 78.6
SIDE = 16384
TIME_STEPS = 1000
RADII = (1, 2, 3, 4)


# HBM traffic of the dominant 2D kernel from rocprofv3 counters (FETCH_SIZE
# and WRITE_SIZE, separate runs, each scaled by its reading for a plain copy
# of known size).  Used only while the kernel's sources are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "star2d_stream_16384sq_pmc_traffic.txt")
KERNEL_SOURCES = ("star2d.hip", "star2d_body.hpp", "common.hpp", "launch.hpp")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2002_05983_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """Counter-measured HBM bytes per launch of `kernel`, or None when no
    record is for this configuration or the record is older than the source.
    Records are blocks of "key: value" lines, each opened by a "kernel:" line."""
    try:
        recs, rec = [], None
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" not in line or line.startswith("#"):
                    continue
                k, v = (t.strip() for t in line.split(":", 1))
                if k == "kernel":
                    rec = {}
                    recs.append(rec)
                if rec is not None:
                    rec[k] = v
        src = kernel_source_hash()
        for rec in recs:
            if rec.get("kernel") == kernel and rec.get("source_sha256") == src:
                return float(rec["traffic_bytes_per_launch"])
        return None
    except (OSError, KeyError, ValueError):
        return None


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def flop_per_cell(ndim: int, radius: int) -> int:
    return 8 * radius + 1 if ndim == 2 else 12 * radius + 1


def cpu_baseline(f0, coeffs_by_r, sample_steps: int = 40):
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


def model_accuracy(plan, rows):
    """The analytic model against the autotuner's measurements of every
    candidate: median |predicted/measured - 1|, Spearman rank correlation,
    and the measured rate of the model's pick over the measured best."""
    import numpy as np
    pred, meas = [], []
    for cfg, g in rows:
        try:
            pred.append(plan.model(cfg)["GCell/s"])
            meas.append(g)
        except Exception:
            continue
    if len(meas) < 2:
        return None
    pred, meas = np.array(pred), np.array(meas)
    rp, rm = pred.argsort().argsort(), meas.argsort().argsort()
    rho = float(np.corrcoef(rp, rm)[0, 1])
    return {"candidates": len(meas), "median_abs_err": round(float(np.median(np.abs(pred / meas - 1))), 4),
            "spearman": round(rho, 3), "pick_over_best": round(float(meas[pred.argmax()] / meas.max()), 4)}


def bench_3d(stencil, synth, torch, dev, side=512, time_steps=200, reps=2, tune=True):
    """3D star stencils r=1..4 on side^3 FP32 (U[0,1)), time_steps steps each."""
    shape = (side, side, side)
    x = torch.from_numpy(synth.grid_uniform(2, shape)).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)
    rows, tot_ms = [], 0.0
    for r in RADII:
        p = stencil.Plan(shape, r, synth.coefficients(2000 + r, 3, r))
        acc = None
        if tune:
            acc = model_accuracy(p, p.autotune(x, y, stream=stream))
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
        err = fp64_error(stencil, torch, y, f"3d512_r{r}", stream) if (side, time_steps) == (512, 200) else None
        rows.append({"radius": r, "ms": round(ms, 3), "GCell/s": round(gc, 1),
                     "GFLOP/s": round(gc * flop_per_cell(3, r), 1),
                     "pct_hbm_roofline": round(100 * gc * 8 / PEAK_HBM_GBS, 1),
                     "config": p.describe(), "model_GCell/s": round(p.model()["GCell/s"], 1),
                     "model_accuracy": acc, "fp64": err})
        p.close()
    total = x.numel() * time_steps * len(RADII) / (tot_ms / 1e3) / 1e9
    return {"workload": f"3D star stencils r=1..4, {side}^3 FP32 U[0,1), {time_steps} steps per "
                        f"radius, clamp", "GCell/s": round(total, 1), "per_radius": rows}


def bench_2d_high(stencil, synth, torch, dev, side=SIDE, time_steps=200, reps=2, tune=True):
    """2D star stencils r=5..8 on side^2 FP32 (U[0,1)), time_steps steps each:
    the radii past the paper's four, where it expects temporal blocking to
    keep paying off in 2D (Sec. VI.A)."""
    shape = (side, side)
    x = torch.from_numpy(synth.grid_uniform(1, shape)).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)
    rows, tot_ms = [], 0.0
    radii = (5, 6, 7, 8)
    for r in radii:
        p = stencil.Plan(shape, r, synth.coefficients(1000 + r, 2, r))
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
        rows.append({"radius": r, "K": p.query()["K"], "ms": round(ms, 3), "GCell/s": round(gc, 1),
                     "GFLOP/s": round(gc * flop_per_cell(2, r), 1),
                     "pct_hbm_roofline": round(100 * gc * 8 / PEAK_HBM_GBS, 1),
                     "config": p.describe()})
        p.close()
    total = x.numel() * time_steps * len(radii) / (tot_ms / 1e3) / 1e9
    return {"workload": f"2D star stencils r=5..8, {side}x{side} FP32 U[0,1), {time_steps} steps "
                        f"per radius, clamp", "GCell/s": round(total, 1), "per_radius": rows}


def bench_single_step(stencil, synth, torch, dev, side2=SIDE, side3=512, time_steps=20, reps=3):
    """Plain single-step sweeps (K = 1: one read and one write of the grid per
    step, 8 B per cell update): 2D r=1..4 on side2^2 and 3D r=1..4 on side3^3,
    FP32 U[0,1), each radius in the best of a few K = 1 configurations, as
    fractions of the 8 TB/s HBM peak and of a plain device copy of the same
    grid timed alongside."""
    def timed(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(dev)
        a.record(torch.cuda.current_stream(dev))
        for _ in range(reps):
            fn()
        b.record(torch.cuda.current_stream(dev))
        torch.cuda.synchronize(dev)
        return a.elapsed_time(b) / reps
    out = {}
    for ndim, shape in ((2, (side2, side2)), (3, (side3, side3, side3))):
        x = torch.from_numpy(synth.grid_uniform(ndim, shape)).to(dev)
        y = torch.empty_like(x)
        copy_gbs = 2 * x.numel() * 4 / (timed(lambda: y.copy_(x)) / 1e3) / 1e9
        rows = []
        if ndim == 2:
            cands = [f"k=1,ly={ly}" for ly in (64, 128, 256)]
        else:
            cands = [f"k=1,wl={wl},vec={v},nw={nw},lz={lz}" for wl, v in ((32, 4), (64, 4), (64, 8))
                     for nw in (12, 16) for lz in (64, 128, 256)]
            cands += [f"k=1,rows={rows},nbp={nbp},lz={lz}" for rows in (1, 2, 4) for nbp in (0, 1)
                      for lz in (32, 64, 128) if not (rows == 4 and nbp)]
        for r in RADII:
            c = synth.coefficients(3000 + 10 * ndim + r, ndim, r)
            # best of the K = 1 configurations, timed on this grid
            best = None
            for cfg in cands:
                try:
                    p = stencil.Plan(shape, r, c, tune=cfg)
                except Exception:
                    continue  # rejected for this radius (e.g. 8 cells per lane)
                try:
                    ms = timed(lambda: p.run(x, y, time_steps))
                except Exception:
                    ms = None
                p.close()
                if ms is not None and (best is None or ms < best[0]):
                    best = (ms, cfg)
            p = stencil.Plan(shape, r, c, tune=best[1])
            ms = timed(lambda: p.run(x, y, time_steps))
            gc = x.numel() * time_steps / (ms / 1e3) / 1e9
            rows.append({"radius": r, "GCell/s": round(gc, 1), "GB/s": round(gc * 8, 1),
                         "pct_hbm_roofline": round(100 * gc * 8 / PEAK_HBM_GBS, 1),
                         "pct_of_copy": round(100 * gc * 8 / copy_gbs, 1), "config": p.describe()})
            p.close()
        out[f"{ndim}d"] = {"grid": list(shape), "copy_GB/s": round(copy_gbs, 1), "per_radius": rows}
        del x, y
        torch.cuda.empty_cache()
    out["workload"] = (f"single-step (K=1) FP32 sweeps, {time_steps} steps: 2D r=1..4 on "
                       f"{side2}^2, 3D r=1..4 on {side3}^3, U[0,1) grids, clamp")
    return out


def bench_3d_high(stencil, synth, torch, dev, side=512, time_steps=50, reps=2, tune=True):
    """3D star stencils r=5..8 on side^3 FP32 (U[0,1)), time_steps steps each:
    single-step passes only (the streaming kernel at k = 1 or the
    one-thread-per-cell kernel, whichever the autotuner measures faster)."""
    shape = (side, side, side)
    x = torch.from_numpy(synth.grid_uniform(2, shape)).to(dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)
    rows, tot_ms = [], 0.0
    radii = (5, 6, 7, 8)
    for r in radii:
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
    total = x.numel() * time_steps * len(radii) / (tot_ms / 1e3) / 1e9
    return {"workload": f"3D star stencils r=5..8, {side}^3 FP32 U[0,1), {time_steps} steps per "
                        f"radius, clamp, single-step passes", "GCell/s": round(total, 1),
            "per_radius": rows}


def bench_forms(stencil, synth, torch, dev, side2=SIDE, side3=512, time_steps2=200,
                time_steps3=50, reps=2):
    """Shared coefficients and the padded-halo boundary next to the per-point
    clamp form, each pair in the same kernel configuration: 2D r=1..4 on
    side2^2 at K = min(4, 16/R) (the shared form is built up to K = 4) and
    3D r=1..4 on side3^3 in the single-step row layout (the one layout the
    3D shared form runs).  The padded grids keep the array the same size
    (interior side - 2R plus a frame of R cells per side, so rows stay 16-byte
    aligned); their rate counts the interior cells each step updates."""
    import numpy as np

    def timed(plan, x, y, steps):
        plan.run(x, y, steps)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(dev)
        a.record(torch.cuda.current_stream(dev))
        for _ in range(reps):
            plan.run(x, y, steps)
        b.record(torch.cuda.current_stream(dev))
        torch.cuda.synchronize(dev)
        return a.elapsed_time(b) / reps

    rows = []
    for ndim, side, steps in ((2, side2, time_steps2), (3, side3, time_steps3)):
        shape = (side,) * ndim
        for r in RADII:
            tune = f"k={min(4, 16 // r)},ly=64" if ndim == 2 else "k=1,rows=1,nbp=1,lz=128"
            c = synth.coefficients(4000 + 10 * ndim + r, ndim, r)
            w = 1.0 + synth.uniform01_f64(4100 + 10 * ndim + r, 1 + ndim * r)
            sym = (w / (w[0] + 2.0 * w[1:].sum())).astype(np.float32)
            row = {"ndim": ndim, "radius": r, "config": tune}
            for name, kw, coeffs in (("per_point", {}, c), ("shared", {"symmetric": True}, sym),
                                     ("padded", {"boundary": "padded"}, c)):
                inner = tuple(n - 2 * r for n in shape) if name == "padded" else shape
                p = stencil.Plan(inner, r, coeffs, tune=tune, **kw)
                x = torch.from_numpy(synth.grid_uniform(ndim, p.array_shape)).to(dev)
                y = torch.empty_like(x)
                ms = timed(p, x, y, steps)
                n_upd = int(np.prod(inner))
                row[f"{name}_GCell/s"] = round(n_upd * steps / (ms / 1e3) / 1e9, 1)
                p.close()
                del x, y
            row["shared_over_per_point"] = round(row["shared_GCell/s"] / row["per_point_GCell/s"], 3)
            row["padded_over_clamp"] = round(row["padded_GCell/s"] / row["per_point_GCell/s"], 3)
            rows.append(row)
        torch.cuda.empty_cache()
    return {"workload": f"per-point clamp vs shared coefficients vs padded halo, same configuration: "
                        f"2D r=1..4 {side2}^2 ({time_steps2} steps), 3D r=1..4 {side3}^3 "
                        f"({time_steps3} steps, row layout), FP32 U[0,1)", "rows": rows}


def read_fp64_reference(name):
    """Stored FP64 oracle values of a full-size workload at its full step
    count (tests/golden/fp64_<name>.txt): header fields, sampled cells
    (x, y[, z]) and their values; None when the file is absent."""
    path = os.path.join(ROOT, "tests", "golden", f"fp64_{name}.txt")
    if not os.path.exists(path):
        return None
    meta, cells, vals = {}, [], []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                parts = line[1:].split()
                if len(parts) >= 2 and parts[0] in ("maxabs", "sum", "steps", "radius"):
                    meta[parts[0]] = float(parts[1])
                continue
            t = line.split()
            cells.append([int(v) for v in t[:-1]])
            vals.append(float(t[-1]))
    return {"meta": meta, "cells": cells, "vals": vals}


def fp64_error(stencil, torch, y, name, stream=None):
    """Normwise relative L-infinity error of the GPU result y against the
    FP64 oracle on the stored cells (normalised by the FP64 grid's max |f|),
    and the relative difference of the two conservation sums (the GPU sum
    reduced in FP64 on the device)."""
    ref = read_fp64_reference(name)
    if ref is None:
        return None
    cells = ref["cells"]
    nd = len(cells[0])
    dims = list(y.shape[::-1])
    flat = [sum(c[a] * int(torch.tensor(dims[:a]).prod()) for a in range(nd)) for c in cells]
    got = y.reshape(-1)[torch.tensor(flat, device=y.device)].double().cpu()
    want = torch.tensor(ref["vals"], dtype=torch.float64)
    err = float((got - want).abs().max()) / ref["meta"]["maxabs"]
    _, _, total = stencil.reduce_f64(y, None, stream=stream)
    want_sum = ref["meta"]["sum"]
    return {"rel_linf_vs_fp64": err, "cells": len(cells), "sum": total, "sum_fp64": want_sum,
            "sum_rel_diff": abs(total - want_sum) / abs(want_sum)}


def read_precision_reference():
    """FP64 oracle values of the reduced precision workload (128^3, radius 4,
    1000 steps) on sampled cells, from the fixture its generator wrote."""
    path = os.path.join(ROOT, "tests", "golden", "precision_128cube_r4_1000.txt")
    maxabs, cells, vals = None, [], []
    with open(path) as fh:
        for line in fh:
            if line.startswith("# maxabs"):
                maxabs = float(line.split()[2])
            elif line.strip() and not line.startswith("#"):
                x, y, z, v = line.split()
                cells.append((int(x), int(y), int(z)))
                vals.append(float(v))
    return maxabs, cells, vals


def bench_precision(stencil, synth, torch, dev, side=768, time_steps=1000, radius=4,
                    anchors=(10, 50), reps=1, tune=True):
    """Precision form: FP32 against FP16/BF16 storage with re-anchoring every m
    steps, 3D radius 4 on the side^3 sinusoid grid.  Error vs the FP32 run on
    the full grid (FP64 reduction on the GPU), and vs the FP64 oracle on the
    sampled cells of the reduced 128^3 workload."""
    shape = (side, side, side)
    c = synth.coefficients(3004, 3, radius)
    x = torch.from_numpy(synth.sinusoid_grid(4, side)).to(dev)
    stream = torch.cuda.current_stream(dev)
    cells = x.numel()

    def timed(plan, y):
        if tune:
            plan.autotune(x, y, stream=stream)  # every form at its best configuration
        plan.run(x, y, 2, stream=stream)  # warm-up
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(dev)
        a.record(stream)
        for _ in range(reps):
            plan.run(x, y, time_steps, stream=stream)
        b.record(stream)
        torch.cuda.synchronize(dev)
        return a.elapsed_time(b) / reps

    full = (side, time_steps, radius) == (768, 1000, 4)
    p32 = stencil.Plan(shape, radius, c)
    ref = torch.empty_like(x)
    ms32 = timed(p32, ref)
    gc32 = cells * time_steps / (ms32 / 1e3) / 1e9
    rows = [{"storage": "f32", "m": None, "ms": round(ms32, 2), "GCell/s": round(gc32, 1),
             "config": p32.describe(),
             "fp64_768cube": fp64_error(stencil, torch, ref, "3d768sin_r4", stream) if full else None}]
    ref64 = ref.double()
    y = torch.empty_like(x)
    for storage in ("f16", "bf16", "f16-scaled", "bf16-scaled"):
        for m in anchors:
            p = stencil.Plan(shape, radius, c, storage=storage, anchor_m=m)
            ms = timed(p, y)
            md, mr, _ = stencil.reduce_f64(y, ref64, stream=stream)
            gc = cells * time_steps / (ms / 1e3) / 1e9
            rows.append({"storage": storage, "m": m, "ms": round(ms, 2), "GCell/s": round(gc, 1),
                         "speedup_vs_f32": round(gc / gc32, 3), "rel_linf_vs_f32": md / mr,
                         "config": p.describe(),
                         "fp64_768cube": fp64_error(stencil, torch, y, "3d768sin_r4", stream)
                         if full else None})
            p.close()
    del ref64, y, ref, x
    torch.cuda.empty_cache()
    # error against the FP64 oracle: reduced workload, stored sampled values
    maxabs, pts, want = read_precision_reference()
    n = 128
    xs = torch.from_numpy(synth.sinusoid_grid(4, n)).to(dev)
    ys = torch.empty_like(xs)
    idx = torch.tensor([(z * n + yy) * n + xx for xx, yy, z in pts], device=dev)
    wantt = torch.tensor(want, dtype=torch.float64, device=dev)
    fp64 = {}
    for storage, m in [("f32", 0)] + [(s_, m_) for s_ in ("f16", "bf16", "f16-scaled", "bf16-scaled")
                                      for m_ in anchors]:
        p = stencil.Plan((n, n, n), radius, c, storage=storage, anchor_m=m)
        p.run(xs, ys, time_steps, stream=stream)
        got = ys.view(-1)[idx].double()
        err = float((got - wantt).abs().max()) / maxabs
        fp64[storage if storage == "f32" else f"{storage}_m{m}"] = err
        p.close()
    for r in rows:
        key = r["storage"] if r["storage"] == "f32" else f"{r['storage']}_m{r['m']}"
        r["rel_linf_vs_fp64_128cube_sampled"] = fp64[key]
    p32.close()
    return {"workload": f"precision form: 3D star r={radius} on {side}^3 seeded sinusoid grid "
                        f"(8 modes + 1e-3 noise), {time_steps} steps, FP32 vs FP16/BF16 storage "
                        f"with per-64^3-tile power-of-two scales and FP32 arithmetic, re-anchored "
                        f"every m steps: anchored delta (f16, bf16) and scaled state "
                        f"(f16-scaled, bf16-scaled)",
            "fp64_error_workload": f"{n}^3, same recipe, {time_steps} steps, FP64 oracle on "
                                   f"{len(pts)} stored cells (8 corners + 248 drawn)",
            "rows": rows}


def bench_batch(stencil, synth, torch, dev, time_steps=100, reps=3, tune=True):
    """Batched form: 256 grids (128 2D with sides log-uniform in 64..4096,
    128 3D with sides log-uniform in 32..256, radius uniform in 1..4, U[0,1)
    values, seeded coefficients), 100 steps each, as one captured batch,
    against 256 separate stencil_run calls on the same stream."""
    shapes = synth.batch_shapes(5)
    stream = torch.cuda.current_stream(dev)
    plans, ins, outs, refs = [], [], [], []
    flop = 0
    for dims, radius, cseed, vseed in shapes:
        shape = tuple(reversed(dims))
        p = stencil.Plan(shape, radius, synth.coefficients(cseed, len(shape), radius))
        x = torch.from_numpy(synth.grid_uniform(vseed, shape)).to(dev)
        plans.append(p)
        ins.append(x)
        outs.append(torch.empty_like(x))
        refs.append(torch.empty_like(x))
        flop += x.numel() * time_steps * flop_per_cell(len(shape), radius)
    cells = sum(x.numel() for x in ins)

    def timed(fn):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(dev)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize(dev)
        return a.elapsed_time(b) / reps

    def per_grid():
        for p, x, r in zip(plans, ins, refs):
            p.run(x, r, time_steps, stream=stream)

    ms_pg = timed(per_grid)
    batch = stencil.Batch(plans, ins, outs, time_steps)
    if tune:
        batch.autotune(stream=stream)
    ms_b = timed(lambda: batch.launch(stream=stream))
    equal = all(torch.equal(o, r) for o, r in zip(outs, refs))
    desc = batch.describe()
    batch.close()
    for p in plans:
        p.close()
    gc = cells * time_steps / (ms_b / 1e3) / 1e9
    return {"workload": "256 grids: 128 2D (sides log-uniform 64..4096) + 128 3D (sides "
                        "log-uniform 32..256), radius uniform 1..4, FP32 U[0,1), seeded "
                        f"coefficients, {time_steps} steps each",
            "cells": cells, "ms": round(ms_b, 2), "GCell/s": round(gc, 1),
            "GFLOP/s": round(flop / (ms_b / 1e3) / 1e9, 1),
            "per_grid_ms": round(ms_pg, 2),
            "per_grid_GCell/s": round(cells * time_steps / (ms_pg / 1e3) / 1e9, 1),
            "speedup_vs_per_grid": round(ms_pg / ms_b, 2),
            "bitwise_equal_to_per_grid": bool(equal),
            "schedule": desc.splitlines()[0]}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="use the plans' default configurations")
    ap.add_argument("--no-3d", action="store_true", help="skip the secondary 3D leg")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision-form leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-high", action="store_true", help="skip the radius 5..8 legs")
    ap.add_argument("--no-single", action="store_true", help="skip the single-step (K=1) leg")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the shared-coefficient / padded-halo leg")
    ap.add_argument("--side", type=int, default=SIDE, help=argparse.SUPPRESS)
    ap.add_argument("--time-steps", type=int, default=TIME_STEPS, help=argparse.SUPPRESS)
    ap.add_argument("--config", action="append", default=[], metavar="R:TUNE", help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB FP32 buffer 4 times (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(a grid would shard along its slowest axis with K*R ghost rows per face "
              "and pass); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2002_05983_amd import stencil, synth

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        # a plain device copy of known size: 1 GiB read + 1 GiB written per launch
        a = torch.ones(1 << 28, device=dev)
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize(dev)
        print(json.dumps({"calibration": "copy", "bytes_read_per_launch": 1 << 30,
                          "bytes_written_per_launch": 1 << 30, "launches": 4}), flush=True)
        return
    time_steps = args.time_steps
    side = args.side
    shape = (side, side)
    f0 = synth.grid_uniform(1, shape)
    coeffs = {r: synth.coefficients(1000 + r, 2, r) for r in RADII}
    x = torch.from_numpy(f0).to(dev)
    y = torch.empty_like(x)
    # --config R:TUNE fixes a radius's configuration (profiling runs)
    fixed = {int(c.split(":", 1)[0]): c.split(":", 1)[1] for c in args.config}
    plans = {r: stencil.Plan(shape, r, coeffs[r], tune=fixed.get(r)) for r in RADII}
    stream = torch.cuda.current_stream(dev)
    accuracy = {}
    if not args.no_tune:
        for r in RADII:
            if r in fixed:
                continue
            accuracy[r] = model_accuracy(plans[r], plans[r].autotune(x, y, stream=stream))
            progress(f"2D radius {r} tuned: {plans[r].describe()}")

    def one_step(record=None):
        for r in RADII:
            if record is not None:
                record[r][0].record(stream)
            plans[r].run(x, y, time_steps, stream=stream)
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
    updates_per_step = cells * time_steps * len(RADII)
    value = updates_per_step * args.steps / (total_ms / 1e3) / 1e9

    # accuracy of the timed workload: each radius once more, against the
    # stored FP64 oracle values at the full step count (outside the timed region)
    fp64 = {}
    if (side, time_steps) == (SIDE, TIME_STEPS):
        for r in RADII:
            plans[r].run(x, y, time_steps, stream=stream)
            torch.cuda.synchronize(dev)
            fp64[r] = fp64_error(stencil, torch, y, f"2d16k_r{r}", stream)

    per_radius = []
    dominant = None
    for r in RADII:
        ms = sum(ev[r][0].elapsed_time(ev[r][1]) for ev in events) / args.steps
        q = plans[r].query()
        K = q["K"]
        npass = -(-time_steps // K)
        gc = cells * time_steps / (ms / 1e3) / 1e9
        row = {"radius": r, "K": K, "tile": q["tile"][:2], "ms": round(ms, 3),
               "GCell/s": round(gc, 1), "GFLOP/s": round(gc * flop_per_cell(2, r), 1),
               "eff_GB/s": round(gc * 8, 1), "pct_hbm_roofline": round(100 * gc * 8 / PEAK_HBM_GBS, 1),
               "passes": npass, "ms_per_pass": round(ms / npass, 4),
               "config": plans[r].describe(),
               "model_GCell/s": round(plans[r].model()["GCell/s"], 1),
               "model_accuracy": accuracy.get(r), "fp64": fp64.get(r),
               "seeds": {"grid": 1, "coefficients": 1000 + r}}
        per_radius.append(row)
        if dominant is None or ms > dominant["ms"]:
            dominant = row
    # roofline of the dominant kernel: one launch = one pass of K steps
    r, K, launch_s = dominant["radius"], dominant["K"], dominant["ms_per_pass"] / 1e3
    hbm_gbs = cells * 8 / launch_s / 1e9
    alu_tflops = cells * K * flop_per_cell(2, r) / launch_s / 1e12
    hbm_frac, alu_frac = hbm_gbs / PEAK_HBM_GBS, alu_tflops / PEAK_FMA_TFLOPS
    kernel = f"star2d_stream R={r} K={K} ly={dominant['tile'][1]} grid={side}x{side}"
    traffic = measured_traffic(kernel)
    # the bound is the ceiling the kernel is closest to
    if hbm_frac >= alu_frac:
        roofline = {"bound": "hbm", "achieved": round(hbm_gbs, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(hbm_frac, 4), "traffic": traffic}
    else:
        roofline = {"bound": "alu", "achieved": round(alu_tflops, 2), "peak": PEAK_FMA_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(alu_frac, 4), "traffic": traffic}
    roofline["kernel"] = kernel
    roofline["algorithmic_bytes_per_launch"] = cells * 8
    roofline["algorithmic_flop_per_launch"] = cells * K * flop_per_cell(2, r)
    roofline["source_sha256"] = kernel_source_hash()
    roofline["other"] = {"hbm_GB/s": round(hbm_gbs, 1), "hbm_frac": round(hbm_frac, 4),
                         "alu_TFLOP/s": round(alu_tflops, 2), "alu_frac": round(alu_frac, 4),
                         "alu_frac_of_packed_peak": round(alu_tflops / PEAK_FP32_PACKED_TFLOPS, 4)}

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
                               f"{time_steps} steps per radius, temporal degree per plan",
                   "radii": list(RADII), "grid": [side, side], "time_steps": time_steps},
        "gflops": round(sum(p["GFLOP/s"] * p["ms"] for p in per_radius) /
                        sum(p["ms"] for p in per_radius), 1),
        "per_radius": per_radius,
        "roofline": roofline,
        "accuracy": {
            "rel_linf_vs_fp64_max": max((v["rel_linf_vs_fp64"] for v in fp64.values() if v),
                                        default=None),
            "tolerance": 1e-5,
            "reference": "FP64 oracle at the full step count on stored cells "
                         "(tests/golden/fp64_2d16k_r*.txt), normalised by the FP64 grid's max |f|"},
    }
    for p in plans.values():
        p.close()
    del x, y
    torch.cuda.empty_cache()
    progress(f"2D: {value:.1f} GCell/s")
    extra = {}
    if not args.no_single:
        extra["single_step"] = bench_single_step(stencil, synth, torch, dev, side2=side)
        progress("single-step sweeps done")
    if not args.no_high:
        extra["2d_high_radius"] = bench_2d_high(stencil, synth, torch, dev, side=side,
                                                tune=not args.no_tune)
        progress(f"2D r=5..8: {extra['2d_high_radius']['GCell/s']} GCell/s")
        extra["3d_high_radius"] = bench_3d_high(stencil, synth, torch, dev, tune=not args.no_tune)
        progress(f"3D r=5..8: {extra['3d_high_radius']['GCell/s']} GCell/s")
    if not args.no_forms:
        extra["forms"] = bench_forms(stencil, synth, torch, dev, side2=side)
        progress("forms done")
    if not args.no_3d:
        extra["3d"] = bench_3d(stencil, synth, torch, dev, tune=not args.no_tune)
        progress(f"3D: {extra['3d']['GCell/s']} GCell/s")
    if not args.no_precision:
        extra["precision"] = bench_precision(stencil, synth, torch, dev, tune=not args.no_tune)
        progress("precision form done")
    if not args.no_batch:
        extra["batch"] = bench_batch(stencil, synth, torch, dev, tune=not args.no_tune)
        progress(f"batch: {extra['batch']['GCell/s']} GCell/s")
    if extra:
        out["extra"] = extra
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(f0, coeffs)
        progress("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
