#!/usr/bin/env python3
"""Benchmark of the constant-OPL vectorial ray march on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload freeform|grid|luneburg]

A "step" of this benchmark is one pass of the whole hot path over one batch:
one vrt_trace call that launches, enters, marches (medium evaluation, normal,
Snell/TIR/tangential/straight dispatch, compensated constant-OPL move,
surface refraction or reflection) and retires every ray of the batch, with the
inputs already resident in HBM.  The default workload is the freeform
analytic configuration: unit cube in air, n = 1.5 + 16 seeded Gaussian bumps,
1,048,576 rays from z = 0 in a 20 deg cone, dL0 = 5e-4, FP32 with
compensated sums and an FP64 discriminant.

Prints one JSON line: ray-steps/s (value), the roofline of the march kernel
(algorithmic work / measured kernel time vs the chip's peak), the FP64 CPU
oracle's rate on a bounded sample of the same rays (cpu_baseline), and the
parity of the timed GPU results against that oracle sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

import workloads

METRIC = "ray-steps/s at oracle-matched accuracy; served p50/p99 latency vs plain FP64 march"

# MI355X peaks: published FP32 vector rate (256 CUs x 2.4 GHz x 256 flop/clk)
# and HBM3E bandwidth.  The march issues more VALU lane-instructions per second
# than 256 x 4 SIMD x 16 lanes x 2.4 GHz (3.93e13/s, measured with
# SQ_INSTS_VALU), so that lower "non-packed" figure is not a ceiling here and
# the published FP32 vector peak is the denominator.
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the march kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE (KiB per dispatch), scaled by what the same counters read for a
# plain 2 GiB device copy (FETCH_SIZE reads half the copied bytes: x2;
# WRITE_SIZE reads them exactly: x1).  Valid only for the kernel sources they
# were taken on (sha256 of the files below); reported as null otherwise.
KERNEL_SOURCES = ("march_fp32c.hip", "media.h", "vrt_common.h", "dispatch.h")
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
TRAFFIC_KIB = {  # workload -> (fetch KiB, write KiB, kernel sha256); profiles/march_fp32c_hbm_traffic.md
    "freeform": (79749.3, 299428.1, "3907978953d2f3f7cccf527d3f8654bea236d0ad5dfc45efd2213bbb9284653b"),
    "grid": (409733720.5, 1584197.1, "3907978953d2f3f7cccf527d3f8654bea236d0ad5dfc45efd2213bbb9284653b"),
}


def kernel_sha():
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2606_22655_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_bytes(workload):
    t = TRAFFIC_KIB.get(workload)
    if t is None or t[2] != kernel_sha():
        return None
    return int((t[0] * FETCH_SCALE + t[1] * WRITE_SCALE) * 1024)


def algo_flops_per_step(workload, K=16):
    """Algorithmic FP32 work of one ray-step (FMA = 2, add/mul/cmp = 1,
    exp/sqrt/rsqrt/div = 1), derived in the design doc."""
    march = 50  # normal, N.I, mu, D, gamma, R = mu I + gamma N, Delta, move, surface test
    if workload == "freeform":
        return 19 * K + march  # per bump: P-c 3, r^2 5, scale 1, exp 1, A e 1, n+= 1, grad 7
    if workload == "grid":
        return 84 + march  # cell locate 12, trilinear n 14, trilinear grad 42, scale/misc 16
    if workload == "luneburg":
        return 16 + march
    raise ValueError(workload)


def algo_bytes_per_step(workload):
    """Algorithmic HBM bytes per ray-step: ray state in/out is 68 B per ray
    (amortised over ~3000 steps); grid media add the 8 corner records of a
    cell (128 B) once per cell visited (~1/12 of the steps at 12 steps per
    cell edge)."""
    if workload == "grid":
        return 128.0 / 12.0
    return 0.0


def build_workload(name, n_rays=None):
    if name == "freeform":
        spec, rays, prm = workloads.gaussian_cube(n_rays=n_rays or (1 << 20))
        desc = ("freeform analytic: unit cube in air, n = 1.5 + 16 seeded Gaussian bumps, "
                f"{rays[0].shape[0]} rays from z=0 in a 20 deg cone, dL0 = 5e-4, "
                "FP32 + compensated sums, FP64 discriminant")
        return spec, rays, prm, "fp32c", desc, 1.0
    if name == "grid":
        spec, rays, prm = workloads.quantized_grid_cube(n_rays=n_rays or (1 << 22))
        desc = ("discretized isoindicial: 256^3 FP32 grid, smoothed noise quantized to 32 "
                f"levels in [1.4, 1.8], {rays[0].shape[0]} rays from z=0 in a 30 deg cone, "
                "dL0 = 5e-4, FP32 + compensated sums")
        return spec, rays, prm, "fp32c", desc, 1.0
    if name == "luneburg":
        spec, rays, prm = workloads.luneburg_beam()
        desc = "Luneburg sphere R=1, 64x64 parallel beam, dL0 = 1e-3, plain FP64"
        return spec, rays, prm, "fp64", desc, 2.0
    raise ValueError(name)


def time_traces(vrt, torch, med, batch, prm, precision, steps, warmup):
    for _ in range(warmup):
        vrt.trace(med, batch, prm, precision)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        vrt.trace(med, batch, prm, precision)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    return wall, per


def cpu_baseline(spec, rays, prm, sample, g_res, aperture):
    import oracle  # CPU-baseline leg only

    oracle.build(force=False)
    n = min(sample, rays[0].shape[0])
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    r = oracle.trace(spec, (rays[0][:n], rays[1][:n]), prm, n_threads=threads)
    steps = int(r["steps"].sum())
    base = {"value": steps / r["seconds"], "unit": "ray-steps/s", "cores": threads,
            "kind": "oracle", "seconds": round(r["seconds"], 3),
            "sample": f"first {n} rays of the same workload ({steps} ray-steps), FP64 C oracle, "
                      f"OpenMP {threads} threads"}
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    from parity import compare

    sub = {k: v[:n] for k, v in g_res.items()}
    if spec["kind"] == "grid":
        # single rays through the quantized grid are chaotic (the oracle's own
        # exits move under 1e-11 launch shifts): compare distributions
        from parity import stat_compare

        rep = stat_compare(r, sub)
        rep["kind"] = "two-sample statistics (chaotic medium)"
        return base, rep
    rep = compare(r, sub, aperture=aperture, spec=spec)
    keys = ("n", "flagged_oracle", "flagged_gpu", "soft_flips", "status_mismatch", "tir_mismatch",
            "btir_mismatch", "pos_fail", "dir_fail", "steps_mismatch", "pos_err_max", "pos_err_p99",
            "dir_err_max", "dir_err_p99", "dir_err_inside_max")
    return base, {k: rep[k] for k in keys}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="freeform", choices=["freeform", "grid", "luneburg"])
    ap.add_argument("--rays", type=int, default=None)
    ap.add_argument("--cpu-sample", type=int, default=524288)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-gpu", action="store_true")
    args = ap.parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the march shards over rays with no exchange, and this "
              "build runs on a single MI355X; --gpus must be 1", file=sys.stderr)
        return 2

    import torch

    import paper_2606_22655_amd as vrt

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    spec, rays, prm, precision, desc, aperture = build_workload(args.workload, args.rays)
    n_rays = rays[0].shape[0]
    print(f"[bench] workload ready: {n_rays} rays", file=sys.stderr, flush=True)

    ctx = vrt.Context(0)
    med = vrt.Medium(ctx, spec)
    batch = vrt.RayBatch(rays[0], rays[1], precision)
    wall, per = time_traces(vrt, torch, med, batch, prm, precision, args.steps, args.warmup)
    cnt = vrt.counters(ctx, batch)
    g_res = batch.results()
    ms = float(np.mean(per))
    ray_steps = cnt["steps"]
    value = ray_steps / (ms / 1e3)
    print(f"[bench] {args.steps} traces, {ms:.3f} ms each, {value:.4g} ray-steps/s",
          file=sys.stderr, flush=True)

    fp64_gpu = None
    if not args.no_fp64_gpu and precision != "fp64":
        b64 = vrt.RayBatch(rays[0], rays[1], "fp64")
        w64, per64 = time_traces(vrt, torch, med, b64, prm, "fp64", max(2, args.steps // 5), 1)
        c64 = vrt.counters(ctx, b64)
        fp64_gpu = {"ms_per_step": round(float(np.mean(per64)), 3),
                    "ray_steps_per_s": c64["steps"] / (float(np.mean(per64)) / 1e3),
                    "note": "plain FP64 GPU march, one lane per ray, one launch per batch"}
        del b64

    flops = algo_flops_per_step(args.workload) * ray_steps
    achieved = flops / (ms / 1e3) / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": traffic_bytes(args.workload) if precision == "fp32c" else None,
            "algo_flops_per_ray_step": algo_flops_per_step(args.workload),
            "kernel": "march_fp32c_kernel" if precision == "fp32c" else "march_fp64_kernel"}
    if args.workload == "grid":
        gbs = algo_bytes_per_step("grid") * ray_steps / (ms / 1e3) / 1e9
        roof["hbm_side"] = {"achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                            "frac": round(gbs / PEAK_HBM_GBS, 4)}

    out = {"metric": METRIC, "value": value, "unit": "ray-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if precision == "fp32c" else "f64", "data": "synthetic",
           "config": {"workload": desc, "rays": n_rays, "ray_steps_per_trace": ray_steps,
                      "dL0": prm["dL0"], "max_steps": prm["max_steps"]},
           "wall_s": round(wall, 3), "roofline": roof, "counters": cnt}
    if fp64_gpu:
        out["fp64_gpu_march"] = fp64_gpu
    if not args.no_cpu_baseline:
        base, par = cpu_baseline(spec, rays, prm, args.cpu_sample, g_res, aperture)
        out["cpu_baseline"] = base
        out["parity_vs_oracle"] = par
    med.close()
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
