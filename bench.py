#!/usr/bin/env python3
"""Benchmark of the constant-OPL vectorial ray march on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload freeform|grid|luneburg|zernike|spherical|helix|served|n2p|
                                adjoint]

A "step" of this benchmark is one pass of the whole hot path over one batch:
one vrt_trace call that launches, enters, marches (medium evaluation, normal,
Snell/TIR/tangential/straight dispatch, compensated constant-OPL move,
surface refraction or reflection) and retires every ray of the batch, with the
inputs already resident in HBM.

The default (headline) workload is the largest single-GPU configuration: the
discretized isoindicial medium, a 256^3 FP32 index grid of smoothed noise
quantized to 32 levels in [1.4, 1.8], 4,194,304 rays from z = 0 in a 30 deg
cone, dL0 = 5e-4, FP32 with compensated sums.  Its record carries the roofline
of the march kernel (algorithmic bytes of the visited cells against HBM, the
VALU side beside it), the FP64 oracle's rate on a bounded sample of the same
rays (cpu_baseline) and the parity of the timed results.  Two sub-records
follow: "freeform" (the 16-Gaussian-bump cube, 1,048,576 rays, 20 deg cone,
with per-ray parity of 524,288 rays against the oracle) and "served" (a
Poisson stream of 120 jobs at 80 % of the measured capacity over eight
resident media, its rays/s and p50/p99 latency next to one plain FP64 launch
per job, and the parity of sampled served rays).  The grid and freeform
records also carry "two_in_flight": the rate of a stream of batches traced
two at a time on two streams, so that the last long rays of one trace share
the device with the start of the next (reported beside value, never as it).

Prints one JSON line.
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
# were taken on (sha256 of the code in the files below, comments and blank
# lines left out); reported as null otherwise.
KERNEL_SOURCES = ("march_fp32c.hip", "lane32.h", "media.h", "vrt_common.h", "dispatch.h")
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
TRAFFIC_KIB = {  # workload -> (fetch KiB, write KiB, kernel code sha256); profiles/march_fp32c_hbm_traffic.md
    "freeform": (79289.96, 304980.59, "22def1ced10ae8adc33b958dea059916a7dafc3a2e08f57ed3de6e4cc4d39406"),
    "grid": (427689715.39, 1578064.37, "22def1ced10ae8adc33b958dea059916a7dafc3a2e08f57ed3de6e4cc4d39406"),
}


def kernel_sha():
    """sha256 of the kernel's code: the files of KERNEL_SOURCES with /* */ and
    // comments, trailing blanks and blank lines removed, so that a change of
    a comment keeps the measured traffic valid (no string literal in these
    files holds a comment marker)."""
    import hashlib
    import re

    h = hashlib.sha256()
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2606_22655_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines())
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()


def traffic_bytes(workload):
    t = TRAFFIC_KIB.get(workload)
    if t is None or t[2] != kernel_sha():
        return None
    return int((t[0] * FETCH_SCALE + t[1] * WRITE_SCALE) * 1024)


def algo_flops_per_step(workload, K=16):
    """Algorithmic FP32 work of one ray-step (FMA = 2, add/mul/cmp = 1,
    exp/sqrt/rsqrt/div = 1): the operations the method itself needs per step,
    counted term by term below."""
    march = 50  # normal, N.I, mu, D, gamma, R = mu I + gamma N, Delta, move, surface test
    if workload == "freeform":
        return 19 * K + march  # per bump: P-c 3, r^2 5, scale 1, exp 1, A e 1, n+= 1, grad 7
    if workload == "grid":
        return 84 + march  # cell locate 12, trilinear n 14, trilinear grad 42, scale/misc 16
    if workload == "luneburg":
        return 16 + march
    if workload in FP64_FLOPS_PER_STEP:
        return march
    raise ValueError(workload)


# Media evaluated in double precision inside the FP32 march: FP64 work per
# ray-step (one index-and-gradient evaluation at P_i -- n(P_{i-1}) is carried
# from the previous step -- plus the index difference), counted as in
# algo_flops_per_step.  Zernike lens with the paper's five active Fringe rows:
# u, v, w 5, Legendre P2, P3 and derivatives 12, per row 31 (A 6, dA 4, Z and
# its partials 13, four sums 8), n and gradient 8 -> 180.  Spherical
# freeform: offsets 3, r^2 5, cos^2 2, n 17, G2 slopes 11, gradient 20 -> 60.
FP64_FLOPS_PER_STEP = {"zernike": 180 + 1, "spherical": 60 + 1}


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
    if name == "zernike":
        spec = workloads.zernike_lens()
        rays = workloads.zernike_rays(n_rays or (1 << 20), seed=900)
        prm = workloads.trace_params(1e-3, 100000)
        desc = ("freeform cylindrical lens (Sec. V): seven Fringe Zernike x Legendre terms, "
                "rho_max = 4.2, z_max = 2.5, n in [1.5261, 1.5608], in air; the Fig. 3(a) ray "
                f"and {rays[0].shape[0] - 1} more from z = -0.5 to points in the lens, "
                "dL0 = 1e-3, FP32 + compensated sums, index in FP64")
        return spec, rays, prm, "fp32c", desc, 4.2
    if name == "spherical":
        spec = workloads.spherical_medium()
        rays = workloads.sphere_aimed_rays(n_rays or (1 << 20), seed=901)
        prm = workloads.trace_params(1e-3, 20000)
        desc = ("spherical freeform medium (Sec. V, Eq. (26)): a = (1.5, 1, -0.2, 0.3) in the "
                f"unit sphere in air, {rays[0].shape[0]} rays aimed into the ball, dL0 = 1e-3, "
                "FP32 + compensated sums, index in FP64")
        return spec, rays, prm, "fp32c", desc, 2.0
    if name == "luneburg":
        side = int(round(math.sqrt(n_rays))) if n_rays else 64
        spec, rays, prm = workloads.luneburg_beam(n_side=side)
        desc = f"Luneburg sphere R=1, {side}x{side} parallel beam, dL0 = 1e-3, plain FP64"
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


def pcie_inclusive(vrt, torch, med, batch, prm, precision, reps=2):
    """The same trace with the batch handed over in pinned host memory: its
    inputs copied in, the trace, its outputs and per-ray words copied out, all
    on one stream and timed with events (reported beside value, never as it)."""
    stream = torch.cuda.current_stream()
    h_in = torch.empty(batch.inp.shape, dtype=batch.inp.dtype, pin_memory=True)
    h_in.copy_(batch.inp)
    h_out = torch.empty(batch.out.shape, dtype=batch.out.dtype, pin_memory=True)
    h_u32 = torch.empty(batch.u32.shape, dtype=batch.u32.dtype, pin_memory=True)
    best = None
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        batch.inp.copy_(h_in, non_blocking=True)
        ev[1].record(stream)
        vrt.trace(med, batch, prm, precision)
        ev[2].record(stream)
        h_out.copy_(batch.out, non_blocking=True)
        h_u32.copy_(batch.u32, non_blocking=True)
        ev[3].record(stream)
        torch.cuda.synchronize()
        t = [ev[k].elapsed_time(ev[k + 1]) for k in range(3)]
        if best is None or sum(t) < sum(best):
            best = t
    b_in = batch.inp.numel() * batch.inp.element_size()
    b_out = batch.out.numel() * batch.out.element_size() + batch.u32.numel() * 4
    return best, b_in, b_out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


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
                      f"OpenMP {threads} threads", "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count()}
    # the same oracle on one core, on the first 1/32 of the sample
    n1 = max(1, n // 32)
    r1 = oracle.trace(spec, (rays[0][:n1], rays[1][:n1]), prm, n_threads=1)
    base["one_core"] = {"value": int(r1["steps"].sum()) / r1["seconds"], "rays": n1,
                        "seconds": round(r1["seconds"], 3)}
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    from parity import compare

    sub = {k: v[:n] for k, v in g_res.items()}
    if spec["kind"] == "grid":
        # single rays through the quantized grid are chaotic (the oracle's own
        # exits move under 1e-11 launch shifts): the caller compares the
        # distributions of these full paths and single rays over 128 moves
        return base, None, (r, np.arange(n))
    chaotic = spec["kind"] in ("spherical", "zernike")
    if chaotic:
        # rays trapped by repeated TIR (in the sphere, along the lens wall)
        # amplify perturbations up to ~1e4-fold: leave out those whose oracle
        # events change, or whose oracle result moves by more than the bar
        # (1e-4), under a float32-sized (1e-7) shift of the launch point or
        # turn of the launch direction (their inputs do not fix them to the bar)
        from parity import exempt, ill_conditioned

        bad = ill_conditioned(lambda *a: oracle.trace(*a, n_threads=threads), spec,
                              (rays[0][:n], rays[1][:n]), prm, delta=1e-7, tol=1e-4, turn=1e-7)
        r, sub = exempt(r, bad), exempt(sub, bad)
    rep = compare(r, sub, aperture=aperture, spec=spec)
    if chaotic:
        rep["ill_conditioned"] = int(bad.sum())
    keys = ("n", "checked", "fail", "exempt_critical", "exempt_grazing", "tie_checked",
            "tie_steps_differ", "flagged_oracle_critical", "flagged_oracle_tie",
            "flagged_oracle_grazing", "flagged_gpu_critical", "status_mismatch", "tir_mismatch",
            "btir_mismatch", "pos_fail", "dir_fail", "fail_in_wide_window", "steps_mismatch",
            "steps_absmax", "pos_err_max", "pos_err_p99", "dir_err_max", "dir_err_p99",
            "dir_err_inside_max", "ill_conditioned", "bad_rays")
    return base, {k: rep[k] for k in keys if k in rep}, None


# ---------------------------------------------------------------------------
# served mix: Poisson stream of jobs against 8 resident media
# ---------------------------------------------------------------------------
POOL_RAYS = 1 << 22  # launch states per medium; a job takes a slice


def served_inputs(torch, media):
    """Per medium, 4M pinned float32 launch states (SoA rows): face launches
    in a 20 deg (analytic) or 30 deg (grid) cone, seeds 600 + medium."""
    pools = []
    for i, spec in enumerate(media):
        cone = 30.0 if spec["kind"] == "grid" else 20.0
        P0, d0 = workloads.face_cone_rays(POOL_RAYS, 600 + i, cone)
        t = torch.empty((6, POOL_RAYS), dtype=torch.float32, pin_memory=True)
        t[0:3].copy_(torch.from_numpy(P0.T.astype(np.float32)))
        t[3:6].copy_(torch.from_numpy(d0.T.astype(np.float32)))
        pools.append(t)
    return pools


def job_buffers(vrt, torch, pool, off, n):
    """vrt_rays over pinned host memory: inputs are rows of the medium's pool,
    outputs fresh pinned arrays."""
    out = torch.empty((6, n), dtype=torch.float32, pin_memory=True)
    u32 = torch.empty((5, n), dtype=torch.int32, pin_memory=True)
    r = vrt.vrt_rays()
    for i, k in enumerate(("px", "py", "pz", "dx", "dy", "dz")):
        setattr(r, k, pool[i].data_ptr() + 4 * off)
    for i, k in enumerate(("ox", "oy", "oz", "odx", "ody", "odz")):
        setattr(r, k, out[i].data_ptr())
    for i, k in enumerate(("status", "steps", "n_tir", "n_btir", "flags")):
        setattr(r, k, u32[i].data_ptr())
    return r, (out, u32)


def served_parity(vrt, torch, jobs, keep, pools, meds, media, prm, offset, pick,
                  n_oracle=256):
    """Parity of the served results: for a seeded sample of jobs, every ray of
    the job against a vrt_trace batch launch of the same rays (bitwise: the
    served kernel runs the batch kernel's per-lane march), and for jobs on
    analytic media n_oracle sampled rays against the oracle under the pass
    rule of tests/parity.py (grid media are chaotic over full paths; their
    batch kernel is checked against the oracle by the headline record)."""
    import oracle

    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    from parity import compare

    rng = np.random.default_rng(78)
    rep = {"jobs": len(pick), "rays_bitwise_checked": 0, "rays_bitwise_differ": 0,
           "oracle_rays": 0, "oracle_fail": 0, "oracle_exempt_critical": 0,
           "oracle_exempt_grazing": 0, "oracle_pos_err_max": 0.0, "oracle_dir_err_max": 0.0}
    for k in pick:
        j = jobs[k]
        n, src, off = j["n_rays"], pools[j["medium"]], offset(j)
        out, u32 = keep[k]
        srv = {"P": out[0:3].numpy().T.astype(np.float64), "D": out[3:6].numpy().T.astype(np.float64)}
        u = u32.numpy().view(np.uint32)
        for i, key in enumerate(("status", "steps", "ntir", "nbtir", "flags")):
            srv[key] = u[i].copy()
        P0 = src[0:3, off:off + n].numpy().T.astype(np.float64)
        d0 = src[3:6, off:off + n].numpy().T.astype(np.float64)
        b = vrt.RayBatch(P0, d0, "fp32c")
        vrt.trace(meds[j["medium"]], b, prm, "fp32c")
        ref = b.results()
        del b
        same = np.ones(n, dtype=bool)
        for key in ("P", "D", "status", "steps", "ntir", "nbtir", "flags"):
            v = ref[key] == srv[key]
            same &= v.all(axis=1) if v.ndim == 2 else v
        rep["rays_bitwise_checked"] += n
        rep["rays_bitwise_differ"] += int((~same).sum())
        if media[j["medium"]]["kind"] != "grid":
            idx = np.sort(rng.choice(n, min(n_oracle, n), replace=False))
            o = oracle.trace(media[j["medium"]], (P0[idx], d0[idx]), prm)
            r = compare(o, {key: v[idx] for key, v in srv.items()}, aperture=1.0,
                        spec=media[j["medium"]])
            rep["oracle_rays"] += r["n"]
            rep["oracle_fail"] += r["fail"]
            rep["oracle_exempt_critical"] += r["exempt_critical"]
            rep["oracle_exempt_grazing"] += r["exempt_grazing"]
            rep["oracle_pos_err_max"] = max(rep["oracle_pos_err_max"], r["pos_err_max"])
            rep["oracle_dir_err_max"] = max(rep["oracle_dir_err_max"], r["dir_err_max"])
    print(f"[served] parity: {json.dumps(rep)}", file=sys.stderr, flush=True)
    return rep


def served_bench(vrt, torch, args):
    """Continuous batching of a Poisson job stream (ray counts log-uniform in
    [1e3, 4e6], 8 resident media) on the served FP32c path, then the same
    stream on the plain one-launch-per-job FP64 march (FIFO, one job at a
    time).  Latency = done - arrival."""
    t_setup = time.perf_counter()
    media = workloads.served_media()
    ctx = vrt.Context(0)
    meds = [vrt.Medium(ctx, m) for m in media]
    pools = served_inputs(torch, media)
    prm = workloads.trace_params(5e-4, 60000)
    budget = 4 << 30
    srv = vrt.Server(ctx, budget)
    print(f"[served] setup {time.perf_counter() - t_setup:.1f} s", file=sys.stderr, flush=True)
    # capacity: one 2^18-ray job per medium, all at once
    keep, ids = [], []
    t0 = time.perf_counter()
    for i, m in enumerate(meds):
        r, bufs = job_buffers(vrt, torch, pools[i], 0, 1 << 18)
        keep.append(bufs)
        ids.append(vrt.vrt_server_submit(srv.handle, m.handle, vrt.make_params(prm, "fp32c"), r,
                                         1 << 18))
    infos = [vrt.vrt_server_wait(srv.handle, j, 600.0) for j in ids]
    cal_s = time.perf_counter() - t0
    print("[served] calibration job ms: " + " ".join(
        f"{1e3 * (i['t_retired'] - i['t_start']):.1f}" for i in infos) + f", total {1e3 * cal_s:.1f}",
        file=sys.stderr, flush=True)
    steps_per_ray = [i["ray_steps"] / (1 << 18) for i in infos]
    cap = sum(i["ray_steps"] for i in infos) / cal_s
    jobs0 = workloads.served_jobs(n_jobs=args.jobs)
    mean_steps = float(np.mean([j["n_rays"] * steps_per_ray[j["medium"]] for j in jobs0]))
    rate = args.load * cap / mean_steps
    jobs = workloads.served_jobs(n_jobs=args.jobs, rate_hz=rate)
    print(f"[served] capacity {cap:.3g} ray-steps/s, rate {rate:.2f} jobs/s, "
          f"{len(jobs)} jobs, {sum(j['n_rays'] for j in jobs)} rays", file=sys.stderr, flush=True)

    def offset(j):
        return j["ray_seed"] % (POOL_RAYS - j["n_rays"] + 1)

    # served run: submit at the arrival times; a job's pinned buffers are
    # released once it is done, except those of the jobs whose results the
    # parity block checks
    sample = set(np.sort(np.random.default_rng(77).choice(len(jobs), min(16, len(jobs)),
                                                          replace=False)).tolist())
    keep, ids, infos, pending = {}, [], [None] * len(jobs), []
    t_base = time.perf_counter()
    every = 10 if len(jobs) <= 1000 else 100

    def reap(block=False):
        while pending:
            k = pending[0]
            info = (vrt.vrt_server_wait(srv.handle, ids[k], 600.0) if block else
                    vrt.vrt_server_query(srv.handle, ids[k]))
            if info["state"] != "DONE":
                return
            infos[k] = info
            pending.pop(0)
            if k not in sample:
                keep.pop(k, None)

    for k, j in enumerate(jobs):
        wait = j["t_arrival"] - (time.perf_counter() - t_base)
        if wait > 0:
            time.sleep(wait)
        if k % every == 0:
            print(f"[served] submitting job {k} at {time.perf_counter() - t_base:.2f} s",
                  file=sys.stderr, flush=True)
        r, bufs = job_buffers(vrt, torch, pools[j["medium"]], offset(j), j["n_rays"])
        keep[k] = bufs
        ids.append(vrt.vrt_server_submit(srv.handle, meds[j["medium"]].handle,
                                         vrt.make_params(prm, "fp32c"), r, j["n_rays"]))
        pending.append(k)
        reap()
    reap(block=True)
    stats = vrt.vrt_server_stats_get(srv.handle)
    srv.close()
    lat = np.array([i["t_done"] - i["t_submit"] for i in infos])
    span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
    steps = sum(i["ray_steps"] for i in infos)
    rays = sum(i["n_rays"] for i in infos)
    served = {"rays_per_s": rays / span, "ray_steps_per_s": steps / span,
              "p50_ms": 1e3 * float(np.percentile(lat, 50)),
              "p99_ms": 1e3 * float(np.percentile(lat, 99)),
              "span_s": span, "kernel_launches": stats["kernel_launches"],
              "pool_peak_bytes": stats["pool_peak_bytes"], "lanes": stats["lanes"]}
    print(f"[served] fp32c: {rays / span:.4g} rays/s, p50 {served['p50_ms']:.1f} ms, "
          f"p99 {served['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    served["parity"] = served_parity(vrt, torch, jobs, keep, pools, meds, media, prm, offset,
                                     sorted(sample))
    del keep
    # the same stream (or its first fp64_jobs jobs), one FP64 launch per job,
    # FIFO on one stream
    stream = torch.cuda.current_stream()
    lat64, busy = [], 0.0
    clock = 0.0  # simulated clock on the arrival axis: a job starts at max(arrival, previous end)
    n64 = len(jobs) if args.fp64_jobs is None else min(args.fp64_jobs, len(jobs))
    rays64 = sum(j["n_rays"] for j in jobs[:n64])
    for k, j in enumerate(jobs[:n64]):
        if k % 10 == 0:
            print(f"[served] fp64 job {k}", file=sys.stderr, flush=True)
        n, src = j["n_rays"], pools[j["medium"]]
        off = offset(j)
        t_start = time.perf_counter()
        b = vrt.RayBatch(src[0:3, off:off + n].T.double(), src[3:6, off:off + n].T.double(), "fp64")
        vrt.trace(meds[j["medium"]], b, prm, "fp64", stream=stream.cuda_stream)
        _ = b.out.cpu(), b.u32.cpu()
        dur = time.perf_counter() - t_start
        busy += dur
        clock = max(clock, j["t_arrival"]) + dur
        lat64.append(clock - j["t_arrival"])
        del b
    lat64 = np.array(lat64)
    fp64 = {"jobs": n64, "rays_per_s": rays64 / busy,
            "p50_ms": 1e3 * float(np.percentile(lat64, 50)),
            "p99_ms": 1e3 * float(np.percentile(lat64, 99)), "busy_s": busy,
            "note": "jobs run back to back on the GPU, one FP64 launch each (inputs copied in, "
                    "outputs copied out); each job starts at max(its arrival, the previous "
                    "job's end) on the arrival clock"}
    print(f"[served] fp64 per job ({n64} jobs): {rays64 / busy:.4g} rays/s, p50 {fp64['p50_ms']:.1f} ms, "
          f"p99 {fp64['p99_ms']:.1f} ms", file=sys.stderr, flush=True)
    for m in meds:
        m.close()
    ctx.close()
    return {"metric": METRIC, "value": served["ray_steps_per_s"], "unit": "ray-steps/s",
            "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * span,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"served mix: {len(jobs)} Poisson jobs at {rate:.2f}/s "
                                   f"({args.load:.0%} of measured capacity), ray counts "
                                   "log-uniform in [1e3, 4e6], 4 Gaussian-bump cubes + grids "
                                   "128/160/192/256^3, dL0 = 5e-4, FP32 + compensation",
                       "rays": rays, "ray_steps": steps, "pool_bytes": budget},
            "served_fp32c": served, "one_launch_per_job_fp64": fp64,
            "p99_speedup_vs_fp64": fp64["p99_ms"] / served["p99_ms"]}


# ---------------------------------------------------------------------------
# the paper's design example: N2P lens design loop (Sec. VI)
# ---------------------------------------------------------------------------
PEAK_FP64_TFLOPS = 78.6
N2P_FLOPS_PER_STEP = 69  # index 19 (rho^2 3, w 4, two powers 2, u 1, gradient 9) + march 50


def n2p_bench(vrt, torch, args, L=0.3, cpu_candidates=256):
    """Successive refinement of the N2P lens of thickness 0.3 R, F = 2R
    (the configuration of the paper's Fig. 6), 10 rays per candidate,
    dL0 = 1e-4 R, a 33 x 33 candidate grid per level; each level is one
    vrt_n2p_sweep launch, timed with HIP events on its stream."""
    from paper_2606_22655_amd import design

    ctx = vrt.Context(0)
    stream = torch.cuda.current_stream()
    spec = workloads.n2p_lens(1.0, 1.0, L)
    y = workloads.n2p_heights()
    P0, _ = workloads.n2p_rays(L)
    prm = vrt.make_params({"dL0": 1e-4, "max_steps": 200000}, "fp64")
    lens = vrt.Medium(ctx, spec)
    per, steps, cands = [], [0], [0]

    def score(bg):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rm, st = vrt.vrt_n2p_sweep(lens.handle, bg, y, P0[0, 2], prm, stream.cuda_stream,
                                   want_steps=True)
        e1.record(stream)
        torch.cuda.synchronize()
        per.append(e0.elapsed_time(e1))
        steps[0] += int(st.sum())
        cands[0] += len(bg)
        print(f"[n2p] level {len(per)}: {len(bg)} candidates, {per[-1]:.1f} ms", file=sys.stderr,
              flush=True)
        return rm

    design.refine(score, levels=1)  # warmup (one level)
    per.clear()
    steps[0] = cands[0] = 0
    t0 = time.perf_counter()
    b, g, e, hist = design.refine(score)
    wall = time.perf_counter() - t0
    lens.close()
    kernel_s = sum(per) / 1e3
    value = steps[0] / kernel_s
    achieved = N2P_FLOPS_PER_STEP * steps[0] / kernel_s / 1e12
    out = {"metric": METRIC, "value": value, "unit": "ray-steps/s", "n_gpus": 1,
           "steps": len(per), "warmup": 1, "ms_per_step": round(float(np.mean(per)), 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"N2P lens design loop (Sec. VI): L = {L} R, F = 2 R, 10 rays "
                                  "at y_i = 0.995 R i / 10, dL0 = 1e-4 R, 33 x 33 (beta, gamma) "
                                  "grid per refinement level, plain FP64 march",
                      "candidates": cands[0], "ray_steps": steps[0]},
           "design": {"beta": b, "gamma": g, "rmse_lsa": e, "levels": len(per),
                      "wall_s": round(wall, 3)},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                        "traffic": None, "algo_flops_per_ray_step": N2P_FLOPS_PER_STEP,
                        "kernel": "n2p_sweep_kernel",
                        "note": "1089 candidates x 10 rays = 10,890 lanes per launch: 170 "
                                "waves for 1,024 SIMDs, so a level is latency-bound"}}
    if not args.no_cpu_baseline:
        import oracle  # CPU-baseline leg only
        from concurrent.futures import ThreadPoolExecutor

        oracle.build(force=False)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        bs = np.linspace(0.2, 2.5, 33)
        gs = np.linspace(0.5, 8.0, 33)
        cand = [(bb, gg) for bb in bs for gg in gs][:cpu_candidates]
        rays = workloads.n2p_rays(L)

        def one(c):
            r = oracle.trace(workloads.n2p_lens(c[0], c[1], L), rays,
                             {"dL0": 1e-4, "max_steps": 200000}, n_threads=1)
            return int(r["steps"].sum())

        t0 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            n_steps = sum(ex.map(one, cand))
        sec = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n_steps / sec, "unit": "ray-steps/s", "cores": threads,
                               "kind": "oracle", "seconds": round(sec, 3),
                               "sample": f"first {len(cand)} candidates of the first refinement "
                                         f"level ({n_steps} ray-steps), FP64 C oracle, one "
                                         f"candidate per thread, {threads} threads"}
    ctx.close()
    return out


# ---------------------------------------------------------------------------
# differentiable design: loss and gradient w.r.t. grid node values
# ---------------------------------------------------------------------------
ADJ_FLOPS_PER_STEP = 134  # the FP64 grid march step (as the grid workload's count)


def adjoint_bench(vrt, torch, args):
    """The differentiable design configuration: 64^3 grid 1.5 + 0.01 N(0,1),
    512 x 512 parallel rays along +z, exit plane z = 1.2, targets on a ring,
    dL0 = 5e-4, FP64.  Times the loss alone and the loss with its gradient
    (forward with checkpoints every 64 steps, replay, reverse sweep)."""
    med, (P0, d0), prm, tgt = workloads.design_problem(max_steps=10000)
    ctx = vrt.Context(0)
    f = vrt.ExitPlaneLoss(ctx, P0, d0, tgt, prm, checkpoint_every=64)
    v = torch.tensor(med["grid"], device="cuda")
    g = torch.empty(v.shape, dtype=torch.float64, device="cuda")
    f.evaluate(v, g)  # warmup
    steps_fwd = None
    t_loss, t_grad = [], []
    for k in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = f.evaluate(v)
        torch.cuda.synchronize()
        t_loss.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        L2 = f.evaluate(v, g)
        torch.cuda.synchronize()
        t_grad.append(time.perf_counter() - t0)
        print(f"[adjoint] iteration {k}: loss {t_loss[-1] * 1e3:.1f} ms, loss+grad "
              f"{t_grad[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    # ray-steps of the forward march (the same rays through the plain FP64 trace)
    b = vrt.RayBatch(P0, d0, "fp64")
    medium = vrt.Medium(ctx, med)
    vrt.trace(medium, b, prm, "fp64")
    steps_fwd = vrt.counters(ctx, b)["steps"]
    medium.close()
    tl, tg = float(np.median(t_loss)), float(np.median(t_grad))
    value = steps_fwd / tg
    out = {"metric": METRIC, "value": value, "unit": "ray-steps/s", "n_gpus": 1,
           "steps": len(t_grad), "warmup": 1, "ms_per_step": round(tg * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "differentiable design: 64^3 grid 1.5 + 0.01 N(0,1), 512 x 512 "
                                  "parallel rays along +z, exit plane z = 1.2, ring targets, "
                                  "dL0 = 5e-4, FP64, gradient of the exit-plane loss w.r.t. the "
                                  "262,144 node values, checkpoints every 64 steps",
                      "rays": len(P0), "ray_steps": steps_fwd},
           "loss": L2, "loss_only_ms": round(tl * 1e3, 3), "loss_and_grad_ms": round(tg * 1e3, 3),
           "grad_over_loss_time": round(tg / tl, 3),
           "roofline": {"bound": "alu", "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "achieved": round(ADJ_FLOPS_PER_STEP * steps_fwd / tl / 1e12, 3),
                        "frac": round(ADJ_FLOPS_PER_STEP * steps_fwd / tl / 1e12 /
                                      PEAK_FP64_TFLOPS, 4),
                        "traffic": None, "kernel": "adj_forward_kernel (loss only)",
                        "algo_flops_per_ray_step": ADJ_FLOPS_PER_STEP}}
    if not args.no_cpu_baseline:
        import oracle  # CPU-baseline leg only

        oracle.build(force=False)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        n = 16384
        r = oracle.trace(med, (P0[:n], d0[:n]), prm, n_threads=threads)
        st = int(r["steps"].sum())
        out["cpu_baseline"] = {"value": st / r["seconds"], "unit": "ray-steps/s", "cores": threads,
                               "kind": "oracle", "seconds": round(r["seconds"], 3),
                               "sample": f"first {n} rays, forward march only ({st} ray-steps): "
                                         "the oracle has no adjoint; its gradient is two marches "
                                         "per node value"}
    ctx.close()
    return out


# ---------------------------------------------------------------------------
# the paper's helix (Sec. IV): one ray, its polyline recorded
# ---------------------------------------------------------------------------
HELIX_FLOPS_PER_STEP = 15 + 50  # fiber index and gradient 15 (rho^2 3, n 5, slope 4, gradient 3)


def helix_rays(P0, d0, n):
    """n copies of the helix launch turned about the fiber axis by 2 pi k / n:
    the fiber is axisymmetric, so each is the same helix, phase-shifted."""
    a = 2.0 * math.pi * np.arange(n) / n
    c, s = np.cos(a), np.sin(a)
    rot = lambda v: np.stack([c * v[0] - s * v[1], s * v[0] + c * v[1], np.full(n, v[2])], axis=1)
    return rot(P0[0]), rot(d0[0])


def helix_bench(vrt, torch, args, n_batch=196608):
    """The helical ray of Sec. IV at dL0 = 1e-4 (808,360 steps).  Timed step:
    a batch of 196,608 copies of the helix (turned about the axis; 3 waves per
    SIMD, the FP64 kernel's occupancy) on the plain FP64 march.  Beside it,
    the paper's single ray with its polyline recorded (vrt_trace_paths): one
    ray is one lane, so that figure is a latency."""
    spec, (P0, d0), hx = workloads.helix_fiber()
    prm = {"dL0": 1e-4, "max_steps": 2_000_000}
    ctx = vrt.Context(0)
    med = vrt.Medium(ctx, spec)
    stream = torch.cuda.current_stream()
    # batch of helices, plain FP64 march
    rays = helix_rays(P0, d0, args.rays or n_batch)
    batch = vrt.RayBatch(rays[0], rays[1], "fp64")
    wall, per = time_traces(vrt, torch, med, batch, prm, "fp64", max(1, args.steps), 1)
    cnt = vrt.counters(ctx, batch)
    ms = float(np.mean(per))
    value = cnt["steps"] / (ms / 1e3)
    print(f"[helix] batch of {batch.n}: {ms:.1f} ms per trace, {value:.4g} ray-steps/s",
          file=sys.stderr, flush=True)
    # the paper's single ray with its polyline
    b1 = vrt.RayBatch(P0, d0, "fp64")
    cap = 808_400
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    path, npts = vrt.trace_paths(med, b1, prm, cap)
    e1.record(stream)
    torch.cuda.synchronize()
    one_ms = e0.elapsed_time(e1)
    res = b1.results()
    m = int(npts[0])
    pts = path[:min(m, cap), 0].cpu().numpy()
    ins = pts[pts[:, 2] >= 0.0]
    z = ins[:, 2]
    rho0, kap = hx["rho0"], hx["kappa"]
    rmse = math.sqrt(np.mean((ins[:, 0] - rho0 * np.cos(kap * z)) ** 2 +
                             (ins[:, 1] - rho0 * np.sin(kap * z)) ** 2))
    achieved = HELIX_FLOPS_PER_STEP * value / 1e12
    out = {"metric": METRIC, "value": value, "unit": "ray-steps/s", "n_gpus": 1,
           "steps": len(per), "warmup": 1, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "helical ray of Sec. IV: parabolic fiber n_c = 1.38, "
                                  "Delta = 0.2, R = 5, length 55, dL0 = 1e-4; "
                                  f"{batch.n} copies turned about the axis, plain FP64 march",
                      "rays": batch.n, "ray_steps_per_trace": cnt["steps"]},
           "single_ray": {"ms": round(one_ms, 3), "ray_steps_per_s": int(res["steps"][0]) / (one_ms / 1e3),
                          "points": m, "points_inside": int(len(ins)), "rmse": rmse,
                          "kernel": "record_paths_kernel",
                          "paper": {"points": 808360, "rmse": 5.0892e-5, "wall_s": 0.5157,
                                    "hardware": "MATLAB R2024b, Apple M4 (trajectory + rendering)"}},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                        "traffic": None, "algo_flops_per_ray_step": HELIX_FLOPS_PER_STEP,
                        "kernel": "march_fp64_kernel"},
           "counters": cnt}
    if not args.no_cpu_baseline:
        import oracle  # CPU-baseline leg only

        oracle.build(force=False)
        t0 = time.perf_counter()
        op, ores = oracle.trace_path(spec, P0[0], d0[0], prm, cap=cap)
        sec = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": ores["steps"] / sec, "unit": "ray-steps/s", "cores": 1,
                               "kind": "oracle", "seconds": round(sec, 3),
                               "sample": "the paper's single ray with its polyline recorded, FP64 "
                                         "C oracle, one thread (one ray)"}
        k = min(len(op), len(pts))
        out["parity_vs_oracle"] = {"points_equal_count": bool(ores["n_path"] == m),
                                   "max_point_diff": float(np.abs(pts[:k] - op[:k]).max()),
                                   "batch_steps_equal": bool(np.all(batch.results()["steps"] ==
                                                                    ores["steps"]))}
    med.close()
    ctx.close()
    return out


def grid_parity(vrt, torch, med, spec, rays, prm, g_full, oracle_full, idx_full, threads):
    """Parity of the timed grid launch configuration against the oracle.  The
    quantized grid is chaotic for the discrete march (a 1e-13 shift of a
    launch moves a third of the oracle's own exits by more than 1e-4), so:
    per ray over the first 128 moves (the whole batch re-run with
    max_steps = 128, a seeded sample of 4,096 rays recomputed by the oracle;
    rays whose own oracle state moves under a 1e-9 launch shift are counted
    and set aside), and two-sample statistics of the full exit states of the
    oracle sample (the cpu_baseline rays) against the same rays of the timed
    run."""
    import oracle

    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests"))
    from parity import compare, exempt, ill_conditioned, stat_compare

    P0, d0 = rays
    n = P0.shape[0]
    p128 = dict(prm, max_steps=128)
    b = vrt.RayBatch(P0, d0, "fp32c")
    vrt.trace(med, b, p128, "fp32c")
    g128 = b.results()
    del b
    idx = np.sort(np.random.default_rng(2025).choice(n, 4096, replace=False))
    sub = {k: v[idx] for k, v in g128.items()}
    rs = (P0[idx], d0[idx])

    def orc(*a):
        return oracle.trace(*a, n_threads=threads)

    o = orc(spec, rs, p128)
    bad = ill_conditioned(orc, spec, rs, p128)
    rep = compare(exempt(o, bad), exempt(sub, bad), aperture=1.0, spec=spec)
    keys = ("n", "checked", "fail", "exempt_critical", "exempt_grazing", "status_mismatch",
            "tir_mismatch", "btir_mismatch", "pos_fail", "dir_fail", "steps_mismatch",
            "pos_err_max", "pos_err_p99", "dir_err_max", "dir_err_p99")
    first = {k: rep[k] for k in keys}
    first["ill_conditioned"] = int(bad.sum())
    first["sample"] = "4096 seeded rays of the 4M batch, first 128 moves each, per ray"
    st = stat_compare(oracle_full, {k: v[idx_full] for k, v in g_full.items()})
    st["sample"] = f"{len(idx_full)} rays (the cpu_baseline sample), full paths"
    return {"first_128_moves": first, "full_path_statistics": st}


def two_in_flight(vrt, torch, med, batch, rays, prm, precision, steps, g_res):
    """A stream of batches with two in flight: consecutive traces of two
    resident batches alternate over two streams, so that the last long rays of
    one trace share the device with the start of the next.  Reported beside
    value (one trace at a time), never as it; the second batch's results must
    equal the first's bitwise."""
    other = vrt.RayBatch(rays[0], rays[1], precision)
    pair = (batch, other)
    streams = (torch.cuda.Stream(), torch.cuda.Stream())
    vrt.trace_batches(med, pair, prm, precision, streams=streams)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vrt.trace_batches(med, [pair[k % 2] for k in range(steps)], prm, precision, streams=streams)
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / steps
    r2 = other.results()
    same = all(np.array_equal(g_res[key], r2[key]) for key in g_res)
    del other
    return per, same


def batch_record(vrt, torch, ctx, name, args, cpu=True):
    """One batch workload: timed traces, roofline, FP64 GPU march, the oracle's
    rate on a sample of the same rays and the parity of the timed results."""
    spec, rays, prm, precision, desc, aperture = build_workload(name, args.rays)
    n_rays = rays[0].shape[0]
    print(f"[bench] {name}: workload ready, {n_rays} rays", file=sys.stderr, flush=True)
    med = vrt.Medium(ctx, spec)
    batch = vrt.RayBatch(rays[0], rays[1], precision)
    wall, per = time_traces(vrt, torch, med, batch, prm, precision, args.steps, args.warmup)
    cnt = vrt.counters(ctx, batch)
    g_res = batch.results()
    ms = float(np.mean(per))
    ray_steps = cnt["steps"]
    value = ray_steps / (ms / 1e3)
    (t_in, t_tr, t_out), b_in, b_out = pcie_inclusive(vrt, torch, med, batch, prm, precision)
    pcie = {"ray_steps_per_s": ray_steps / ((t_in + t_tr + t_out) / 1e3),
            "ms_in": round(t_in, 3), "ms_trace": round(t_tr, 3), "ms_out": round(t_out, 3),
            "GBps_in": round(b_in / t_in / 1e6, 1), "GBps_out": round(b_out / t_out / 1e6, 1),
            "note": "batch handed over in pinned host memory: inputs in, trace, outputs out "
                    "on one stream; not value"}
    print(f"[bench] {name}: {args.steps} traces, {ms:.3f} ms each, {value:.4g} ray-steps/s",
          file=sys.stderr, flush=True)
    overlap = None
    if args.two_in_flight:
        per2, same2 = two_in_flight(vrt, torch, med, batch, rays, prm, precision, args.steps,
                                    g_res)
        overlap = {"ray_steps_per_s": ray_steps / per2, "ms_per_step": round(per2 * 1e3, 3),
                   "gain": round(ms / 1e3 / per2, 3), "bitwise_equal": bool(same2),
                   "note": "two resident batches traced alternately on two streams, host clock "
                           "around the traces; a stream of batches, not value"}
        print(f"[bench] {name}: two in flight {per2 * 1e3:.3f} ms per trace "
              f"({ray_steps / per2:.4g} ray-steps/s), bitwise equal {same2}",
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
    flops = algo_flops_per_step(name) * ray_steps
    achieved = flops / (ms / 1e3) / 1e12
    peak = PEAK_FP32_TFLOPS if precision == "fp32c" else PEAK_FP64_TFLOPS
    kernel = "march_fp32c_kernel" if precision == "fp32c" else "march_fp64_kernel"
    valu = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "algo_flops_per_ray_step": algo_flops_per_step(name)}
    if name in FP64_FLOPS_PER_STEP:
        # FP64 and FP32 work share the vector ALU: price both in FP64 time
        # (an FP32 flop costs PEAK_FP64 / PEAK_FP32 of an FP64 flop)
        f64 = FP64_FLOPS_PER_STEP[name]
        eq = f64 + algo_flops_per_step(name) * PEAK_FP64_TFLOPS / PEAK_FP32_TFLOPS
        achieved = eq * ray_steps / (ms / 1e3) / 1e12
        valu.update({"achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                     "algo_fp64_flops_per_ray_step": f64,
                     "note": "FP64-equivalent rate: FP64 flops plus FP32 flops x 78.6/157.3"})
    traffic = traffic_bytes(name) if precision == "fp32c" else None
    if name == "grid":
        # discretized media: the corner records of each visited cell from memory
        bps = algo_bytes_per_step("grid")
        gbs = bps * ray_steps / (ms / 1e3) / 1e9
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
                "algo_bytes_per_ray_step": round(bps, 3), "kernel": kernel, "valu_side": valu}
    else:
        roof = dict(valu, traffic=traffic, kernel=kernel)
    rec = {"value": value, "unit": "ray-steps/s", "ms_per_step": round(ms, 4),
           "dtype": "f32" if precision == "fp32c" else "f64",
           "config": {"workload": desc, "rays": n_rays, "ray_steps_per_trace": ray_steps,
                      "dL0": prm["dL0"], "max_steps": prm["max_steps"]},
           "wall_s": round(wall, 3), "roofline": roof, "counters": cnt,
           "pcie_inclusive": pcie}
    if overlap:
        rec["two_in_flight"] = overlap
    if fp64_gpu:
        rec["fp64_gpu_march"] = fp64_gpu
    if cpu and not args.no_cpu_baseline:
        sample = args.cpu_sample or CPU_SAMPLE.get(name, 524288)
        base, par, extra = cpu_baseline(spec, rays, prm, sample, g_res, aperture)
        rec["cpu_baseline"] = base
        if name == "grid":
            threads = base["cores"]
            rec["parity_vs_oracle"] = grid_parity(vrt, torch, med, spec, rays, prm, g_res,
                                                  extra[0], extra[1], threads)
        else:
            rec["parity_vs_oracle"] = par
    med.close()
    return rec


# oracle sample per workload: about 10-30 s of host work on 16 threads
CPU_SAMPLE = {"zernike": 32768, "spherical": 65536, "grid": 262144, "freeform": 524288}


def header(args, rec):
    out = {"metric": METRIC, "value": rec["value"], "unit": "ray-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": rec["dtype"], "data": "synthetic"}
    out.update({k: v for k, v in rec.items() if k not in out})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "freeform", "grid", "luneburg", "zernike", "spherical",
                             "helix", "served", "n2p", "adjoint"])
    ap.add_argument("--jobs", type=int, default=120, help="served: jobs in the arrival stream")
    ap.add_argument("--fp64-jobs", type=int, default=None,
                    help="served: run the one-launch-per-job FP64 baseline on this prefix")
    ap.add_argument("--load", type=float, default=0.8,
                    help="served: offered load as a fraction of the measured capacity")
    ap.add_argument("--rays", type=int, default=None)
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="rays of the oracle sample (default: about 10-30 s of host work)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-gpu", action="store_true")
    ap.add_argument("--two-in-flight", action="store_true",
                    help="single workloads: add the record of two batches in flight (the "
                         "headline run always has it)")
    ap.add_argument("--no-served", action="store_true", help="headline: skip the served record")
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
    if args.workload == "served":
        print(json.dumps(served_bench(vrt, torch, args)), flush=True)
        return 0
    if args.workload == "n2p":
        print(json.dumps(n2p_bench(vrt, torch, args)), flush=True)
        return 0
    if args.workload == "adjoint":
        print(json.dumps(adjoint_bench(vrt, torch, args)), flush=True)
        return 0
    if args.workload == "helix":
        print(json.dumps(helix_bench(vrt, torch, args)), flush=True)
        return 0
    ctx = vrt.Context(0)
    if args.workload != "headline":
        out = header(args, batch_record(vrt, torch, ctx, args.workload, args))
        ctx.close()
        print(json.dumps(out), flush=True)
        return 0
    # headline: the largest single-GPU configuration (4M rays through the
    # 256^3 quantized grid), with the freeform configuration and the served
    # mix as sub-records
    grid_args = argparse.Namespace(**vars(args))
    grid_args.rays = None
    grid_args.two_in_flight = True
    out = header(args, batch_record(vrt, torch, ctx, "grid", grid_args))
    ff_args = argparse.Namespace(**vars(args))
    ff_args.rays = None
    ff_args.two_in_flight = True
    out["freeform"] = batch_record(vrt, torch, ctx, "freeform", ff_args)
    ctx.close()
    if not args.no_served:
        out["served"] = served_bench(vrt, torch, args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
