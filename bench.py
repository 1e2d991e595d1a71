#!/usr/bin/env python3
"""Throughput of the fused grid+degrid cadence step on one MI355X.

A step is one pass of the whole hot path over one cadence of synthetic input that
is already resident in HBM: re-plan (FP64 uv -> grid coordinates, segmentation,
counting sort of the work list by (channel, tile)) followed by the fused residual
pass (degrid the model grid, residual, grid the weighted residual, chi-squared)
over every channel and time step, replayed from the captured cadence graph at the
tile edge the library's autotuner picks.  The default workload is the batched
cadence: 768 channels x 130,816 baselines x 4 time steps, 1024^2 grids.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Prints one JSON line.  `value` is valid visibilities gridded and degridded per
second (Mvis/s) over the whole step; the plain path (one plan per channel, its
re-plan, rts_grid and rts_degrid launched channel by channel) is timed beside it,
the dominant kernel is reported against the HBM roofline (and the library's
streaming-copy bandwidth), and the FP64 oracle is timed on a channel sample on
every host core and on one core.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
METRIC = "Mvis/s gridded+degridded (support 7, FP32) and % HBM roofline vs plain path"
C_LIGHT = 299_792_458.0

WORKLOAD_TEXT = {
    "single_cadence": "plain single-cadence: 512 antennas in a 1.5 km disc (130,816 baselines), 8 time "
                      "steps of Earth rotation at dec -27 deg, 32 channels over 140-170 MHz, vis CN(0,1) + 10 "
                      "point sources, 2048x2048 complex64 grid per channel, Kaiser-Bessel W=7 OS=8",
    "batched": "batched: 512 antennas (130,816 baselines), 768 channels x 40 kHz over 139-170 MHz, 4 time "
               "steps, per-channel flags U(0,30%), 1024x1024 complex64 grid per channel, W=7 OS=8",
    "tiny": "plain gridding, tiny: 32 antennas (496 baselines), 1 time step, 1 channel at 150 MHz, 256x256 "
            "complex64 grid, Kaiser-Bessel W=7 OS=8 (launch latency)",
    "differentiated": "differentiated: as single_cadence with weights U(0.5,1.5); chi-squared "
                      "sum w|V - degrid(G)|^2 and its gradients with respect to G and w (torch.autograd)",
    "mixed": "mixed precision: 512 antennas (130,816 baselines), 64 channels over 140-170 MHz, 8 time steps, "
             "4096x4096 complex64 grid per channel, Kaiser-Bessel W=16 OS=16, BF16x3 matrix-core grid and degrid",
    "pervis": "per-visibility kernels: 512 antennas (130,816 baselines), 12 channels over 140-170 MHz, 8 time "
              "steps, 1152x1152 complex64 grid per channel, a separable W=24 OS=8 kernel per baseline (synthetic "
              "smooth bumps of per-baseline width), BF16x3 matrix-core grid and degrid",
    "polconv": "polarisation conversion: 12 channels of 1125x1125-pixel images, four complex64 polarisation "
               "products per pixel, one 4x4 complex64 matrix per pixel shared by the channels (162 MB)",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def touched_cells(uvw_m, freq_hz, N, du, W, OS):
    """Cells under at least one valid footprint, summed over channels (the grid-in
    bytes the method must read).  Snapped positions as in the library header."""
    r0 = -(OS // 2) if W % 2 else 0
    h_lo = (W - 1) // 2 if W % 2 else W // 2 - 1
    total = 0
    u = uvw_m[:, :, 0].ravel()
    v = uvw_m[:, :, 1].ravel()
    for f in freq_hz:
        s = f / (C_LIGHT * du)
        xs = np.floor((u * s + N / 2) * OS + 0.5).astype(np.int64)
        ys = np.floor((v * s + N / 2) * OS + 0.5).astype(np.int64)
        cx = np.floor_divide(xs - r0, OS)
        cy = np.floor_divide(ys - r0, OS)
        ok = (cx - h_lo >= 0) & (cx - h_lo + W <= N) & (cy - h_lo >= 0) & (cy - h_lo + W <= N)
        img = np.zeros((N + W, N + W), np.int32)
        img[cy[ok] - h_lo + W, cx[ok] - h_lo + W] = 1
        cs = img.cumsum(0).cumsum(1)
        box = cs[W:, W:] - cs[:-W, W:] - cs[W:, :-W] + cs[:-W, :-W]   # W x W box ending at (y, x)
        total += int(np.count_nonzero(box))
    return total


# The fused tile kernel's sources, and the plan's (its work list sets how many
# listings the kernel walks, so a plan change also changes the kernel's traffic).
KERNEL_SOURCES = ("tile_kernel.h", "tile_dispatch.h", "tile_fused.hip", "internal.h", "plan.hip")
POLCONV_SOURCES = ("polconv.hip", "internal.h")


def kernel_source_sha(names=KERNEL_SOURCES):
    """SHA-256 over the sources a kernel is compiled from (default: the fused tile kernel)."""
    import hashlib
    h = hashlib.sha256()
    for name in names:
        h.update(open(os.path.join(ROOT, "paper_1003_5575_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic(summary="k_tile_fused_single_cadence_traffic.json", names=KERNEL_SOURCES):
    """HBM bytes per launch of a kernel from its committed counter summary, or None
    when the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary)
    try:
        rec = json.load(open(path))
        sha = kernel_source_sha(names)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha256") != sha:
        return None
    return rec.get("traffic_bytes_per_launch")


def stats_ms(xs):
    xs = sorted(float(x) for x in xs)
    return {"mean": round(float(np.mean(xs)), 4), "median": round(float(np.median(xs)), 4),
            "min": round(xs[0], 4)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def device_copy_gbs(torch, rts, nbytes=4 << 30, reps=5):
    """Bandwidth of the library's streaming copy (each byte read and written once)
    on a 4 GiB buffer: the attainable HBM rate printed beside the published peak."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    src.fill_(1)
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        rts.stream_copy(src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        rts.stream_copy(src, dst)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return round(2 * nbytes / (ms * 1e-3) / 1e9, 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0, help="uv tile edge (0: the autotuner's choice)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-channels", type=int, default=0,
                    help="channels the CPU oracle runs on all host cores (0: a bounded default per workload)")
    ap.add_argument("--cpu-channels-1t", type=int, default=0,
                    help="channels the CPU oracle runs on one core (0: a bounded default per workload)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "tiles", "persistent"])
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-image", action="store_true", help="skip timing the imager (rts_image)")
    ap.add_argument("--no-copy", action="store_true", help="skip the reference streaming-copy bandwidth")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB buffer 5 times with the library's streaming copy "
                         "(calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: channels would shard across GPUs with "
                                   "no exchange, but no multi-GPU launch path is built", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    import paper_1003_5575_amd as rts
    if args.calibrate_copy:
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            rts.stream_copy(src, dst)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 1 << 30, "copies": 5, "kernel": "k_stream_copy"}))
        return
    from synth import make_workload

    if args.workload == "mixed":
        return bench_mixed(args, torch, rts, make_workload)
    if args.workload == "polconv":
        return bench_polconv(args, torch, rts)
    if args.workload == "pervis":
        return bench_pervis(args, torch, rts, make_workload)
    return bench_gridding(args, torch, rts, make_workload)


def bench_gridding(args, torch, rts, make_workload):
    """The W = 7 FP32 workloads.  A step is one cadence: re-plan (FP64 uv -> grid
    coordinates, segments, counting sort of the work list by (channel, tile))
    followed by the fused residual pass over every channel and time step, replayed
    from the captured cadence graph at the autotuner's tile edge."""
    dev = torch.device("cuda:0")
    t0 = time.time()
    wl = make_workload(args.workload, seed=args.seed)
    cfg = wl.cfg
    N, W, OS, C = cfg.n_grid, cfg.support, cfg.oversample, cfg.n_chan
    log(f"[bench] inputs {args.workload}: B={wl.n_base} T={wl.n_time} C={C} N={N} ({time.time() - t0:.1f}s)")
    uvw = torch.from_numpy(wl.uvw_m).to(dev)
    vis = torch.from_numpy(wl.vis).to(dev)
    w = torch.from_numpy(wl.weights).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed + 7)
    shape = (C, N, N)
    gin = torch.complex(torch.randn(shape, generator=gen, device=dev) * 0.1,
                        torch.randn(shape, generator=gen, device=dev) * 0.1)
    model = torch.empty_like(vis)
    gout = torch.empty(shape, dtype=torch.complex64, device=dev)
    chi2 = torch.empty((), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    K = args.steps

    # ---- tile edge: the library's autotuner times whole cadence steps per legal edge
    tune = None
    tile = args.tile
    if tile == 0:
        tile, tune_ms = rts.autotune_tile(uvw, wl.freq_hz, w, vis, gin, N, wl.cell_lambda, support=W,
                                          oversample=OS)
        tune = {"tile": tile, "ms_per_step": {int(k): round(float(v), 4) for k, v in tune_ms.items()}}
        log(f"[bench] autotune: {tune}")
    plan = rts.GridPlan(uvw, wl.freq_hz, w, N, wl.cell_lambda, support=W, oversample=OS, tile=tile,
                        schedule=args.schedule)
    info = plan.info
    n_valid = info["n_valid"]
    log(f"[bench] plan: {info}")

    # ---- eager steps, timed per part with HIP events on the library's stream
    for _ in range(args.warmup):
        plan.update(uvw, w)
        plan.grid_degrid(vis, w, gin, model_out=model, grid_out=gout, chi2_out=chi2)
    torch.cuda.synchronize()
    if plan.info["n_dropped"]:
        raise RuntimeError("work list overflow")
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    for k in range(K):
        ev[k][0].record(stream)
        plan.update(uvw, w)
        ev[k][1].record(stream)
        plan.grid_degrid(vis, w, gin, model_out=model, grid_out=gout, chi2_out=chi2)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    plan_ms = [ev[k][0].elapsed_time(ev[k][1]) for k in range(K)]
    fused_ms = [ev[k][1].elapsed_time(ev[k][2]) for k in range(K)]
    log(f"[bench] eager: plan {stats_ms(plan_ms)} ms, fused {stats_ms(fused_ms)} ms")

    # ---- the timed step: the captured cadence graph (re-plan + fused pass) replayed
    graph = plan.cadence_graph(uvw, vis, w, gin, model, gout, chi2)
    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()
    evg = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    t_start = time.perf_counter()
    evg[0].record(stream)
    for k in range(K):
        graph.launch()
        evg[k + 1].record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_start
    ms_step = t_wall / K * 1e3
    graph_gpu_ms = [evg[k].elapsed_time(evg[k + 1]) for k in range(K)]
    graph.close()
    if plan.info["n_dropped"]:
        raise RuntimeError("work list overflow")
    log(f"[bench] graph step: {ms_step:.3f} ms wall, gpu {stats_ms(graph_gpu_ms)} ms")

    # ---- plain path: one plan per channel, per-channel FP32 rts_grid + rts_degrid
    # launches (the paper's per-channel processing), timed with and without the
    # per-channel re-plan
    plain = None
    if not args.no_plain:
        plain = bench_plain_per_channel(torch, rts, wl, uvw, vis, w, gin, N, W, OS, tile, K, ms_step)
        log(f"[bench] plain: {plain}")

    # ---- reference bandwidth and the imager (not part of the timed step)
    copy_gbs = None if args.no_copy else device_copy_gbs(torch, rts)
    imager = None
    if not args.no_image:
        img = torch.empty_like(gout)
        plan.image(gout, out=img)          # first call builds the FFT plan
        torch.cuda.synchronize()
        evi = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        evi[0].record(stream)
        for _ in range(5):
            plan.image(gout, out=img)
        evi[1].record(stream)
        torch.cuda.synchronize()
        im_ms = evi[0].elapsed_time(evi[1]) / 5
        # In place (image over a copy of the grid): the grid is transformed as it
        # is and one pass swaps quadrants with sign and correction.  The copy is
        # made before each call, outside the timed interval.
        ip_ms = []
        for _ in range(5):
            img.copy_(gout)
            evi[0].record(stream)
            plan.image(img, out=img)
            evi[1].record(stream)
            torch.cuda.synchronize()
            ip_ms.append(evi[0].elapsed_time(evi[1]))
        ip = float(np.median(ip_ms))
        pix = C * N * N
        im_bytes = 2 * pix * 8          # grid read once, image written once
        imager = {"ms": round(im_ms, 4), "mpix_per_s": round(pix / im_ms / 1e3, 1),
                  "alg_bytes": im_bytes, "achieved_gbs": round(im_bytes / (im_ms * 1e-3) / 1e9, 1),
                  "frac_of_hbm_peak": round(im_bytes / (im_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "in_place_ms": round(ip, 4),
                  "in_place_frac_of_hbm_peak": round(im_bytes / (ip * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "fft": "hipFFT batched in-place C2C inverse (rocFFT: row FFT, transpose, row FFT, transpose); "
                         "out of place a sign pass precedes it, and a correction pass (in place: a quadrant-swap, "
                         "sign and correction pass) follows"}
        log(f"[bench] imager: {imager}")
        del img

    # ---- roofline of the dominant kernel (the fused tile kernel; its duration is
    # the rts_grid_degrid call, which adds a chi-squared reduction of a few us)
    fstat = stats_ms(fused_ms)
    touched = touched_cells(wl.uvw_m, wl.freq_hz, N, wl.cell_lambda, W, OS)
    grid_cells = C * N * N
    alg_bytes = n_valid * (8 + 4 + 8) + grid_cells * 8 + touched * 8
    achieved = alg_bytes / (fstat["mean"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(TRAFFIC_SUMMARY.get(args.workload, ""))
                if (args.tile in (0, tile) and args.schedule == "auto") else None,
                "kernel": fused_kernel_name(W, info), "kernel_ms": fstat,
                "alg_bytes_per_launch": int(alg_bytes), "touched_cells": int(touched),
                "device_copy_GBs": copy_gbs,
                "frac_of_device_copy": round(achieved / copy_gbs, 4) if copy_gbs else None,
                "full_grid_read_frac": round((n_valid * 20 + 2 * grid_cells * 8) / (fstat["mean"] * 1e-3) / 1e9
                                             / HBM_PEAK_GBS, 4)}

    # ---- CPU baseline: the FP64 C oracle on a bounded channel sample, on every host
    # core and on one core; the GPU results on those channels are checked against it.
    cpu = parity = None
    if not args.no_cpu:
        cpu, parity = cpu_baseline_and_parity(args, wl, gin, gout, model, N, W, OS)
        log(f"[bench] cpu: {cpu}  parity: {parity}")

    out = {
        "metric": METRIC,
        "value": round(n_valid / ms_step / 1e3, 1),
        "unit": "Mvis/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "n_valid": int(n_valid),
                   "n_chan": C, "n_base": wl.n_base, "n_time": wl.n_time, "n_grid": N,
                   "support": W, "oversample": OS, "cell_lambda": wl.cell_lambda, "tile": info["tile"],
                   "step": "captured cadence graph replay: plan update + fused grid/degrid, one launch each "
                           "over all channels; inputs resident in device memory"},
        "breakdown": {"plan_ms": stats_ms(plan_ms), "fused_ms": fstat,
                      "graph_gpu_ms": stats_ms(graph_gpu_ms),
                      "fused_kernel_value": round(n_valid / fstat["mean"] / 1e3, 1),
                      "n_segments": info["n_segments"], "n_listings": info["n_listings"],
                      "plan_note": "the plan update (coordinates, segments, counting sort) is the paper's "
                                   "gridding preparation; it is inside the timed step"},
        "autotune": tune,
        "plain_path": plain,
        "imager": imager,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "context": {"paper_gpu_gridding_mvis_s_derived": 2.66, "paper_hardware": "Tesla C1060",
                    "realtime_budget": "5 GiB/s input, 8 s cadence, ~2.5 TFLOP/s whole pipeline"},
    }
    plan.close()
    print(json.dumps(out), flush=True)


TRAFFIC_SUMMARY = {"single_cadence": "k_tile_fused_single_cadence_traffic.json",
                   "batched": "k_tile_fused_batched_traffic.json"}


def fused_kernel_name(W, info):
    if W + 1 <= 8:
        block = 128 if info["tile"] <= 32 else 512
    else:
        block = 256
    return f"k_tile<{W + 1}, {info['seg_max']}, 2, {block}, 4> (fused)"


def bench_plain_per_channel(torch, rts, wl, uvw, vis, w, gin, N, W, OS, tile, K, ms_fused_step):
    """Per-channel FP32 path: one plan per channel (built once, outside the timing),
    then for every channel its re-plan, rts_grid and rts_degrid launches.  The C
    entry points are called directly (no Python argument checks in the loop)."""
    import ctypes
    from paper_1003_5575_amd import _lib
    lib = _lib.load()
    C = vis.shape[0]
    gplain = torch.empty((C, N, N), dtype=torch.complex64, device=vis.device)
    mplain = torch.empty_like(vis)
    plans = []
    t0 = time.time()
    for c in range(C):
        plans.append(rts.GridPlan(uvw, wl.freq_hz[c:c + 1], w[c:c + 1], N, wl.cell_lambda, support=W,
                                  oversample=OS, tile=tile))
    build_s = time.time() - t0
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    P = ctypes.c_void_p
    ue = [(plans[c].handle, P(w[c].data_ptr()), P(vis[c].data_ptr()), P(gplain[c].data_ptr()),
           P(gin[c].data_ptr()), P(mplain[c].data_ptr())) for c in range(C)]
    up = P(uvw.data_ptr())

    def step(replan):
        for h, wp, vp, gp, gi, mp in ue:
            if replan:
                lib.rts_plan_update(h, up, wp, sp)
            lib.rts_grid(h, vp, wp, gp, sp)
            lib.rts_degrid(h, gi, mp, sp)

    out = {"plans": C, "plan_build_s": round(build_s, 2)}
    for replan in (True, False):
        step(replan)
        torch.cuda.synchronize()
        kp = max(2, K // 4)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        e0.record(stream)
        for _ in range(kp):
            step(replan)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / kp * 1e3
        gpu = e0.elapsed_time(e1) / kp
        key = "with_replan" if replan else "grid_degrid_only"
        out[key] = {"ms_per_step": round(wall, 4), "gpu_ms_per_step": round(gpu, 4), "steps": kp}
    n_valid = sum(p.info["n_valid"] for p in plans)
    out["value"] = round(n_valid / out["with_replan"]["ms_per_step"] / 1e3, 1)
    out["fused_speedup"] = round(out["with_replan"]["ms_per_step"] / ms_fused_step, 3)
    out["launches_per_step"] = "per channel: re-plan (5-7 kernels) + rts_grid + rts_degrid"
    for p in plans:
        p.close()
    del gplain, mplain
    torch.cuda.empty_cache()
    return out


def cpu_baseline_and_parity(args, wl, gin, gout, model, N, W, OS):
    from oracle import cpu as ocpu
    from oracle import oracle as O
    ocpu.load()
    C = wl.vis.shape[0]
    # about 10-30 core-seconds of oracle work on the all-core sample
    defaults = {"batched": (256, 32), "single_cadence": (32, 4), "differentiated": (32, 4), "tiny": (1, 1)}
    n_all, n_one = defaults.get(args.workload, (8, 1))
    n_all = min(args.cpu_channels or n_all, C)
    n_one = min(args.cpu_channels_1t or n_one, C)
    chans = np.linspace(0, C - 1, n_all).round().astype(int)
    gin_s = gin[chans].cpu().numpy()
    cores = host_cores()
    ocpu.set_num_threads(cores)
    threads = int(ocpu.num_threads())
    tc = time.perf_counter()
    Mo, Go, chi2o = ocpu.grid_degrid(wl.uvw_m, wl.freq_hz[chans], wl.vis[chans], wl.weights[chans], gin_s,
                                     N, wl.cell_lambda, W, OS)
    t_all = time.perf_counter() - tc
    valid = O.coords(wl.uvw_m, wl.freq_hz[chans], wl.weights[chans], N, wl.cell_lambda, W, OS)[4]
    nv = int(valid.sum())
    # one core, the first n_one channels of the sample
    sub = chans[:n_one]
    ocpu.set_num_threads(1)
    tc = time.perf_counter()
    ocpu.grid_degrid(wl.uvw_m, wl.freq_hz[sub], wl.vis[sub], wl.weights[sub], gin_s[:n_one], N, wl.cell_lambda,
                     W, OS, want_model=False)
    t_one = time.perf_counter() - tc
    ocpu.set_num_threads(cores)
    nv1 = int(valid[:n_one].sum())
    cpu = {"value": round(nv / t_all / 1e6, 3), "unit": "Mvis/s", "cores": threads, "kind": "oracle",
           "sample": f"fused grid+degrid of {n_all} of {C} channels ({nv} valid visibilities) in FP64 "
                     f"(C, OpenMP over channels), {t_all:.2f} s",
           "cpu_model": cpu_model(),
           "single_thread": {"value": round(nv1 / t_one / 1e6, 3), "unit": "Mvis/s", "cores": 1,
                             "sample": f"{n_one} of those channels ({nv1} valid visibilities), {t_one:.2f} s"}}
    gg = gout[chans].cpu().numpy()
    mm = model[chans].cpu().numpy()
    rel_g = max(float(np.linalg.norm(gg[i] - Go[i]) / np.linalg.norm(Go[i])) for i in range(n_all))
    rel_m = max(float(np.linalg.norm(mm[i] - Mo[i]) / np.linalg.norm(Mo[i])) for i in range(n_all))
    parity = {"channels": [int(c) for c in chans], "max_rel_l2_grid": rel_g, "max_rel_l2_model": rel_m,
              "tolerance": 1e-5, "ok": bool(rel_g <= 1e-5 and rel_m <= 1e-5)}
    return cpu, parity


def bench_mixed(args, torch, rts, make_workload):
    """The mixed-precision configuration: a step is the plan update plus BF16x3
    gridding and BF16x3 degridding (two launches over all channels).  The FP32
    path on the same inputs is timed beside it, and the BF16x3 error against the
    FP64 oracle is reported per channel on a sample of channels."""
    dev = torch.device("cuda:0")
    wl = make_workload("mixed", seed=args.seed)
    cfg = wl.cfg
    N, W, OS = cfg.n_grid, cfg.support, cfg.oversample
    uvw = torch.from_numpy(wl.uvw_m).to(dev)
    vis = torch.from_numpy(wl.vis).to(dev)
    w = torch.from_numpy(wl.weights).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed + 7)
    shape = (cfg.n_chan, N, N)
    gin = torch.complex(torch.randn(shape, generator=gen, device=dev) * 0.1,
                        torch.randn(shape, generator=gen, device=dev) * 0.1)
    gout = torch.empty(shape, dtype=torch.complex64, device=dev)
    model = torch.empty_like(vis)
    stream = torch.cuda.current_stream()
    plan = rts.GridPlan(uvw, wl.freq_hz, w, N, wl.cell_lambda, support=W, oversample=OS, precision="bf16x3")
    info = plan.info
    n_valid = info["n_valid"]
    log(f"[bench] mixed plan: {info}")

    def timed(p, K):
        for _ in range(args.warmup):
            p.update(uvw, w); p.grid(vis, w, out=gout); p.degrid(gin, out=model)
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
        t0 = time.perf_counter()
        for k in range(K):
            ev[k][0].record(stream)
            p.update(uvw, w)
            ev[k][1].record(stream)
            p.grid(vis, w, out=gout)
            ev[k][2].record(stream)
            p.degrid(gin, out=model)
            ev[k][3].record(stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / K * 1e3
        parts = [float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(K)])) for i in range(3)]
        return ms, parts

    chi2 = torch.empty((), dtype=torch.float64, device=dev)

    def timed_fused(p, K):
        """The fused residual step alone (degrid, grid w (V - M), chi2) on the same inputs."""
        for _ in range(args.warmup):
            p.grid_degrid(vis, w, gin, model_out=model, grid_out=gout, chi2_out=chi2)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
        ev[0].record(stream)
        for k in range(K):
            p.grid_degrid(vis, w, gin, model_out=model, grid_out=gout, chi2_out=chi2)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(K)]))

    K = args.steps
    fused_ms = timed_fused(plan, K)
    ms, (plan_ms, g_ms, d_ms) = timed(plan, K)
    # per-channel error of the BF16x3 results on sampled channels
    errs = None
    if not args.no_cpu:
        from oracle import cpu as ocpu
        chans = np.linspace(0, cfg.n_chan - 1, 4).round().astype(int)
        Gb = gout[chans].cpu().numpy()
        Mb = model[chans].cpu().numpy()
        tc = time.perf_counter()
        Go = ocpu.grid(wl.uvw_m, wl.freq_hz[chans], wl.vis[chans], wl.weights[chans], N, wl.cell_lambda, W, OS)
        Mo = ocpu.degrid(wl.uvw_m, wl.freq_hz[chans], wl.weights[chans], gin[chans].cpu().numpy(), N,
                         wl.cell_lambda, W, OS)
        t_cpu = time.perf_counter() - tc
        errs = {"channels": [int(c) for c in chans],
                "grid_rel_l2": [float(np.linalg.norm(Gb[i] - Go[i]) / np.linalg.norm(Go[i])) for i in range(len(chans))],
                "degrid_rel_l2": [float(np.linalg.norm(Mb[i] - Mo[i]) / np.linalg.norm(Mo[i])) for i in range(len(chans))],
                "oracle_seconds": round(t_cpu, 2), "oracle_cores": int(ocpu.num_threads())}
        log(f"[bench] mixed errors: {errs}")
    plan.close()
    plan32 = rts.GridPlan(uvw, wl.freq_hz, w, N, wl.cell_lambda, support=W, oversample=OS)
    ms32, (p32, g32, d32) = timed(plan32, K)
    fused32 = timed_fused(plan32, K)
    tile32 = plan32.info["tile"]
    plan32.close()
    # FP32 operands on the matrix cores, same inputs; error on the same channels
    planm = rts.GridPlan(uvw, wl.freq_hz, w, N, wl.cell_lambda, support=W, oversample=OS, precision="fp32_mfma")
    fusedm = timed_fused(planm, K)
    msm, (pm, gm, dm) = timed(planm, K)
    planm.close()
    errs_m = None
    if errs is not None:
        Gm = gout[chans].cpu().numpy()
        Mm = model[chans].cpu().numpy()
        errs_m = {"channels": errs["channels"],
                  "grid_rel_l2": [float(np.linalg.norm(Gm[i] - Go[i]) / np.linalg.norm(Go[i])) for i in range(len(chans))],
                  "degrid_rel_l2": [float(np.linalg.norm(Mm[i] - Mo[i]) / np.linalg.norm(Mo[i])) for i in range(len(chans))]}
        log(f"[bench] mixed fp32_mfma errors: {errs_m}")
    nl = info["n_listings"]
    out = {
        "metric": METRIC, "value": round(n_valid / ms / 1e3, 1), "unit": "Mvis/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["mixed"], "n_valid": int(n_valid), "n_chan": cfg.n_chan,
                   "n_grid": N, "support": W, "oversample": OS, "tile": info["tile"],
                   "step": "plan update + BF16x3 grid + BF16x3 degrid, one launch each over all channels"},
        "breakdown": {"plan_ms": round(plan_ms, 4), "grid_ms": round(g_ms, 4), "degrid_ms": round(d_ms, 4),
                      "fused_step_ms": round(fused_ms, 4), "n_listings": nl, "seg_max": info["seg_max"]},
        "fp32_path": {"ms_per_step": round(ms32, 4), "value": round(n_valid / ms32 / 1e3, 1), "tile": tile32,
                      "plan_ms": round(p32, 4), "grid_ms": round(g32, 4), "degrid_ms": round(d32, 4),
                      "fused_step_ms": round(fused32, 4)},
        "fp32_mfma_path": {"ms_per_step": round(msm, 4), "value": round(n_valid / msm / 1e3, 1),
                           "plan_ms": round(pm, 4), "grid_ms": round(gm, 4), "degrid_ms": round(dm, 4),
                           "fused_step_ms": round(fusedm, 4), "error": errs_m},
        "bf16x3_error": errs,
    }
    print(json.dumps(out), flush=True)


def bench_pervis(args, torch, rts, make_workload):
    """Per-visibility kernels (a separable W=24 kernel per baseline): a step is the
    plan update plus BF16x3 gridding and degridding over all channels with the
    per-baseline tables; the same plan with the shared Kaiser-Bessel kernel is
    timed beside it.  The BF16x3 error and the CPU baseline use the FP64 oracle on
    a sample (one channel, the first 8192 baselines) gridded by its own plan."""
    from synth import make_baseline_kernels
    import oracle as O
    dev = torch.device("cuda:0")
    wl = make_workload("pervis", seed=args.seed)
    cfg = wl.cfg
    N, W, OS, C = cfg.n_grid, cfg.support, cfg.oversample, cfg.n_chan
    B = wl.uvw_m.shape[0]
    tab_np = make_baseline_kernels(B, W, OS, seed=args.seed + 11)
    uvw = torch.from_numpy(wl.uvw_m).to(dev)
    vis = torch.from_numpy(wl.vis).to(dev)
    w = torch.from_numpy(wl.weights).to(dev)
    tab = torch.from_numpy(tab_np).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed + 7)
    shape = (C, N, N)
    gin = torch.complex(torch.randn(shape, generator=gen, device=dev) * 0.1,
                        torch.randn(shape, generator=gen, device=dev) * 0.1)
    gout = torch.empty(shape, dtype=torch.complex64, device=dev)
    model = torch.empty_like(vis)
    stream = torch.cuda.current_stream()
    plan = rts.GridPlan(uvw, wl.freq_hz, w, N, wl.cell_lambda, support=W, oversample=OS, precision="bf16x3")
    plan.set_baseline_kernels(tab)
    info = plan.info
    n_valid = info["n_valid"]
    log(f"[bench] pervis plan: {info}")

    def timed(K):
        for _ in range(args.warmup):
            plan.update(uvw, w); plan.grid(vis, w, out=gout); plan.degrid(gin, out=model)
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
        t0 = time.perf_counter()
        for k in range(K):
            ev[k][0].record(stream)
            plan.update(uvw, w)
            ev[k][1].record(stream)
            plan.grid(vis, w, out=gout)
            ev[k][2].record(stream)
            plan.degrid(gin, out=model)
            ev[k][3].record(stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / K * 1e3
        return ms, [float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(K)])) for i in range(3)]

    chi2 = torch.empty((), dtype=torch.float64, device=dev)

    def timed_fused(K):
        """The fused residual step alone (degrid, grid w (V - M), chi2) with the plan's kernels."""
        for _ in range(args.warmup):
            plan.grid_degrid(vis, w, gin, model_out=model, grid_out=gout, chi2_out=chi2)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
        ev[0].record(stream)
        for k in range(K):
            plan.grid_degrid(vis, w, gin, model_out=model, grid_out=gout, chi2_out=chi2)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(K)]))

    K = args.steps
    fused_ms = timed_fused(K)
    ms, (plan_ms, g_ms, d_ms) = timed(K)
    plan.set_baseline_kernels(None)
    ms_sh, (_, g_sh, d_sh) = timed(K)
    plan.close()
    # FP32 operands on the matrix cores, per-baseline kernels
    plan = rts.GridPlan(uvw, wl.freq_hz, w, N, wl.cell_lambda, support=W, oversample=OS, precision="fp32_mfma")
    plan.set_baseline_kernels(tab)
    ms_m, (_, g_m, d_m) = timed(K)
    fused_m = timed_fused(K)
    plan.close()
    # algorithmic bytes of grid + degrid: visibilities and weights read and model
    # written (20 B per valid sample), the grids written, the touched cells read,
    # and the per-baseline tables once
    touched = touched_cells(wl.uvw_m, wl.freq_hz, N, wl.cell_lambda, W, OS)
    alg = n_valid * 20 + C * N * N * 8 + touched * 8 + B * OS * W * 4
    kms = g_ms + d_ms
    errs, cpu = None, None
    if not args.no_cpu:
        nb = 8192
        sub_uvw = np.ascontiguousarray(wl.uvw_m[:nb])
        sub_vis = np.ascontiguousarray(wl.vis[:1, :nb])
        sub_w = np.ascontiguousarray(wl.weights[:1, :nb])
        f1 = wl.freq_hz[:1]
        sp = rts.GridPlan(torch.from_numpy(sub_uvw).to(dev), f1, torch.from_numpy(sub_w).to(dev), N, wl.cell_lambda,
                          support=W, oversample=OS, precision="bf16x3")
        sp.set_baseline_kernels(torch.from_numpy(np.ascontiguousarray(tab_np[:nb])).to(dev))
        Gs = sp.grid(torch.from_numpy(sub_vis).to(dev), torch.from_numpy(sub_w).to(dev)).cpu().numpy()
        Ms = sp.degrid(gin[:1].contiguous()).cpu().numpy()
        sp.close()
        tc = time.perf_counter()
        geom = O.Geometry(sub_uvw, f1, sub_w, N, wl.cell_lambda, W, OS)
        Go = O.grid_per_baseline(geom, sub_vis, sub_w, tab_np[:nb])
        Mo = O.degrid_per_baseline(geom, gin[:1].cpu().numpy().astype(np.complex128), tab_np[:nb])
        dt = time.perf_counter() - tc
        nv = int(geom.valid.sum())
        errs = {"sample": f"channel 0, baselines 0-{nb - 1} ({nv} valid samples), own plan",
                "grid_rel_l2": float(np.linalg.norm(Gs[0] - Go[0]) / np.linalg.norm(Go[0])),
                "degrid_rel_l2": float(np.linalg.norm(Ms - Mo) / np.linalg.norm(Mo))}
        cpu = {"value": round(nv / dt / 1e6, 3), "unit": "Mvis/s", "cores": 1, "kind": "oracle",
               "sample": f"grid + degrid of channel 0, baselines 0-{nb - 1} ({nv} valid samples) with "
                         f"per-baseline kernels in FP64 (numpy), {dt:.1f} s"}
        log(f"[bench] pervis errors: {errs}")
    out = {
        "metric": "Mvis/s gridded+degridded with per-visibility kernels (W=24, BF16x3)",
        "value": round(n_valid / ms / 1e3, 1), "unit": "Mvis/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16x3", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["pervis"], "n_valid": int(n_valid), "n_chan": C, "n_grid": N,
                   "support": W, "oversample": OS, "tile": info["tile"],
                   "step": "plan update + BF16x3 grid + BF16x3 degrid with per-baseline kernels"},
        "breakdown": {"plan_ms": round(plan_ms, 4), "grid_ms": round(g_ms, 4), "degrid_ms": round(d_ms, 4),
                      "fused_step_ms": round(fused_ms, 4), "n_listings": info["n_listings"],
                      "seg_max": info["seg_max"]},
        "shared_kernel": {"ms_per_step": round(ms_sh, 4), "grid_ms": round(g_sh, 4), "degrid_ms": round(d_sh, 4)},
        "fp32_mfma": {"ms_per_step": round(ms_m, 4), "grid_ms": round(g_m, 4), "degrid_ms": round(d_m, 4),
                      "fused_step_ms": round(fused_m, 4)},
        "roofline": {"bound": "hbm", "achieved": round(alg / kms / 1e6, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / kms / 1e6 / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_grid_mfma_bf16x3<2, true, false, false> + k_degrid_mfma_bf16x3<2, true, false>",
                     "kernel_ms": round(kms, 4), "alg_bytes_per_launch": int(alg), "touched_cells": int(touched)},
        "cpu_baseline": cpu,
        "bf16x3_error": errs,
    }
    print(json.dumps(out), flush=True)


def bench_polconv(args, torch, rts):
    """Polarisation conversion S_i = A_i P_i on the image sizes of the paper's
    timing run (12 channels, 1125 x 1125 pixels); a step is one rts_polconvert
    launch over all channels.  HBM-bound: 128 bytes of matrix per pixel plus 64
    bytes of products in and out per pixel and channel."""
    from synth import make_polconv_inputs
    n_side, C = 1125, 12
    n = n_side * n_side
    A_np, P_np = make_polconv_inputs(n, C, seed=args.seed)
    A = torch.from_numpy(A_np).cuda()
    P = torch.from_numpy(P_np).cuda()
    S = torch.empty_like(P)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        rts.polconvert(A, P, out=S)
    torch.cuda.synchronize()
    K = args.steps
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(K):
        rts.polconvert(A, P, out=S)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / K * 1e3
    kms = float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(K)]))
    alg = n * (16 * 8 + C * 8 * 8)
    # reference: a 1 GiB device-to-device copy (read + write) on the same device
    src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * (1 << 30) * 5 / e0.elapsed_time(e1) / 1e6
    del src, dst
    cpu = None
    if not args.no_cpu:
        from oracle import polconvert as opc
        tc = time.perf_counter()
        opc(A_np.reshape(4, 4, n), P_np)
        dt = time.perf_counter() - tc
        cpu = {"value": round(n * C / dt / 1e6, 2), "unit": "Mpix/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole workload ({C} channels x {n} pixels) in FP64 (numpy), {dt:.2f} s"}
    out = {
        "metric": "polarisation conversion S_i = A_i P_i, pixel-channels per second", "value":
        round(n * C / ms / 1e3, 1), "unit": "Mpix/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT["polconv"], "n_pix": n, "n_chan": C},
        "roofline": {"bound": "hbm", "achieved": round(alg / kms / 1e6, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / kms / 1e6 / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("k_polconv_traffic.json", POLCONV_SOURCES),
                     "kernel": "k_polconv_pairs" if n % 2 == 0 else "k_polconv_single", "kernel_ms": round(kms, 4),
                     "alg_bytes_per_launch": alg, "device_copy_GBs": round(copy_gbs, 1)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
