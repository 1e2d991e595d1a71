#!/usr/bin/env python3
"""Throughput of the fused grid+degrid cadence step on one MI355X.

A step is one pass of the whole hot path over one cadence of synthetic input that
is already resident in HBM: re-plan (FP64 uv -> grid coordinates, segmentation,
counting sort of the work list by (channel, tile)) followed by the fused residual
pass (degrid the model grid, residual, grid the weighted residual, chi-squared)
over every channel and time step in one launch.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Prints one JSON line.  `value` is valid visibilities gridded and degridded per
second (Mvis/s) over the whole step; the plain path (separate grid and degrid
launches on the same plan) is timed beside it, and the dominant kernel is
reported against the HBM roofline.
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


KERNEL_SOURCES = ("tile_kernel.h", "tile_dispatch.h", "tile_fused.hip", "internal.h")
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="single_cadence", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-channels", type=int, default=32,
                    help="channels of the workload the CPU oracle runs (the whole single-cadence workload)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "tiles", "persistent"])
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-image", action="store_true", help="skip timing the imager (rts_image)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB buffer 5 times (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: channels would shard across GPUs with no exchange, "
                                   "but that layout is not a launch path of this library", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.calibrate_copy:
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 1 << 30, "copies": 5}))
        return
    import paper_1003_5575_amd as rts
    from synth import make_workload

    if args.workload == "mixed":
        return bench_mixed(args, torch, rts, make_workload)
    if args.workload == "polconv":
        return bench_polconv(args, torch, rts)
    if args.workload == "pervis":
        return bench_pervis(args, torch, rts, make_workload)
    dev = torch.device("cuda:0")
    t0 = time.time()
    wl = make_workload(args.workload, seed=args.seed)
    cfg = wl.cfg
    N, W, OS = cfg.n_grid, cfg.support, cfg.oversample
    log(f"[bench] inputs {args.workload}: B={wl.n_base} T={wl.n_time} C={cfg.n_chan} N={N} "
        f"({time.time() - t0:.1f}s)")
    uvw = torch.from_numpy(wl.uvw_m).to(dev)
    vis = torch.from_numpy(wl.vis).to(dev)
    w = torch.from_numpy(wl.weights).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed + 7)
    shape = (cfg.n_chan, N, N)
    gin = torch.complex(torch.randn(shape, generator=gen, device=dev) * 0.1,
                        torch.randn(shape, generator=gen, device=dev) * 0.1)
    model = torch.empty_like(vis)
    gout = torch.empty(shape, dtype=torch.complex64, device=dev)
    chi2 = torch.empty((), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    plan = rts.GridPlan(uvw, wl.freq_hz, w, N, wl.cell_lambda, support=W, oversample=OS, tile=args.tile,
                        schedule=args.schedule)
    info = plan.info
    n_valid = info["n_valid"]
    log(f"[bench] plan: {info}")

    def step():
        plan.update(uvw, w)
        plan.grid_degrid(vis, w, gin, model_out=model, grid_out=gout, chi2_out=chi2)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if plan.info["n_dropped"]:
        raise RuntimeError("work list overflow")

    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(K):
        ev[k][0].record(stream)
        plan.update(uvw, w)
        ev[k][1].record(stream)
        plan.grid_degrid(vis, w, gin, model_out=model, grid_out=gout, chi2_out=chi2)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_start
    ms_step = t_wall / K * 1e3
    plan_ms = float(np.mean([ev[k][0].elapsed_time(ev[k][1]) for k in range(K)]))
    fused_ms = float(np.mean([ev[k][1].elapsed_time(ev[k][2]) for k in range(K)]))
    log(f"[bench] fused step: {ms_step:.3f} ms/step (plan {plan_ms:.3f} ms, fused {fused_ms:.3f} ms)")

    plain = None
    if not args.no_plain:
        gplain = torch.empty_like(gout)
        mplain = torch.empty_like(model)
        for _ in range(2):
            plan.update(uvw, w); plan.grid(vis, w, out=gplain); plan.degrid(gin, out=mplain)
        torch.cuda.synchronize()
        evp = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
        tp = time.perf_counter()
        for k in range(K):
            evp[k][0].record(stream)
            plan.update(uvw, w)
            evp[k][1].record(stream)
            plan.grid(vis, w, out=gplain)
            evp[k][2].record(stream)
            plan.degrid(gin, out=mplain)
            evp[k][3].record(stream)
        torch.cuda.synchronize()
        ms_plain = (time.perf_counter() - tp) / K * 1e3
        g_ms = float(np.mean([evp[k][1].elapsed_time(evp[k][2]) for k in range(K)]))
        d_ms = float(np.mean([evp[k][2].elapsed_time(evp[k][3]) for k in range(K)]))
        plain = {"ms_per_step": round(ms_plain, 4), "value": round(n_valid / ms_plain / 1e3, 1),
                 "grid_kernel_ms": round(g_ms, 4), "degrid_kernel_ms": round(d_ms, 4),
                 "kernels_value": round(n_valid / (g_ms + d_ms) / 1e3, 1),
                 "fused_speedup": round(ms_plain / ms_step, 3)}
        log(f"[bench] plain: {plain}")
        del gplain, mplain

    # ---- the same step replayed from a captured HIP graph (rts_cadence_graph_*)
    graph = None
    try:
        g = plan.cadence_graph(uvw, vis, w, gin, model, gout, chi2)
        for _ in range(2):
            g.launch()
        torch.cuda.synchronize()
        evg = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        tg = time.perf_counter()
        evg[0].record(stream)
        for _ in range(K):
            g.launch()
        evg[1].record(stream)
        torch.cuda.synchronize()
        g_ms = (time.perf_counter() - tg) / K * 1e3
        graph = {"ms_per_step": round(g_ms, 4), "gpu_ms_per_step": round(evg[0].elapsed_time(evg[1]) / K, 4),
                 "value": round(n_valid / g_ms / 1e3, 1)}
        g.close()
        log(f"[bench] graph: {graph}")
    except Exception as e:      # e.g. conjugate plans, which the fused step rejects
        log(f"[bench] graph: skipped ({e})")

    # ---- differentiated configuration: forward (fused pass) + backward of the
    # chi-squared with respect to the grid and the weights, through torch.autograd
    autograd = None
    if args.workload == "differentiated":
        from paper_1003_5575_amd import autograd as ag
        Gp = gin.clone().requires_grad_(True)
        wp = w.clone().requires_grad_(True)
        def fb():
            Gp.grad = None; wp.grad = None
            loss = ag.chi2(vis, wp, Gp, plan)
            loss.backward()
        for _ in range(2):
            plan.update(uvw, w); fb()
        torch.cuda.synchronize()
        tf = time.perf_counter()
        for _ in range(K):
            plan.update(uvw, w); fb()
        torch.cuda.synchronize()
        a_ms = (time.perf_counter() - tf) / K * 1e3
        autograd = {"ms_per_step": round(a_ms, 4), "value": round(n_valid / a_ms / 1e3, 1),
                    "step": "plan update + chi2 forward (one fused pass) + backward (dL/dG, dL/dw)"}
        log(f"[bench] autograd: {autograd}")
        del Gp, wp

    # ---- imager (the step after gridding; not part of the timed step): grid ->
    # dirty image for every channel, one rts_image call
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
        pix = cfg.n_chan * N * N
        im_bytes = 2 * pix * 8          # grid read once, image written once
        imager = {"ms": round(im_ms, 4), "mpix_per_s": round(pix / im_ms / 1e3, 1),
                  "alg_bytes": im_bytes, "achieved_gbs": round(im_bytes / (im_ms * 1e-3) / 1e9, 1),
                  "frac_of_hbm_peak": round(im_bytes / (im_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "fft": "hipFFT batched in-place C2C inverse; sign and grid-correction passes are library kernels"}
        log(f"[bench] imager: {imager}")
        del img

    # ---- roofline of the dominant kernel (the fused tile kernel; its duration is
    # the rts_grid_degrid call, which adds a few-microsecond chi-squared reduction)
    block = 128 if info["tile"] <= 32 and W + 1 <= 8 else 256
    kernel_name = f"k_tile<{W + 1}, {info['seg_max']}, 2, {block}, 4> (fused)"
    touched = touched_cells(wl.uvw_m, wl.freq_hz, N, wl.cell_lambda, W, OS)
    grid_cells = cfg.n_chan * N * N
    alg_bytes = n_valid * (8 + 4 + 8) + grid_cells * 8 + touched * 8
    achieved = alg_bytes / (fused_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                # the committed counters were taken on the single-cadence workload with
                # the default tile and schedule: only that run reports them
                "traffic": measured_traffic() if (args.workload == "single_cadence" and args.tile == 0
                                                  and args.schedule == "auto") else None,
                "kernel": kernel_name, "kernel_ms": round(fused_ms, 4),
                "alg_bytes_per_launch": int(alg_bytes), "touched_cells": int(touched),
                "full_grid_read_frac": round((n_valid * 20 + 2 * grid_cells * 8) / (fused_ms * 1e-3) / 1e9
                                             / HBM_PEAK_GBS, 4)}

    # ---- CPU baseline: the FP64 oracle on a bounded sample of channels; also a
    # sampled parity check of the GPU results on those channels.
    cpu = None
    parity = None
    if not args.no_cpu:
        from oracle import cpu as ocpu
        ocpu.load()
        nch = min(args.cpu_channels, cfg.n_chan)
        chans = np.linspace(0, cfg.n_chan - 1, nch).round().astype(int)
        gin_s = gin[chans].cpu().numpy()
        tc = time.perf_counter()
        Mo, Go, chi2o = ocpu.grid_degrid(wl.uvw_m, wl.freq_hz[chans], wl.vis[chans], wl.weights[chans], gin_s,
                                         N, wl.cell_lambda, W, OS)
        t_cpu = time.perf_counter() - tc
        from oracle import oracle as O
        valid = O.coords(wl.uvw_m, wl.freq_hz[chans], wl.weights[chans], N, wl.cell_lambda, W, OS)[4]
        nv = int(valid.sum())
        cpu = {"value": round(nv / t_cpu / 1e6, 3), "unit": "Mvis/s", "cores": int(ocpu.num_threads()),
               "kind": "oracle", "sample": f"fused grid+degrid of {nch} of {cfg.n_chan} channels "
                                           f"({nv} valid visibilities) in FP64, {t_cpu:.2f} s"}
        gg = gout[chans].cpu().numpy()
        mm = model[chans].cpu().numpy()
        rel_g = max(float(np.linalg.norm(gg[i] - Go[i]) / np.linalg.norm(Go[i])) for i in range(nch))
        rel_m = max(float(np.linalg.norm(mm[i] - Mo[i]) / np.linalg.norm(Mo[i])) for i in range(nch))
        parity = {"channels": [int(c) for c in chans], "max_rel_l2_grid": rel_g, "max_rel_l2_model": rel_m,
                  "tolerance": 1e-5, "ok": bool(rel_g <= 1e-5 and rel_m <= 1e-5)}
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
                   "n_chan": cfg.n_chan, "n_base": wl.n_base, "n_time": wl.n_time, "n_grid": N,
                   "support": W, "oversample": OS, "cell_lambda": wl.cell_lambda, "tile": info["tile"],
                   "step": "plan update + fused grid/degrid, one launch each over all channels"},
        "breakdown": {"plan_ms": round(plan_ms, 4), "fused_ms": round(fused_ms, 4),
                      "fused_kernel_value": round(n_valid / fused_ms / 1e3, 1),
                      "n_segments": info["n_segments"], "n_listings": info["n_listings"]},
        "plain_path": plain,
        "graph": graph,
        "autograd": autograd,
        "imager": imager,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "context": {"paper_gpu_gridding_mvis_s_derived": 2.66, "paper_hardware": "Tesla C1060",
                    "realtime_budget": "5 GiB/s input, 8 s cadence, ~2.5 TFLOP/s whole pipeline"},
    }
    print(json.dumps(out), flush=True)


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
