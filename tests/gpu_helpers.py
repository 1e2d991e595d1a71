"""Helpers shared by the GPU tests: move a synthetic workload to the device and
compare the HIP results with the FP64 oracle."""
from __future__ import annotations

import math

import numpy as np

import oracle as O
from synth import make_workload

RTOL_L2 = 1e-5          # relative L2 bound for FP32 results against the FP64 oracle


def rel_l2(got, ref) -> float:
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(got - ref)
    return float(num / den) if den > 0 else float(num)


def fit_cell(uvw_m, freq_hz, N, W):
    umax = np.max(np.abs(uvw_m[:, :, :2])) * np.max(freq_hz) / O.C_LIGHT
    return umax / (N // 2 - (math.ceil(W / 2) + 1))


def to_dev(torch, wl, freq=None, weights=None):
    dev = torch.device("cuda:0")
    uvw = torch.from_numpy(np.ascontiguousarray(wl.uvw_m)).to(dev)
    vis = torch.from_numpy(np.ascontiguousarray(wl.vis)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(wl.weights if weights is None else weights)).to(dev)
    return uvw, vis, w


def small_case(name="single_cadence", seed=0, n_ant=40, channels=(0, 13, 31), N=256, W=7, OS=8,
               weights="ones", flag_frac=0.0, offgrid_frac=0.0):
    """A reduced workload: few antennas and channels, with optional random flags
    and samples pushed off the grid (ragged, uneven counts)."""
    wl = make_workload(name, seed=seed, channels=list(channels), n_ant=n_ant)
    freq = wl.freq_hz[wl.channels]
    du = fit_cell(wl.uvw_m, freq, N, W)
    rng = np.random.default_rng(seed + 100)
    w = wl.weights.copy()
    if weights == "uniform":
        w = rng.uniform(0.5, 1.5, w.shape).astype(np.float32)
    if flag_frac:
        w[rng.random(w.shape) < flag_frac] = 0.0
    uvw = wl.uvw_m.copy()
    if offgrid_frac:
        sel = rng.random(uvw.shape[:2]) < offgrid_frac
        uvw[sel, 0] *= 3.0
    wl.uvw_m = uvw
    wl.weights = w
    return wl, freq, du
