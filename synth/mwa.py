"""Seeded, synthetic stand-ins for the MWA visibility data of one 8 s cadence.

The paper's measurements use live MWA data, which is not available here.  These
generators reproduce its shapes instead: 512 tiles (130,816 baselines), up to 768
fine channels, a few integration steps per cadence (Table 1 and the integrator
described in Section 3), complex visibilities that are noise plus a handful of
point sources, and per-channel flagging.

Array and layout conventions (all arrays are C-contiguous):
  * uvw_m   float64 [B][T][3]  baseline coordinates in metres, time fastest
  * freq_hz float64 [C]        channel centre frequencies
  * vis     complex64 [C][B][T]
  * weights float32 [C][B][T]  0 marks a flagged sample

A baseline's T samples are contiguous ("tracks"): Earth rotation moves them by
less than one uv cell over a cadence, which is the structure the gridder exploits.

Readings that are not fixed by the paper (stated once here, listed in the design
notes as well):
  * antennas are uniform in a disc of radius 1.5 km;
  * array latitude -26.70 deg (the Boolardy site), declination -27 deg;
  * hour angles h_t = (t - (T-1)/2) * dt * omega_E with dt = 8 s / T;
  * channel centres f_c = f0 + (c + 1/2) * df;
  * point sources: S ~ U(1, 10), (l, m) ~ U(-1/(4 du), 1/(4 du)), V += S exp(-2 pi i (u l + v m));
  * the cell size du is chosen so that the longest projected baseline of the
    cadence (at the highest channel frequency, in either axis) lands
    ceil(W/2) + 1 cells inside the grid edge.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
import os

import numpy as np

C_LIGHT = 299_792_458.0          # m/s
OMEGA_EARTH = 7.2921159e-5       # rad/s (sidereal rate)
SITE_LAT_DEG = -26.70            # Boolardy station


def antenna_positions(rng: np.random.Generator, n_ant: int, radius_m: float = 1500.0) -> np.ndarray:
    """East/North/Up positions [n_ant][3] uniform in a disc (up = 0)."""
    r = radius_m * np.sqrt(rng.random(n_ant))
    th = 2.0 * np.pi * rng.random(n_ant)
    pos = np.zeros((n_ant, 3))
    pos[:, 0] = r * np.cos(th)
    pos[:, 1] = r * np.sin(th)
    return pos


def baseline_enu(pos: np.ndarray) -> np.ndarray:
    """Baselines pos[j] - pos[i] for i < j in numpy triu order, shape [B][3]."""
    i, j = np.triu_indices(pos.shape[0], k=1)
    return pos[j] - pos[i]


def uvw_tracks(enu: np.ndarray, n_time: int, dt_s: float, dec_deg: float = -27.0,
               lat_deg: float = SITE_LAT_DEG) -> np.ndarray:
    """Earth-rotation uvw tracks [B][T][3] in metres.

    Local (E, N, U) goes to equatorial (X, Y, Z) and then to (u, v, w) for hour
    angle H and declination dec, the textbook interferometry transform.
    """
    lat = math.radians(lat_deg)
    dec = math.radians(dec_deg)
    e, n, up = enu[:, 0], enu[:, 1], enu[:, 2]
    X = -n * math.sin(lat) + up * math.cos(lat)
    Y = e
    Z = n * math.cos(lat) + up * math.sin(lat)
    h = (np.arange(n_time) - (n_time - 1) / 2.0) * dt_s * OMEGA_EARTH
    sh, ch = np.sin(h)[None, :], np.cos(h)[None, :]
    X, Y, Z = X[:, None], Y[:, None], Z[:, None]
    u = sh * X + ch * Y
    v = -math.sin(dec) * ch * X + math.sin(dec) * sh * Y + math.cos(dec) * Z
    w = math.cos(dec) * ch * X - math.cos(dec) * sh * Y + math.sin(dec) * Z
    return np.ascontiguousarray(np.stack([u, v, w], axis=-1))


def channel_frequencies(n_chan: int, f0_hz: float, df_hz: float) -> np.ndarray:
    return f0_hz + (np.arange(n_chan) + 0.5) * df_hz


@dataclass(frozen=True)
class Config:
    name: str
    n_ant: int
    n_time: int
    n_chan: int
    f0_hz: float
    df_hz: float
    n_grid: int
    support: int
    oversample: int
    n_sources: int = 0
    flag_max: float = 0.0          # per-channel flag fraction ~ U(0, flag_max)
    weights: str = "ones"          # "ones" or "uniform" (U(0.5, 1.5))
    cell_lambda: float | None = None  # None: sized from the array (see module doc)
    cadence_s: float = 8.0


CONFIGS = {
    # 32 antennas, 1 time step, 1 channel at 150 MHz, 256^2 grid, W=7, OS=8.
    "tiny": Config("tiny", 32, 1, 1, 150e6 - 0.5e6, 1e6, 256, 7, 8),
    # the literal 0.5-lambda cell of the tiny case: nearly everything is off the grid
    "tiny_literal": Config("tiny_literal", 32, 1, 1, 150e6 - 0.5e6, 1e6, 256, 7, 8, cell_lambda=0.5),
    # 512 antennas, 8 steps, 32 channels over 140-170 MHz, 2048^2, W=7, OS=8, 10 sources
    "single_cadence": Config("single_cadence", 512, 8, 32, 140e6, 30e6 / 32, 2048, 7, 8, n_sources=10),
    # 768 x 40 kHz over 139-170 MHz, 4 steps, flags U(0, 0.3), 1024^2
    "batched": Config("batched", 512, 4, 768, 139e6, 40e3, 1024, 7, 8, n_sources=10, flag_max=0.3),
    # as single_cadence with weights U(0.5, 1.5) for the chi-squared fit
    "differentiated": Config("differentiated", 512, 8, 32, 140e6, 30e6 / 32, 2048, 7, 8, n_sources=10,
                             weights="uniform"),
    # 64 channels, 8 steps, 4096^2, W=16, OS=16
    "mixed": Config("mixed", 512, 8, 64, 140e6, 30e6 / 64, 4096, 16, 16, n_sources=10),
    # per-visibility kernels at the paper's timing-run sizes (12 channels, a 24 x 24
    # kernel, ~1125^2 images: 1152^2 is the nearest grid edge divisible by 64), 8 steps
    "pervis": Config("pervis", 512, 8, 12, 140e6, 30e6 / 12, 1152, 24, 8, n_sources=10),
}


@dataclass
class Workload:
    cfg: Config
    seed: int
    uvw_m: np.ndarray            # [B][T][3] float64
    freq_hz: np.ndarray          # [C] float64
    cell_lambda: float
    channels: np.ndarray         # which channels vis/weights hold
    vis: np.ndarray              # [len(channels)][B][T] complex64
    weights: np.ndarray          # [len(channels)][B][T] float32
    sources: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))

    @property
    def n_base(self) -> int:
        return self.uvw_m.shape[0]

    @property
    def n_time(self) -> int:
        return self.uvw_m.shape[1]


def _cell_size(uvw_m: np.ndarray, freq_hz: np.ndarray, n_grid: int, support: int) -> float:
    umax = float(np.max(np.abs(uvw_m[:, :, :2]))) * float(np.max(freq_hz)) / C_LIGHT
    margin = math.ceil(support / 2) + 1
    return umax / (n_grid // 2 - margin)


def _channel(args):
    (seed, c, uvw_m, f_hz, src, flag_max, weights_kind) = args
    rng = np.random.default_rng([seed, 1, c])
    B, T = uvw_m.shape[0], uvw_m.shape[1]
    noise = rng.standard_normal((B, T, 2), dtype=np.float32) * np.float32(math.sqrt(0.5))
    v = noise[..., 0].astype(np.complex128) + 1j * noise[..., 1].astype(np.complex128)
    if len(src):
        k = 2.0 * np.pi * f_hz / C_LIGHT
        u, vv = uvw_m[:, :, 0], uvw_m[:, :, 1]
        for s, l, m in src:
            v += s * np.exp(-1j * (k * (u * l + vv * m)))
    frac = rng.uniform(0.0, flag_max) if flag_max > 0 else 0.0
    flagged = rng.random((B, T)) < frac if frac > 0 else np.zeros((B, T), bool)
    if weights_kind == "uniform":
        w = rng.uniform(0.5, 1.5, (B, T)).astype(np.float32)
    else:
        w = np.ones((B, T), np.float32)
    w[flagged] = 0.0
    return v.astype(np.complex64), w


def make_workload(name_or_cfg, seed: int = 0, channels=None, threads: int | None = None,
                  n_ant: int | None = None) -> Workload:
    """Build the synthetic workload of a named configuration.

    ``channels`` selects a subset of channel indices (default: all); each channel
    is generated from its own seeded stream, so any subset reproduces exactly
    the same values as the full set.  ``n_ant`` overrides the antenna count
    (used to shrink a configuration for quick tests).
    """
    cfg = CONFIGS[name_or_cfg] if isinstance(name_or_cfg, str) else name_or_cfg
    nant = cfg.n_ant if n_ant is None else n_ant
    rng = np.random.default_rng([seed, 0])
    pos = antenna_positions(rng, nant)
    dt = cfg.cadence_s / cfg.n_time
    uvw_m = uvw_tracks(baseline_enu(pos), cfg.n_time, dt)
    freq = channel_frequencies(cfg.n_chan, cfg.f0_hz, cfg.df_hz)
    du = cfg.cell_lambda if cfg.cell_lambda is not None else _cell_size(uvw_m, freq, cfg.n_grid, cfg.support)
    srng = np.random.default_rng([seed, 2])
    src = np.zeros((cfg.n_sources, 3))
    if cfg.n_sources:
        src[:, 0] = srng.uniform(1.0, 10.0, cfg.n_sources)
        lim = 1.0 / (4.0 * du)
        src[:, 1] = srng.uniform(-lim, lim, cfg.n_sources)
        src[:, 2] = srng.uniform(-lim, lim, cfg.n_sources)
    chans = np.arange(cfg.n_chan) if channels is None else np.asarray(channels, dtype=np.int64)
    B, T = uvw_m.shape[0], uvw_m.shape[1]
    vis = np.empty((len(chans), B, T), np.complex64)
    wts = np.empty((len(chans), B, T), np.float32)
    jobs = [(seed, int(c), uvw_m, float(freq[c]), src, cfg.flag_max, cfg.weights) for c in chans]
    nthr = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=nthr) as ex:
        for i, (v, w) in enumerate(ex.map(_channel, jobs)):
            vis[i] = v
            wts[i] = w
    return Workload(cfg, seed, uvw_m, freq, du, chans, vis, wts, src)
