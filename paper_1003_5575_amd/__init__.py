"""rtsgrid for AMD MI355X: convolutional gridding / degridding of radio visibilities.

A thin binding over librtsgrid.so (C ABI, hand-written HIP kernels for gfx950).
PyTorch supplies device memory and streams only; every step of the computation
runs in the library's kernels.  See include/rtsgrid.h for the exact semantics.

    plan = GridPlan(uvw, freq_hz, weights, n_grid=2048, cell_lambda=du)
    G = plan.grid(vis, weights)                 # Eq. (1)
    M = plan.degrid(G)                          # adjoint
    M, G_out, chi2 = plan.grid_degrid(vis, weights, G_in)
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import RtsError, RtsParams, RtsPlanInfo  # noqa: F401

__all__ = ["GridPlan", "CadenceGraph", "autotune_tile", "compute_coords", "polconvert", "stream_copy", "RtsError", "library_path", "version", "GridFn", "DegridFn",
           "Chi2Fn", "grid", "degrid", "chi2"]


def _torch():
    import torch
    return torch


def library_path() -> str:
    return _lib.LIB_PATH


def version() -> str:
    return _lib.load().rts_version().decode()


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_dev(t, name, dtype, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


PRECISIONS = {"fp32": 0, "bf16x3": 1, "fp32_mfma": 2}
SCHEDULES = {"auto": 0, "tiles": 1, "persistent": 2}


def make_params(n_grid, cell_lambda, support, oversample, n_chan, n_base, n_time, beta=None,
                conjugate=False, tile=0, precision="fp32", schedule="auto") -> RtsParams:
    p = RtsParams()
    p.n_grid, p.support, p.oversample = int(n_grid), int(support), int(oversample)
    p.n_chan, p.n_base, p.n_time = int(n_chan), int(n_base), int(n_time)
    p.cell_lambda = float(cell_lambda)
    p.beta = float(beta) if beta is not None else 0.0
    p.conjugate = int(bool(conjugate))
    p.tile = int(tile)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    return p


class GridPlan:
    """A gridding plan over one cadence: uvw [B][T][3] (float64, metres, device),
    freq_hz [C] (host sequence), weights [C][B][T] (float32, device; 0 = flagged).

    precision: "fp32" (vector tile kernels, FP64 tile accumulation), "bf16x3"
    (grid and degrid on the matrix cores with BF16 hi+lo operands) or "fp32_mfma"
    (the same with FP32 operands); the matrix-core modes accept supports up to 24
    and per-baseline kernels (set_baseline_kernels).  schedule: "auto", "tiles"
    or "persistent" (launch of the FP32 tile kernels)."""

    def __init__(self, uvw, freq_hz, weights, n_grid, cell_lambda, support=7, oversample=8,
                 beta=None, conjugate=False, tile=0, stream=None, precision="fp32", schedule="auto"):
        torch = _torch()
        lib = _lib.load()
        _check_dev(uvw, "uvw", torch.float64)
        if uvw.dim() != 3 or uvw.shape[2] != 3:
            raise ValueError("uvw must be [B][T][3]")
        B, T = int(uvw.shape[0]), int(uvw.shape[1])
        freq = [float(f) for f in freq_hz]
        C = len(freq)
        _check_dev(weights, "weights", torch.float32, (C, B, T))
        self.params = make_params(n_grid, cell_lambda, support, oversample, C, B, T, beta, conjugate, tile,
                                  precision, schedule)
        self.C, self.B, self.T, self.N = C, B, T, int(n_grid)
        self.device = uvw.device
        self._freq = (ctypes.c_double * C)(*freq)
        h = ctypes.c_void_p()
        _lib.check(lib.rts_grid_plan(ctypes.byref(h), ctypes.byref(self.params), _ptr(uvw),
                                     ctypes.cast(self._freq, ctypes.c_void_p), _ptr(weights), _stream(stream)),
                   "rts_grid_plan")
        self._h = h

    # ------------------------------------------------------------------ queries
    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise RuntimeError("plan has been destroyed")
        return self._h

    @property
    def info(self) -> dict:
        inf = RtsPlanInfo()
        _lib.check(_lib.load().rts_plan_get_info(self.handle, ctypes.byref(inf)), "rts_plan_get_info")
        return {k: getattr(inf, k) for k, _ in RtsPlanInfo._fields_}

    def valid_mask(self, stream=None):
        """bool [C][B][T]: samples this plan grids (w != 0 at plan time, all taps on the grid)."""
        torch = _torch()
        out = torch.empty((self.C, self.B, self.T), dtype=torch.uint8, device=self.device)
        _lib.check(_lib.load().rts_plan_valid_mask(self.handle, _ptr(out), _stream(stream)), "rts_plan_valid_mask")
        return out.bool()

    def table(self):
        import numpy as np
        n = self.params.oversample * self.params.support
        buf = np.zeros(n, np.float32)
        _lib.check(_lib.load().rts_plan_get_table(self.handle, ctypes.c_void_p(buf.ctypes.data), n),
                   "rts_plan_get_table")
        return buf.reshape(self.params.oversample, self.params.support)

    def update(self, uvw, weights, stream=None):
        """Re-plan in place for new uvw / weights of the same shape (asynchronous)."""
        torch = _torch()
        _check_dev(uvw, "uvw", torch.float64, (self.B, self.T, 3))
        _check_dev(weights, "weights", torch.float32, (self.C, self.B, self.T))
        _lib.check(_lib.load().rts_plan_update(self.handle, _ptr(uvw), _ptr(weights), _stream(stream)),
                   "rts_plan_update")

    # -------------------------------------------------------------- operations
    def _vis_shape(self):
        return (self.C, self.B, self.T)

    def _grid_shape(self):
        return (self.C, self.N, self.N)

    def grid(self, vis, weights, out=None, stream=None):
        """Eq. (1): complex64 [C][N][N] (overwritten)."""
        torch = _torch()
        _check_dev(vis, "vis", torch.complex64, self._vis_shape())
        _check_dev(weights, "weights", torch.float32, self._vis_shape())
        if out is None:
            out = torch.empty(self._grid_shape(), dtype=torch.complex64, device=vis.device)
        _check_dev(out, "out", torch.complex64, self._grid_shape())
        _lib.check(_lib.load().rts_grid(self.handle, _ptr(vis), _ptr(weights), _ptr(out), _stream(stream)),
                   "rts_grid")
        return out

    def degrid(self, grid, out=None, stream=None):
        """Adjoint (no weights): complex64 [C][B][T], 0 at invalid samples."""
        torch = _torch()
        _check_dev(grid, "grid", torch.complex64, self._grid_shape())
        if out is None:
            out = torch.empty(self._vis_shape(), dtype=torch.complex64, device=grid.device)
        _check_dev(out, "out", torch.complex64, self._vis_shape())
        _lib.check(_lib.load().rts_degrid(self.handle, _ptr(grid), _ptr(out), _stream(stream)), "rts_degrid")
        return out

    def set_baseline_kernels(self, tab, stream=None):
        """Per-visibility kernels (rts_plan_set_baseline_kernels): ``tab`` float32
        [B, OS, W] on the device, baseline b's separable kernel sampled in the
        layout of ``table``; None restores the shared kernel.  Matrix-core plans only
        (precision "bf16x3" or "fp32_mfma")."""
        torch = _torch()
        if tab is None:
            _lib.check(_lib.load().rts_plan_set_baseline_kernels(self.handle, None, _stream(stream)),
                       "rts_plan_set_baseline_kernels")
            return
        p = self.params
        _check_dev(tab, "tab", torch.float32, (p.n_base, p.oversample, p.support))
        _lib.check(_lib.load().rts_plan_set_baseline_kernels(self.handle, _ptr(tab), _stream(stream)),
                   "rts_plan_set_baseline_kernels")

    def image(self, grid, out=None, stream=None):
        """Dirty image of every channel: complex64 [C][N][N], the centred inverse FFT of
        the grid (unnormalised) divided by the grid correction (rts_image)."""
        torch = _torch()
        _check_dev(grid, "grid", torch.complex64, self._grid_shape())
        if out is None:
            out = torch.empty(self._grid_shape(), dtype=torch.complex64, device=grid.device)
        _check_dev(out, "out", torch.complex64, self._grid_shape())
        _lib.check(_lib.load().rts_image(self.handle, _ptr(grid), _ptr(out), _stream(stream)), "rts_image")
        return out

    def grid_degrid(self, vis, weights, grid_in, model_out=True, grid_out=None, chi2_out=True,
                    stream=None):
        """Fused residual step.  Returns (model or None, grid_out, chi2 tensor or None)."""
        torch = _torch()
        _check_dev(vis, "vis", torch.complex64, self._vis_shape())
        _check_dev(weights, "weights", torch.float32, self._vis_shape())
        _check_dev(grid_in, "grid_in", torch.complex64, self._grid_shape())
        dev = vis.device
        if model_out is True:
            model_out = torch.empty(self._vis_shape(), dtype=torch.complex64, device=dev)
        elif model_out is False:
            model_out = None
        if model_out is not None:
            _check_dev(model_out, "model_out", torch.complex64, self._vis_shape())
        if grid_out is None:
            grid_out = torch.empty(self._grid_shape(), dtype=torch.complex64, device=dev)
        _check_dev(grid_out, "grid_out", torch.complex64, self._grid_shape())
        if chi2_out is True:
            chi2_out = torch.empty((), dtype=torch.float64, device=dev)
        elif chi2_out is False:
            chi2_out = None
        if chi2_out is not None:
            _check_dev(chi2_out, "chi2_out", torch.float64)
        _lib.check(_lib.load().rts_grid_degrid(self.handle, _ptr(vis), _ptr(weights), _ptr(grid_in),
                                               _ptr(model_out), _ptr(grid_out), _ptr(chi2_out),
                                               _stream(stream)), "rts_grid_degrid")
        return model_out, grid_out, chi2_out

    def grid_backward(self, vis, weights, grad_grid, want_weights=True, stream=None):
        """Gradients through grid(vis, weights) (rts_grid_backward): returns
        (w * D(grad_grid), Re(conj(vis) * D(grad_grid)) or None)."""
        torch = _torch()
        _check_dev(vis, "vis", torch.complex64, self._vis_shape())
        _check_dev(weights, "weights", torch.float32, self._vis_shape())
        _check_dev(grad_grid, "grad_grid", torch.complex64, self._grid_shape())
        gv = torch.empty(self._vis_shape(), dtype=torch.complex64, device=vis.device)
        gw = torch.empty(self._vis_shape(), dtype=torch.float32, device=vis.device) if want_weights else None
        _lib.check(_lib.load().rts_grid_backward(self.handle, _ptr(vis), _ptr(weights), _ptr(grad_grid), _ptr(gv),
                                                 _ptr(gw), _stream(stream)), "rts_grid_backward")
        return gv, gw

    def chi2_backward(self, vis, weights, model, grid_resid, grad_chi2, want=(True, True, True), stream=None):
        """Gradients of the fused step's chi-squared (rts_chi2_backward): from the
        model and the residual grid it wrote and dL/dchi2 (a float64 device scalar),
        returns (dL/dvis, dL/dweights, dL/dgrid), each None where not wanted."""
        torch = _torch()
        _check_dev(vis, "vis", torch.complex64, self._vis_shape())
        _check_dev(weights, "weights", torch.float32, self._vis_shape())
        _check_dev(model, "model", torch.complex64, self._vis_shape())
        _check_dev(grid_resid, "grid_resid", torch.complex64, self._grid_shape())
        _check_dev(grad_chi2, "grad_chi2", torch.float64)
        if grad_chi2.numel() != 1:
            raise ValueError("grad_chi2 must hold one value")
        dev = vis.device
        gv = torch.empty(self._vis_shape(), dtype=torch.complex64, device=dev) if want[0] else None
        gw = torch.empty(self._vis_shape(), dtype=torch.float32, device=dev) if want[1] else None
        gg = torch.empty(self._grid_shape(), dtype=torch.complex64, device=dev) if want[2] else None
        _lib.check(_lib.load().rts_chi2_backward(self.handle, _ptr(vis), _ptr(weights), _ptr(model),
                                                 _ptr(grid_resid), _ptr(grad_chi2), _ptr(gv), _ptr(gw), _ptr(gg),
                                                 _stream(stream)), "rts_chi2_backward")
        return gv, gw, gg

    def cadence_graph(self, uvw, vis, weights, grid_in, model_out, grid_out, chi2_out, stream=None):
        """Capture [update(uvw, weights); grid_degrid(...)] once; see CadenceGraph."""
        return CadenceGraph(self, uvw, vis, weights, grid_in, model_out, grid_out, chi2_out, stream)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.load().rts_plan_destroy(self._h), "rts_plan_destroy")
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class CadenceGraph:
    """A captured cadence step (re-plan + fused pass) replayed with one graph launch.

    The tensors passed at capture are the ones every replay reads and writes: copy
    the next cadence's uvw, weights and visibilities into them, then launch()."""

    def __init__(self, plan, uvw, vis, weights, grid_in, model_out, grid_out, chi2_out, stream=None):
        torch = _torch()
        _check_dev(uvw, "uvw", torch.float64, (plan.B, plan.T, 3))
        _check_dev(vis, "vis", torch.complex64, plan._vis_shape())
        _check_dev(weights, "weights", torch.float32, plan._vis_shape())
        _check_dev(grid_in, "grid_in", torch.complex64, plan._grid_shape())
        _check_dev(grid_out, "grid_out", torch.complex64, plan._grid_shape())
        if model_out is not None:
            _check_dev(model_out, "model_out", torch.complex64, plan._vis_shape())
        if chi2_out is not None:
            _check_dev(chi2_out, "chi2_out", torch.float64)
        self._keep = (plan, uvw, vis, weights, grid_in, model_out, grid_out, chi2_out)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().rts_cadence_graph_create(ctypes.byref(h), plan.handle, _ptr(uvw), _ptr(vis),
                                                        _ptr(weights), _ptr(grid_in), _ptr(model_out),
                                                        _ptr(grid_out), _ptr(chi2_out), _stream(stream)),
                   "rts_cadence_graph_create")
        self._h = h

    def launch(self, stream=None):
        _lib.check(_lib.load().rts_cadence_graph_launch(self._h, _stream(stream)), "rts_cadence_graph_launch")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().rts_cadence_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_tile(uvw, freq_hz, weights, vis, grid_in, n_grid, cell_lambda, support=7, oversample=8,
                  beta=None, conjugate=False, stream=None, measure=True):
    """Time each legal tile edge on these inputs; returns (best_tile, {tile: ms})."""
    torch = _torch()
    B, T = int(uvw.shape[0]), int(uvw.shape[1])
    freq = [float(f) for f in freq_hz]
    C = len(freq)
    _check_dev(uvw, "uvw", torch.float64, (B, T, 3))
    _check_dev(weights, "weights", torch.float32, (C, B, T))
    _check_dev(vis, "vis", torch.complex64, (C, B, T))
    _check_dev(grid_in, "grid_in", torch.complex64, (C, n_grid, n_grid))
    p = make_params(n_grid, cell_lambda, support, oversample, C, B, T, beta, conjugate, 0)
    fr = (ctypes.c_double * C)(*freq)
    best = ctypes.c_int32()
    ms = (ctypes.c_float * 8)()
    tiles = (ctypes.c_int32 * 8)()
    n = ctypes.c_int32()
    _lib.check(_lib.load().rts_autotune_tile(ctypes.byref(p), _ptr(uvw), ctypes.cast(fr, ctypes.c_void_p),
                                             _ptr(weights), _ptr(vis), _ptr(grid_in), _stream(stream),
                                             ctypes.byref(best), ms if measure else None, tiles, 8,
                                             ctypes.byref(n)), "rts_autotune_tile")
    return best.value, {tiles[k]: ms[k] for k in range(n.value)}


def polconvert(A, P, out=None, stream=None):
    """Polarisation conversion S_i = A_i P_i per pixel (rts_polconvert).

    A: complex64 [16, n_pix] (entry r*4+k of each pixel's 4x4 matrix, shared by
    all channels) or [C, 16, n_pix] (one set per channel).  P: complex64
    [C, 4, n_pix].  Returns S complex64 [C, 4, n_pix]; ``out`` may be P itself."""
    torch = _torch()
    if P.dim() != 3 or P.shape[1] != 4:
        raise ValueError(f"P must have shape [C, 4, n_pix], got {tuple(P.shape)}")
    C, n = int(P.shape[0]), int(P.shape[2])
    _check_dev(P, "P", torch.complex64)
    if A.dim() == 2:
        _check_dev(A, "A", torch.complex64, (16, n))
        stride = 0
    else:
        _check_dev(A, "A", torch.complex64, (C, 16, n))
        stride = 16 * n
    if out is None:
        out = torch.empty_like(P)
    _check_dev(out, "out", torch.complex64, (C, 4, n))
    _lib.check(_lib.load().rts_polconvert(_ptr(A), _ptr(P), _ptr(out), n, C, stride, _stream(stream)),
               "rts_polconvert")
    return out


def stream_copy(src, dst, stream=None):
    """Reference streaming copy src -> dst (device tensors of equal byte size,
    16-byte aligned): the attainable-bandwidth figure beside throughput results."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous and of equal byte size")
    _lib.check(_lib.load().rts_stream_copy(_ptr(src), _ptr(dst), n, _stream(stream)), "rts_stream_copy")
    return dst


def compute_coords(uvw, freq_hz, weights, n_grid, cell_lambda, support=7, oversample=8, stream=None):
    """Snapped oversampled coordinates int32 [C][B][T][3] = (xs, ys, valid) of the +uv copy."""
    torch = _torch()
    _check_dev(uvw, "uvw", torch.float64)
    B, T = int(uvw.shape[0]), int(uvw.shape[1])
    freq = [float(f) for f in freq_hz]
    C = len(freq)
    _check_dev(weights, "weights", torch.float32, (C, B, T))
    p = make_params(n_grid, cell_lambda, support, oversample, C, B, T)
    fr = (ctypes.c_double * C)(*freq)
    out = torch.empty((C, B, T, 3), dtype=torch.int32, device=uvw.device)
    _lib.check(_lib.load().rts_compute_coords(ctypes.byref(p), _ptr(uvw), ctypes.cast(fr, ctypes.c_void_p),
                                              _ptr(weights), _ptr(out), _stream(stream)), "rts_compute_coords")
    return out


def grid_degrid_noalloc(uvw, freq_hz, weights, vis, grid_in, n_grid, cell_lambda, support=7, oversample=8,
                        beta=None, tile=0, model_out=None, grid_out=None, chi2_out=None, stream=None):
    """Plan and fused residual step in one call of rts_grid_degrid_noalloc, whose
    workspace is the library's static device array (no device allocation inside
    the call).  Outputs are caller tensors (allocated here when not given).
    Returns (model_out or None, grid_out, chi2_out or None)."""
    torch = _torch()
    _check_dev(uvw, "uvw", torch.float64)
    B, T = int(uvw.shape[0]), int(uvw.shape[1])
    freq = [float(f) for f in freq_hz]
    C = len(freq)
    _check_dev(weights, "weights", torch.float32, (C, B, T))
    _check_dev(vis, "vis", torch.complex64, (C, B, T))
    _check_dev(grid_in, "grid_in", torch.complex64, (C, n_grid, n_grid))
    if grid_out is None:
        grid_out = torch.empty((C, n_grid, n_grid), dtype=torch.complex64, device=vis.device)
    _check_dev(grid_out, "grid_out", torch.complex64, (C, n_grid, n_grid))
    if model_out is not None:
        _check_dev(model_out, "model_out", torch.complex64, (C, B, T))
    if chi2_out is not None:
        _check_dev(chi2_out, "chi2_out", torch.float64)
    p = make_params(n_grid, cell_lambda, support, oversample, C, B, T, beta=beta, tile=tile)
    fr = (ctypes.c_double * C)(*freq)
    _lib.check(_lib.load().rts_grid_degrid_noalloc(ctypes.byref(p), _ptr(uvw), ctypes.cast(fr, ctypes.c_void_p),
                                                   _ptr(weights), _ptr(vis), _ptr(grid_in), _ptr(model_out),
                                                   _ptr(grid_out), _ptr(chi2_out), _stream(stream)),
               "rts_grid_degrid_noalloc")
    return model_out, grid_out, chi2_out


from .autograd import Chi2Fn, DegridFn, GridFn, chi2, degrid, grid  # noqa: E402,F401
