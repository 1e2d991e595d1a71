"""ctypes front-end of the C oracle (oracle_cpu.c).  TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import oracle as _o

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_cpu.c")
_LIB = os.path.join(_HERE, "liboracle_cpu.so")
_lib = None


def build() -> str:
    """Compile the C oracle in place (gcc, FP64, no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        lib.orc_grid.argtypes = [I, I, I, P, P, P, P, I, D, I, I, P, I, P]
        lib.orc_degrid.argtypes = [I, I, I, P, P, P, I, D, I, I, P, P, P]
        lib.orc_grid_degrid.argtypes = [I, I, I, P, P, P, P, I, D, I, I, P, P, P, P, P]
        lib.orc_num_threads.restype = I
        lib.orc_set_num_threads.argtypes = [I]
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _prep(uvw_m, freq_hz, vis, weights):
    uvw = np.ascontiguousarray(uvw_m, np.float64)
    f = np.ascontiguousarray(freq_hz, np.float64)
    v = np.ascontiguousarray(vis, np.complex64) if vis is not None else None
    w = np.ascontiguousarray(weights, np.float32)
    C = f.shape[0]
    B, T = uvw.shape[0], uvw.shape[1]
    assert w.shape == (C, B, T)
    return uvw, f, v, w, C, B, T


def num_threads() -> int:
    return load().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel channel loops (its OpenMP team size)."""
    load().orc_set_num_threads(int(n))


def grid(uvw_m, freq_hz, vis, weights, N, du, W=7, OS=8, beta=None, conjugate=False):
    lib = load()
    uvw, f, v, w, C, B, T = _prep(uvw_m, freq_hz, vis, weights)
    tab = np.ascontiguousarray(_o.table(W, OS, _o.default_beta(W) if beta is None else beta))
    G = np.empty((C, N, N), np.complex128)
    lib.orc_grid(C, B, T, _p(uvw), _p(f), _p(v), _p(w), N, du, W, OS, _p(tab), int(bool(conjugate)), _p(G))
    return G


def degrid(uvw_m, freq_hz, weights, G, N, du, W=7, OS=8, beta=None):
    lib = load()
    uvw, f, _, w, C, B, T = _prep(uvw_m, freq_hz, None, weights)
    tab = np.ascontiguousarray(_o.table(W, OS, _o.default_beta(W) if beta is None else beta))
    Gd = np.ascontiguousarray(G, np.complex128)
    M = np.empty((C, B, T), np.complex128)
    lib.orc_degrid(C, B, T, _p(uvw), _p(f), _p(w), N, du, W, OS, _p(tab), _p(Gd), _p(M))
    return M


def grid_degrid(uvw_m, freq_hz, vis, weights, G_in, N, du, W=7, OS=8, beta=None, want_model=True):
    """Returns (M or None, G_out, chi2 per channel)."""
    lib = load()
    uvw, f, v, w, C, B, T = _prep(uvw_m, freq_hz, vis, weights)
    tab = np.ascontiguousarray(_o.table(W, OS, _o.default_beta(W) if beta is None else beta))
    Gi = np.ascontiguousarray(G_in, np.complex128)
    M = np.empty((C, B, T), np.complex128) if want_model else None
    Go = np.empty((C, N, N), np.complex128)
    chi2 = np.empty(C, np.float64)
    lib.orc_grid_degrid(C, B, T, _p(uvw), _p(f), _p(v), _p(w), N, du, W, OS, _p(tab), _p(Gi), _p(M),
                        _p(Go), _p(chi2))
    return M, Go, chi2
