"""CPU checks of the C ABI: the library loads, exports every entry point that
include/rtsgrid.h declares, and rejects bad arguments on the host (before any HIP
call) with RTS_E_INVALID and a message."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1003_5575_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("librtsgrid.so is not built (run python -m paper_1003_5575_amd.build)")
    return _lib.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rtsgrid.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rts_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    from paper_1003_5575_amd import _lib
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTED)


def test_version_and_empty_error(lib):
    assert lib.rts_version().decode().startswith("rtsgrid")
    assert isinstance(lib.rts_last_error(), bytes)


def good_params():
    import paper_1003_5575_amd as rts
    return rts.make_params(256, 10.0, 7, 8, 2, 100, 8)


def plan_call(lib, p, uvw=1, freq=(150e6, 151e6), w=1):
    h = ctypes.c_void_p()
    f = (ctypes.c_double * len(freq))(*freq)
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: validation fails first
    return lib.rts_grid_plan(ctypes.byref(h), ctypes.byref(p) if p is not None else None,
                             fake if uvw else None, ctypes.cast(f, ctypes.c_void_p), fake if w else None, None), h


@pytest.mark.parametrize("field,value,msg", [
    ("n_grid", 8, "n_grid"), ("n_grid", 255, "n_grid"), ("n_grid", 16384, "n_grid"),
    ("support", 1, "support"), ("support", 17, "support"),
    ("oversample", 0, "oversample"), ("oversample", 65, "oversample"),
    ("n_chan", 0, "n_chan"), ("n_base", 0, "n_chan"), ("n_time", 0, "n_chan"),
    ("cell_lambda", 0.0, "cell_lambda"), ("cell_lambda", float("nan"), "cell_lambda"),
    ("beta", float("inf"), "beta"),
    ("conjugate", 2, "conjugate"), ("precision", 7, "precision"), ("precision", 3, "precision"), ("schedule", 3, "schedule"), ("schedule", -1, "schedule"),
    ("tile", 48, "tile"), ("tile", 4, "tile"), ("tile", 128, "tile"), ("tile", 7, "tile"),
])
def test_invalid_params_rejected_on_host(lib, field, value, msg):
    p = good_params()
    setattr(p, field, value)
    st, h = plan_call(lib, p)
    assert st == 1 and not h.value
    assert msg in lib.rts_last_error().decode()


def test_size_overflow_rejected(lib):
    import paper_1003_5575_amd as rts
    p = rts.make_params(256, 10.0, 7, 8, 4096, 130816, 8)
    st, _ = plan_call(lib, p, freq=[150e6] * 4096)
    assert st == 1 and "2^31" in lib.rts_last_error().decode()
    # one channel of 2^29 samples: within 2^31 overall, beyond the kernels'
    # 32-bit per-channel byte offsets
    p = rts.make_params(256, 10.0, 7, 8, 1, 1 << 22, 128)
    st, _ = plan_call(lib, p, freq=[150e6])
    assert st == 1 and "n_base*n_time" in lib.rts_last_error().decode()


def test_null_arguments_rejected(lib):
    st, _ = plan_call(lib, None)
    assert st == 1
    st, _ = plan_call(lib, good_params(), uvw=0)
    assert st == 1 and "non-NULL" in lib.rts_last_error().decode()
    st, _ = plan_call(lib, good_params(), freq=(150e6, -1.0))
    assert st == 1 and "freq_hz" in lib.rts_last_error().decode()
    assert lib.rts_grid_plan(None, ctypes.byref(good_params()), None, None, None, None) == 1


def test_calls_on_null_plan(lib):
    assert lib.rts_plan_destroy(None) == 0
    assert lib.rts_grid(None, None, None, None, None) == 1
    assert lib.rts_degrid(None, None, None, None) == 1
    assert lib.rts_grid_degrid(None, None, None, None, None, None, None, None) == 1
    assert lib.rts_plan_update(None, None, None, None) == 1
    assert lib.rts_plan_get_info(None, None) == 1
    assert lib.rts_plan_get_table(None, None, 0) == 1
    assert lib.rts_image(None, None, None, None) == 1
    assert "plan is NULL" in lib.rts_last_error().decode()


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    import paper_1003_5575_amd as rts
    with pytest.raises(TypeError):
        rts.GridPlan(torch.zeros(4, 2, 3, dtype=torch.float64), [150e6], torch.zeros(1, 4, 2), 64, 10.0)


def test_polconvert_argument_checks_on_host(lib):
    """Host-side validation of rts_polconvert: no HIP call is reached."""
    assert lib.rts_polconvert(None, None, None, -1, 1, 0, None) == 1
    assert "n_pix and n_chan" in lib.rts_last_error().decode()
    assert lib.rts_polconvert(None, None, None, 10, -2, 0, None) == 1
    assert lib.rts_polconvert(None, None, None, 10, 1, 100, None) == 1     # stride below 16 * n_pix
    assert "a_chan_stride" in lib.rts_last_error().decode()
    assert lib.rts_polconvert(None, None, None, 1 << 40, 1, 0, None) == 1
    assert "too large" in lib.rts_last_error().decode()
    assert lib.rts_polconvert(None, None, None, 0, 4, 0, None) == 0         # empty: no-op
    assert lib.rts_polconvert(None, None, None, 10, 0, 0, None) == 0
    assert lib.rts_polconvert(None, None, None, 10, 2, 0, None) == 1
    assert "non-NULL" in lib.rts_last_error().decode()
    assert lib.rts_polconvert(ctypes.c_void_p(4), ctypes.c_void_p(8), ctypes.c_void_p(16), 10, 2, 0, None) == 1
    assert "aligned" in lib.rts_last_error().decode()


def test_bf16x3_support_limits_on_host(lib):
    """Supports up to 24 are accepted for BF16x3 plans only.  (The matrix-core
    kernels' LDS budget check, 64 KiB, is not reached by any valid geometry: the
    widest, support 24 at oversampling 64, needs 63,680 bytes with regions of two
    subtiles; the GPU tests run the widest tables at support 16.)"""
    import paper_1003_5575_amd as rts
    p = rts.make_params(192, 10.0, 25, 8, 2, 100, 8, precision=1)
    st, _ = plan_call(lib, p)
    assert st == 1 and "support must be in [2, 24]" in lib.rts_last_error().decode()
    assert lib.rts_plan_set_baseline_kernels(None, None, None) == 1
