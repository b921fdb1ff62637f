"""The C-ABI library loads and exports every symbol include/ksc.h declares
(CPU only: no call that touches a device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ksc.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ksc_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_binding_set():
    from paper_2301_11704_amd import _lib
    assert _declared() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_2301_11704_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libksc.so not built")
    L = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_pure_host_calls():
    from paper_2301_11704_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libksc.so not built")
    L = _lib.lib()
    for nx, km in ((8, 3), (16, 6), (32, 11), (64, 22), (128, 43), (256, 86)):
        assert L.ksc_n_modes(nx) == km
    for bad in (0, 7, 48, 512):
        assert L.ksc_n_modes(bad) == -1
    # null-pointer validation happens before any HIP call
    assert L.ksc_create(None, 1, 0, None, None) == -1
    assert b"null" in L.ksc_last_error()
    assert L.ksc_destroy(None) == -1
    assert L.ksc_state_numel(None) == -1
    assert L.ksc_eval_J(None, None, None, None) == -1
    assert L.ksc_set_timing(None, 1) == -1
    f, q, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    assert L.ksc_read_timing(None, ctypes.byref(f), ctypes.byref(q), ctypes.byref(n)) == -1
    sc = ctypes.c_int32()
    assert L.ksc_set_scheme(None, 1) == -1
    assert L.ksc_get_scheme(None, ctypes.byref(sc)) == -1


def test_create_validates_before_touching_the_device():
    """Shape and argument errors of ksc_create are reported before any HIP
    call (so they are testable without a GPU): empty batch, n_s < 3, an
    unsupported grid, L <= 0, an unknown map, a non-positive scale."""
    from paper_2301_11704_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libksc.so not built")
    L = _lib.lib()
    out = ctypes.c_void_p()

    def create(n_s=64, n_x=32, length=22.0, map_=0, scale=40.0, n=1):
        arr = (_lib.CurveDescC * max(n, 1))(*[_lib.CurveDescC(n_s, n_x, length, map_, scale, 0.0)
                                              for _ in range(max(n, 1))])
        return L.ksc_create(arr, n, 0, None, ctypes.byref(out))

    assert create(n=0) == -2
    assert create(n_s=2) == -2
    assert create(n_s=(1 << 26) + 1) == -2
    assert create(n_x=48) == -3
    assert create(n_x=512) == -3
    assert create(length=0.0) == -1
    assert create(length=float("nan")) == -1
    assert create(map_=7) == -1
    assert create(scale=0.0) == -1
    assert b"scale" in L.ksc_last_error()
    assert create(n_x=48) == -3 and b"n_x=48" in L.ksc_last_error()
    assert out.value is None


def test_create2_validates_the_state_space():
    """ksc_create2: an unknown state space is an argument error; the
    inversion-symmetric subspace in FP64 stops at n_x = 128 (one lane per row);
    both are reported before any HIP call."""
    from paper_2301_11704_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libksc.so not built")
    L = _lib.lib()
    out = ctypes.c_void_p()

    def create2(space, dtype, n_x=32):
        arr = (_lib.CurveDescC * 1)(_lib.CurveDescC(64, n_x, 22.0, 0, 40.0, 0.0))
        return L.ksc_create2(arr, 1, dtype, space, None, ctypes.byref(out))

    assert create2(2, 0) == -1 and b"space" in L.ksc_last_error()
    assert create2(-1, 1) == -1
    assert create2(_lib.KSC_SPACE_ODD, _lib.KSC_F64, 256) == -3
    assert b"n_x <= 128" in L.ksc_last_error()
    assert create2(_lib.KSC_SPACE_ODD, _lib.KSC_F64, 48) == -3
    assert out.value is None


def test_create_opts_validates_the_spectral_ds():
    """ksc_create_opts: the spectral d/ds needs the rational map, one row per
    lane (n_x <= 128 in FP32, <= 64 in FP64, in either space) and
    n_s <= 16384; unknown options and a non-zero reserved field are argument
    errors; all reported before any HIP call."""
    from paper_2301_11704_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libksc.so not built")
    L = _lib.lib()
    out = ctypes.c_void_p()

    def create(dtype=0, space=0, ds=1, reserved=0, n_x=32, n_s=64, map_=0):
        arr = (_lib.CurveDescC * 1)(_lib.CurveDescC(n_s, n_x, 22.0, map_, 40.0, 0.0))
        o = _lib.OptionsC(dtype, space, ds, reserved)
        return L.ksc_create_opts(arr, 1, ctypes.byref(o), None, ctypes.byref(out))

    assert L.ksc_create_opts(None, 1, None, None, ctypes.byref(out)) == -1
    assert create(ds=2) == -1
    assert create(reserved=1) == -1
    assert create(map_=1) == -1 and b"rational" in L.ksc_last_error()
    assert create(space=1, n_x=256) == -3
    assert create(n_x=256) == -3
    assert create(dtype=1, n_x=128) == -3 and b"64 in FP64" in L.ksc_last_error()
    assert create(n_s=16385) == -3
    assert out.value is None
