"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol the header declares, and rejects bad arguments before device work."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1907_02731_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfseg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfseg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sfseg_create", "sfseg_power_iterate", "sfseg_eigvec", "sfseg_destroy",
                     "sfseg_apply", "sfseg_status_string", "sfseg_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(_lib.LIB_PATH), "build libsfseg.so first"
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], check=True,
                         capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (sfseg_[a-z_]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    L = _lib.lib()
    for n in declared_functions():
        assert getattr(L, n) is not None


def test_struct_layout_matches_header():
    # sfseg_config: 6 int32 then 4 doubles = 56 bytes; result 24; timing 32
    assert ctypes.sizeof(_lib.Config) == 56
    assert ctypes.sizeof(_lib.Result) == 24
    assert ctypes.sizeof(_lib.Timing) == 32
    assert ctypes.sizeof(_lib.Binarize) == 16


def test_config_default_and_validate():
    c = _lib.Config()
    _lib.lib().sfseg_config_default(ctypes.byref(c))
    assert (c.r_t, c.r_s, c.storage) == (1, 2, 0)
    assert (c.sigma_t, c.sigma_s, c.alpha, c.p) == (1.0, 1.0, 1.0, 0.2)
    assert _lib.validate(c) == _lib.SFSEG_ERR_INVALID_ARG  # T = H = W = 0
    c.T, c.H, c.W = 8, 64, 96
    assert _lib.validate(c) == _lib.SFSEG_OK


@pytest.mark.parametrize("field,value,code", [
    ("T", 0, _lib.SFSEG_ERR_INVALID_ARG),
    ("W", -3, _lib.SFSEG_ERR_INVALID_ARG),
    ("r_t", -1, _lib.SFSEG_ERR_INVALID_ARG),
    ("r_s", _lib.MAX_RS + 1, _lib.SFSEG_ERR_UNSUPPORTED),
    ("r_t", _lib.MAX_RT + 1, _lib.SFSEG_ERR_UNSUPPORTED),
    ("sigma_t", 0.0, _lib.SFSEG_ERR_INVALID_ARG),
    ("sigma_s", float("nan"), _lib.SFSEG_ERR_INVALID_ARG),
    ("alpha", -0.5, _lib.SFSEG_ERR_INVALID_ARG),
    ("p", float("inf"), _lib.SFSEG_ERR_INVALID_ARG),
    ("storage", 3, _lib.SFSEG_ERR_INVALID_ARG),
])
def test_bad_config_rejected_before_device_work(field, value, code):
    c = _lib.make_config(4, 8, 8)
    setattr(c, field, value)
    assert _lib.validate(c) == code
    out = ctypes.c_void_p(1234)
    rc = _lib.lib().sfseg_create(ctypes.byref(c), ctypes.c_void_p(1), None, None, ctypes.byref(out))
    assert rc == code
    assert out.value is None
    assert _lib.lib().sfseg_last_error().decode()


def test_oversized_volume_rejected():
    c = _lib.make_config(2048, 1024, 1024)
    assert _lib.validate(c) == _lib.SFSEG_ERR_INVALID_ARG


def test_null_arguments_rejected():
    L = _lib.lib()
    c = _lib.make_config(4, 8, 8)
    out = ctypes.c_void_p()
    assert L.sfseg_create(ctypes.byref(c), None, None, None, ctypes.byref(out)) == \
        _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_create(ctypes.byref(c), ctypes.c_void_p(1), None, None, None) == \
        _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_create(None, ctypes.c_void_p(1), None, None, ctypes.byref(out)) == \
        _lib.SFSEG_ERR_INVALID_ARG
    res = _lib.Result()
    assert L.sfseg_power_iterate(None, None, 5, 1e-5, ctypes.byref(res)) == \
        _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_eigvec(None, ctypes.c_void_p(1)) == _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_apply(None, ctypes.c_void_p(1), ctypes.c_void_p(2)) == \
        _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_set_features(None, ctypes.c_void_p(1), None) == _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_apply_noalloc(None, ctypes.c_void_p(1), ctypes.c_void_p(2)) == \
        _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_apply_noalloc_bytes(None) == 0
    assert L.sfseg_spectral_grad(None, None, None, 1, None, None) == _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_refine_frames(None, None, None) == _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_last_timing(None, None) == _lib.SFSEG_ERR_INVALID_ARG
    b = _lib.Binarize()
    L.sfseg_binarize_default(ctypes.byref(b))
    assert (b.iters, b.project_from, b.slope, b.threshold) == (5, 3, 10.0, 0.5)
    assert L.sfseg_project(None, 10.0, 0.5) == _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_threshold(None, 0.5, ctypes.c_void_p(1)) == _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_segment(None, None, ctypes.byref(b), None, None) == \
        _lib.SFSEG_ERR_INVALID_ARG
    L.sfseg_binarize_default(None)  # NULL-safe
    L.sfseg_destroy(None)  # NULL-safe


def test_status_strings():
    L = _lib.lib()
    for code in range(-7, 1):
        s = L.sfseg_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.sfseg_status_string(-99).decode() == "unknown status"


def test_solver_rejects_cpu_tensors():
    torch = pytest.importorskip("torch")
    from paper_1907_02731_amd.solver import Solver
    with pytest.raises(TypeError):
        Solver(torch.zeros(2, 3, 4))
