"""The C ABI library loads and exports every function include/h6.h declares,
and argument validation answers before any device work (CPU only)."""

import ctypes as C
import os
import re

import pytest

from paper_1901_08532_amd import h6

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "h6.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(h6_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert _declared() == sorted(h6.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = C.CDLL(h6.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_error_texts():
    L = h6.lib()
    for code in (h6.H6_OK, h6.H6_EINVAL, h6.H6_ENOMEM, h6.H6_EHIP, h6.H6_ESTATE, h6.H6_EDTMIN,
                 h6.H6_ENONFINITE):
        assert L.h6_strerror(code)
    assert L.h6_strerror(12345) == b"unknown error"
    assert L.h6_last_error(None) == b""


def test_null_context_and_bad_create_arguments():
    L = h6.lib()
    assert L.h6_create(None, 10, 0.1, None) == h6.H6_EINVAL
    out = C.c_void_p()
    assert L.h6_create(C.byref(out), 0, 0.1, None) == h6.H6_EINVAL
    assert L.h6_create(C.byref(out), 10, -1.0, None) == h6.H6_EINVAL
    assert L.h6_create(C.byref(out), 10, float("nan"), None) == h6.H6_EINVAL
    assert L.h6_create(C.byref(out), (1 << 30) + 1, 0.1, None) == h6.H6_EINVAL
    assert out.value is None
    assert L.h6_destroy(None) == h6.H6_OK
    st = h6.h6_state()
    assert L.h6_evaluate(None, None, None, 1, None, 1, 0, None) == h6.H6_EINVAL
    assert L.h6_energy(None, C.byref(st), 1, None) == h6.H6_EINVAL
    assert L.h6_check_status(None) == h6.H6_EINVAL
    assert L.h6_set_eval_config(None, 64, 1, 1, -1) == h6.H6_EINVAL


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(h6, "_lib", None)
    monkeypatch.setattr(h6, "LIB_PATH", "/nonexistent/libh6.so")
    with pytest.raises(h6.H6Error):
        h6.lib()


def _self_term(m, eps, dtype):
    # the self pair's acceleration term as the kernels form it: R^2 = eps^2,
    # 1/R, 1/R^2, m/R^3, times the exact zero separation
    import numpy as np

    with np.errstate(over="ignore", invalid="ignore"):
        e2 = dtype(eps) * dtype(eps)
        rinv = dtype(1.0) / np.sqrt(e2)
        mr3 = (dtype(m) * rinv) * (rinv * rinv)
        return mr3 * dtype(0.0)


def test_self_pair_mask_limits():
    import numpy as np

    L = h6.lib()
    lim = {h6.H6_FP64: 2.0 ** -300, h6.H6_MIXED: 2.0 ** -30, h6.H6_EX: 2.0 ** -30,
           h6.H6_SP: 2.0 ** -30}
    for prec, e in lim.items():
        assert L.h6_self_pair_masked(0.0, prec) == 1
        assert L.h6_self_pair_masked(e * 0.5, prec) == 1
        assert L.h6_self_pair_masked(e, prec) == 0
        assert L.h6_self_pair_masked(1e-4, prec) == 0
    # a softening of 1e-15 with a mass of 1e-3 overflows m eps^-3 in FP32:
    # the FP32-range arithmetics mask it, FP64 need not
    assert L.h6_self_pair_masked(1e-15, h6.H6_MIXED) == 1
    assert L.h6_self_pair_masked(1e-15, h6.H6_FP64) == 0
    assert L.h6_self_pair_masked(1e-104, h6.H6_FP64) == 1
    assert L.h6_self_pair_masked(-1.0, h6.H6_FP64) == h6.H6_EINVAL
    assert L.h6_self_pair_masked(float("inf"), h6.H6_FP64) == h6.H6_EINVAL
    assert L.h6_self_pair_masked(1e-4, 99) == h6.H6_EINVAL
    # at the limit the unmasked self term is an exact zero for every mass up
    # to the stated bound (2^38 FP32, 2^124 FP64), and NaN just past it
    for dtype, eps, mmax in ((np.float32, 2.0 ** -30, 2.0 ** 38),
                             (np.float64, 2.0 ** -300, 2.0 ** 124)):
        assert _self_term(mmax * 0.99, eps, dtype) == 0.0
        assert np.isnan(_self_term(mmax * 4.0, eps, dtype))
    assert np.isnan(_self_term(1e-3, 1e-15, np.float32))  # the failure masking avoids
