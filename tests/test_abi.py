"""The C ABI library loads on the CPU host, exports every function the header
declares, and rejects bad configurations before touching a device."""
import os
import re

import numpy as np
import pytest

from paper_1805_08995_amd import binding, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "cashash.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cashash_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    L = binding.lib()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(binding.EXPORTED)


def test_default_config():
    c = binding.default_config()
    assert (c.k, c.ratio_num, c.ratio_den, c.max_hamming, c.mode, c.mem) == (10, 4, 5, 128, 0, 1)
    assert c.margin_coef == 1e-3


def _create(rc, rb, **kw):
    import ctypes as C
    cfg = binding.default_config()
    for k, v in kw.items():
        setattr(cfg, k, v)
    h = C.c_void_p()
    rc = np.ascontiguousarray(rc, np.float64)
    rb = np.ascontiguousarray(rb, np.float64)
    rcode = binding.lib().cashash_create(C.byref(h), rc.ctypes.data, rb.ctypes.data, C.byref(cfg))
    return rcode, binding.lib().cashash_last_error().decode()


@pytest.mark.parametrize("field,value,code", [("k", 0, binding.E_LIMIT), ("k", 65, binding.E_LIMIT),
                                              ("max_hamming", 129, binding.E_LIMIT),
                                              ("ratio_den", 0, binding.E_INVAL), ("mode", 7, binding.E_INVAL),
                                              ("mem", 3, binding.E_INVAL), ("margin_coef", 0.0, binding.E_INVAL)])
def test_config_rejected(field, value, code):
    rc, rb = synth.projection_matrices()
    rcode, msg = _create(rc, rb, **{field: value})
    assert rcode == code and msg


def test_unsafe_matrix_rejected():
    rc, rb = synth.projection_matrices()
    rcode, msg = _create(rc * 100.0, rb)  # row norms ~1100: 5e-5 * |r| > 1e-3
    assert rcode == binding.E_UNSAFE_MATRIX and "norm" in msg
    bad = rc.copy()
    bad[3, 4] = np.nan
    assert _create(bad, rb)[0] == binding.E_UNSAFE_MATRIX
    # a larger margin makes the same long rows acceptable to the proof
    rcode, _ = _create(rc * 100.0, rb * 100.0, margin_coef=1.0)
    assert rcode != binding.E_UNSAFE_MATRIX
