"""The C ABI library loads and exports every entry point include/teuk.h
declares; host-only entry points (descriptor validation, orbit builder) work
without a device.  No kernel is launched here."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1001_3631_amd import _lib as L
from oracle import teuk_oracle as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "teuk.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(teuk_[a-z0-9_]+)\s*\(", src)))


def test_header_matches_binding():
    assert declared_functions() == sorted(L.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def _desc(**kw):
    base = dict(M=1.0, a=0.5, s=-2, m=2, nr=101, nth=17, rs_min=-50.0, rs_max=100.0, cfl=0.5,
                rs_extract=50.0, ko_eps=0.5)
    base.update(kw)
    return L.GridDesc(*[base[k] for k, _ in L.GridDesc._fields_])


@pytest.mark.parametrize("bad", [dict(a=1.0), dict(a=-1.2), dict(nr=4), dict(nth=6), dict(cfl=0.0),
                                 dict(cfl=1.5), dict(rs_max=-60.0), dict(s=3), dict(ko_eps=-0.1),
                                 dict(ko_eps=2.0), dict(rs_extract=1e4), dict(M=0.0)])
def test_invalid_descriptor_is_rejected_before_any_device_call(bad):
    lib = L.load()
    ctx = ctypes.c_void_p()
    rc = lib.teuk_init_grid(ctypes.byref(_desc(**bad)), None, ctypes.byref(ctx))
    assert rc == L.TEUK_EINVAL
    assert ctx.value is None
    assert len(lib.teuk_last_error()) > 0


def test_null_arguments_are_rejected():
    lib = L.load()
    assert lib.teuk_init_grid(None, None, None) == L.TEUK_EINVAL
    assert lib.teuk_step_n(None, 1, None) == L.TEUK_EINVAL
    assert lib.teuk_get_info(None, None) == L.TEUK_EINVAL
    assert lib.teuk_destroy(None) == L.TEUK_OK


@pytest.mark.parametrize("a", [0.0, 0.7, 0.9])
def test_host_orbit_builder_matches_oracle(a):
    """teuk_orbit_circular (library, host code) vs the oracle's orbit."""
    lib = L.load()
    dt, n = 0.0177, 1001
    out = np.zeros((n, 3))
    L.check(lib.teuk_orbit_circular(1.0, a, 10.0, dt, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    ref = T.circular_orbit(1.0, a, 10.0, dt, (n - 1) // 2)
    np.testing.assert_allclose(out[:, 0], ref["rs"], rtol=1e-14)
    np.testing.assert_allclose(out[:, 1], ref["th"], rtol=0, atol=0)
    np.testing.assert_allclose(out[:, 2], ref["phi"], rtol=1e-14, atol=1e-300)
    assert lib.teuk_orbit_circular(1.0, a, 1.0, dt, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == L.TEUK_EINVAL
