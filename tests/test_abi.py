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


@pytest.mark.parametrize("M,a,p,e,chi0,dt,ns", [
    (1.0, 0.9, 10.0, 0.4, 0.7, 0.02, 300),
    (1.0, 0.3, 8.0, 0.5, 0.0, 0.05, 300),
    (2.0, 1.0, 20.0, 0.3, 2.0, 0.1, 200),
    (1.0, 0.95, 14.0, 0.5, 3.0, 1.0, 300),
])
def test_host_eccentric_orbit_matches_oracle(M, a, p, e, chi0, dt, ns):
    """teuk_orbit_eccentric (closed-form constants, cosine series in chi,
    Newton inversion) vs the oracle's orbit (root-found constants, adaptive
    quadrature from sample to sample), over several radial periods."""
    lib = L.load()
    n = 2 * ns + 1
    out = np.zeros((n, 3))
    L.check(lib.teuk_orbit_eccentric(M, a, p, e, chi0, dt, n,
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    ref = T.eccentric_orbit(M, a, p, e, chi0, dt, ns)
    np.testing.assert_allclose(out[:, 0], ref["rs"], rtol=1e-13)
    np.testing.assert_array_equal(out[:, 1], ref["th"])
    np.testing.assert_allclose(out[:, 2], ref["phi"], rtol=0, atol=1e-13)


def test_host_eccentric_orbit_circular_limit_and_errors():
    lib = L.load()
    dt, n = 0.0177, 1001
    out = np.zeros((n, 3))
    ptr = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    L.check(lib.teuk_orbit_eccentric(1.0, 0.7, 10.0, 0.0, 0.0, dt, n, ptr))
    ref = T.circular_orbit(1.0, 0.7, 10.0, dt, (n - 1) // 2)
    np.testing.assert_allclose(out[:, 0], ref["rs"], rtol=1e-14)
    np.testing.assert_allclose(out[:, 2], ref["phi"], rtol=1e-13, atol=1e-300)
    for args in [(1.0, 0.9, 10.0, 0.95, 0.0, dt),     # e beyond the series' range
                 (1.0, 0.0, 6.5, 0.5, 0.0, dt),       # inside the separatrix p = 6 + 2e
                 (1.0, 1.0, 10.0, 0.2, 0.0, dt),      # |a| = M
                 (1.0, 0.5, 10.0, 0.2, 0.0, 0.0),     # dt = 0
                 (1.0, 0.5, 10.0, -0.1, 0.0, dt)]:
        assert lib.teuk_orbit_eccentric(*args, n, ptr) == L.TEUK_EINVAL, args
    assert lib.teuk_orbit_eccentric(1.0, 0.5, 10.0, 0.2, 0.0, dt, n, None) == L.TEUK_EINVAL
