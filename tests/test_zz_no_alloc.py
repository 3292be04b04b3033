"""teuk_init_grid_static: a context in the library's static device workspace
(no device allocation), checked through the C ABI against a context in a
caller's workspace (teuk_init_grid) on the same inputs: same kernels, so the
waveform and the state must be bitwise equal.  Two static contexts in a row,
the second on a smaller grid; a second one while the first lives is refused;
a grid beyond the static workspace is refused with a clear message."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1001_3631_amd import workloads as W


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1001_3631_amd import _lib
    return _lib.load()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def run(lib, ctx, grid, nsteps, pulse=None, source=None):
    """Drive a context through the C ABI: initial data, source, nsteps
    iterations; returns (waveform, Phi, Pi) on the host."""
    from paper_1001_3631_amd import _lib as L
    nth, nr = grid["nth"], grid["nr"]
    keep = []
    if pulse is not None:
        L.check(lib.teuk_init_pulse(ctx, pulse["center"], pulse["width"], pulse["amplitude"]))
    if source is not None:
        info = L.Info()
        L.check(lib.teuk_get_info(ctx, ctypes.byref(info)))
        ns = 2 * nsteps + 1
        orbit = np.zeros((ns, 3))
        L.check(lib.teuk_orbit_circular(grid["M"], grid["a"], source["r0"], info.dt, ns,
                                        orbit.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        dev = torch.empty(3 * ns, dtype=torch.float64, device="cuda")
        keep += [orbit, dev]
        desc = L.SourceDesc(source["amplitude"], source["sigma_r_cells"], source["sigma_th_cells"],
                            source["cutoff_sigmas"], ns, orbit.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            _ptr(dev))
        L.check(lib.teuk_set_source(ctx, ctypes.byref(desc)))
    w = torch.empty((nsteps, nth), dtype=torch.complex128, device="cuda")
    L.check(lib.teuk_step_n(ctx, nsteps, _ptr(w)))
    p = torch.empty((nth, nr), dtype=torch.complex128, device="cuda")
    q = torch.empty_like(p)
    L.check(lib.teuk_get_state(ctx, _ptr(p), _ptr(q)))
    torch.cuda.synchronize()
    return w.cpu().numpy(), p.cpu().numpy(), q.cpu().numpy()


def reference(lib, grid, nsteps, req, pulse=None, source=None):
    from paper_1001_3631_amd import _lib as L
    from paper_1001_3631_amd.engine import device_buffer, grid_desc
    desc = grid_desc(grid)
    n = ctypes.c_size_t()
    L.check(lib.teuk_workspace_size(ctypes.byref(desc), ctypes.byref(req), ctypes.byref(n)))
    ws = device_buffer(n.value)
    ctx = ctypes.c_void_p()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L.check(lib.teuk_init_grid(ctypes.byref(desc), ctypes.byref(req), stream, _ptr(ws), n.value, ctypes.byref(ctx)))
    try:
        return run(lib, ctx, grid, nsteps, pulse, source)
    finally:
        L.check(lib.teuk_destroy(ctx))


def static_ctx(lib, grid, req):
    from paper_1001_3631_amd import _lib as L
    from paper_1001_3631_amd.engine import grid_desc
    ctx = ctypes.c_void_p()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.teuk_init_grid_static(ctypes.byref(grid_desc(grid)), ctypes.byref(req), stream, ctypes.byref(ctx))
    return rc, ctx


def test_static_workspace_matches_caller_workspace_twice(lib):
    from paper_1001_3631_amd import _lib as L
    from paper_1001_3631_amd.engine import ws_request
    cases = [
        (W.KERR_EMRI["grid"], 300, None, W.KERR_EMRI["source"], ws_request((2.0, 2.0, 8.0), False)),
        (W.SCHWARZSCHILD_PULSE["grid"], 500, W.SCHWARZSCHILD_PULSE["pulse"], None, ws_request(None, True)),
    ]
    for grid, n, pulse, source, req in cases:
        print("case", grid["nr"], "x", grid["nth"], n, "iterations", flush=True)
        ref = reference(lib, grid, n, req, pulse, source)
        rc, ctx = static_ctx(lib, grid, req)
        assert rc == L.TEUK_OK, lib.teuk_last_error()
        # the static workspace is held: a second static context is refused
        rc2, ctx2 = static_ctx(lib, grid, req)
        assert rc2 == L.TEUK_ESTATE and ctx2.value is None
        got = run(lib, ctx, grid, n, pulse, source)
        L.check(lib.teuk_destroy(ctx))
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
        assert np.max(np.abs(got[1])) > 0


def test_static_workspace_refuses_a_grid_beyond_its_size(lib):
    from paper_1001_3631_amd import _lib as L
    from paper_1001_3631_amd.engine import ws_request
    rc, ctx = static_ctx(lib, W.HBM_PLAIN["grid"], ws_request((2.0, 2.0, 8.0), True))
    assert rc == L.TEUK_ENOMEM and ctx.value is None
    assert b"static workspace holds" in lib.teuk_last_error()
    # and the workspace is still free for a grid that fits
    rc, ctx = static_ctx(lib, W.SCHWARZSCHILD_PULSE["grid"], ws_request(None, False))
    assert rc == L.TEUK_OK
    L.check(lib.teuk_destroy(ctx))
