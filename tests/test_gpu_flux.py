"""Radiated energy and momentum on the GPU (teuk_radiated_flux) against the
oracle's radiated_flux, on seeded synthetic waveforms of the all-m shape
(m = 1..4, 128 theta rows, 4000 iterations) and on ragged and degenerate
shapes; argument checks.  Bar: every one of the ten outputs within 1e-12 of
the largest value of its column (the time integrals are summed in the same
order on both sides; the theta sums differ in order)."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import teuk_oracle as T
from paper_1001_3631_amd import workloads as W


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1001_3631_amd import _lib
    _lib.load()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("ms,nsteps,nth", [
    ([1, 2, 3, 4], 4000, 128),          # the all-m batch's shape
    ([2], 300, 33),
    ([3, 2, 5, 4], 257, 7),             # unsorted m, pairs (2,3) and (4,5), fewest rows
    ([2, 3], 0, 65),                    # only the initial sample
    (list(range(-4, 12)), 50, 129),     # 16 modes, more rows than a wave's lanes
])
def test_flux_matches_oracle(ms, nsteps, nth):
    from paper_1001_3631_amd.engine import radiated_flux
    dt = 0.0177598
    waves = W.synthetic_waveforms(ms, nsteps, nth, dt, seed=len(ms) + nth)
    got = radiated_flux(ms, [_dev(w) for w in waves], dt).cpu().numpy()
    ref = T.radiated_flux(ms, waves, dt, np.pi / (nth - 1))
    scale = np.maximum(np.max(np.abs(ref), axis=0), 1e-300)
    err = np.max(np.abs(got - ref), axis=0) / scale
    print(ms, nsteps, nth, "worst per column", np.array2string(err, precision=2))
    assert np.all(err <= 1e-12), err
    if not any(m + 1 in ms for m in ms):
        assert np.all(got[:, 1:3] == 0.0)


def test_flux_argument_checks():
    from paper_1001_3631_amd import _lib as L
    lib = L.load()
    w = torch.zeros((11, 9), dtype=torch.complex128, device="cuda")
    out = torch.empty((11, 10), dtype=torch.float64, device="cuda")

    def desc(ms, nsteps=10, nth=9, dt=0.1):
        m_arr = (ctypes.c_int32 * len(ms))(*ms)
        p_arr = (ctypes.c_void_p * len(ms))(*[w.data_ptr()] * len(ms))
        return L.FluxDesc(len(ms), m_arr, p_arr, nsteps, nth, dt), m_arr, p_arr

    n = ctypes.c_size_t()
    for bad in (dict(ms=[2, 2]), dict(ms=list(range(17))), dict(ms=[1], dt=0.0), dict(ms=[1], nth=2)):
        d = desc(**bad)
        assert lib.teuk_flux_workspace_size(ctypes.byref(d[0]), ctypes.byref(n)) == L.TEUK_EINVAL
    d = desc([1, 2])
    assert lib.teuk_flux_workspace_size(ctypes.byref(d[0]), ctypes.byref(n)) == L.TEUK_OK
    assert n.value >= 2 * 2 * 11 * 9 * 16
    ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
    rc = lib.teuk_radiated_flux(ctypes.byref(d[0]), None, ctypes.c_void_p(ws.data_ptr()), n.value - 1,
                                ctypes.c_void_p(out.data_ptr()))
    assert rc == L.TEUK_ENOMEM
