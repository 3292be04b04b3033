"""GPU adjoint (teuk_adjoint_*) against the oracle's hand-transposed sweep,
the dot-product identity, central differences of the GPU forward, and the
torch.autograd wrapper."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import teuk_oracle as T
from paper_1001_3631_amd import workloads as W
from test_gpu_parity import (SRC, STEP_GRIDS, gpu_engine, gpu_source, host, oracle_source, rel,
                             to_dev)


def vdot2(a, b):
    return np.vdot(a[0], b[0]) + np.vdot(a[1], b[1])


@pytest.mark.parametrize("grid", STEP_GRIDS)
@pytest.mark.parametrize("with_source", [False, True])
def test_single_reverse_iteration_matches_oracle(grid, with_source):
    g = T.Grid(**grid)
    lp, lq = W.random_state(g.nth, g.nr, seed=21)
    eng = gpu_engine(grid)
    src = None
    if with_source:
        gpu_source(eng, grid, SRC, 4)
        src = oracle_source(g, SRC, 4)
    eng.adjoint_begin(3, to_dev(lp), to_dev(lq))
    eng.adjoint_step(1)
    p, q, dA = eng.adjoint_get(want_dA=with_source)
    rp, rq, rdA = T.adjoint_step(g, lp, lq, 2, src)
    assert rel(host(p), rp) <= 1e-13
    assert rel(host(q), rq) <= 1e-13
    if with_source:
        assert abs(dA - rdA) <= 1e-12 * max(abs(rdA), 1e-300), (dA, rdA)


@pytest.mark.parametrize("grid", STEP_GRIDS[:3])
def test_gpu_dot_product_identity(grid):
    x = W.random_state(grid["nth"], grid["nr"], seed=31)
    y = W.random_state(grid["nth"], grid["nr"], seed=32)
    eng = gpu_engine(grid)
    eng.set_state(to_dev(x[0]), to_dev(x[1]))
    eng.step(1, waveform=False)
    Gx = [host(t) for t in eng.get_state()]
    eng.adjoint_begin(1, to_dev(y[0]), to_dev(y[1]))
    eng.adjoint_step(1)
    p, q, _ = eng.adjoint_get(want_dA=False)
    GHy = (host(p), host(q))
    lhs, rhs = vdot2(Gx, y), vdot2(x, GHy)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def _adjoint_case(n=120):
    grid = dict(M=1.0, a=0.7, s=-2, m=2, nr=181, nth=37, rs_min=-30.0, rs_max=60.0, cfl=0.5,
                rs_extract=40.0, ko_eps=0.5)
    return grid, n


def test_reverse_sweep_matches_oracle_gradient():
    """Loss sum |w - y|^2 with y a seeded noise field; the GPU gradient
    (initial data and amplitude) against the oracle's reverse sweep."""
    grid, n = _adjoint_case()
    g = T.Grid(**grid)
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    y = W.target_noise((n, g.nth), 0.05, seed=4)
    # oracle
    src = oracle_source(g, SRC, n)
    w = T.evolve(g, phi0, pi0, n, src)[2]
    _, gw = T.waveform_loss(w, y)
    rgp, rgq, rdA = T.adjoint_evolve(g, gw, n, src)
    # GPU (its own forward; the adjoint takes its own waveform residual)
    eng = gpu_engine(grid)
    gpu_source(eng, grid, SRC, n)
    eng.set_state(to_dev(phi0), to_dev(pi0))
    wg = eng.step(n)
    gwg = (2.0 * (wg - to_dev(y))).contiguous()
    eng.adjoint_begin(n, gw=gwg)
    eng.adjoint_step(n)
    p, q, dA = eng.adjoint_get()
    e = (rel(host(p), rgp), rel(host(q), rgq), abs(dA - rdA) / abs(rdA))
    print("reverse sweep vs oracle (grad Phi0, grad Pi0, dL/dA):", e)
    assert max(e) <= 1e-12, e


def test_gradient_matches_central_differences_on_gpu():
    grid, n = _adjoint_case()
    g = T.Grid(**grid)
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    y = to_dev(W.target_noise((n, g.nth), 0.05, seed=4))
    eng = gpu_engine(grid)
    gpu_source(eng, grid, SRC, n)

    def loss(p, q, A):
        eng.set_amplitude(A)
        eng.set_state(p, q)
        w = eng.step(n)
        return float(torch.sum(torch.abs(w - y) ** 2)), w

    P0, Q0 = to_dev(phi0), to_dev(pi0)
    L0, w = loss(P0, Q0, 1.0)
    gw = (2.0 * (w - y)).contiguous()
    eng.adjoint_begin(n, gw=gw)
    eng.adjoint_step(n)
    gp, gq, gA = eng.adjoint_get()
    x2 = float(torch.sum(torch.abs(P0) ** 2) + torch.sum(torch.abs(Q0) ** 2) + 1.0)
    h = 1e-3 * np.sqrt(x2)
    for vp, vq, vA in W.fd_directions(g.nth, g.nr, ndir=8, seed=44):
        Vp, Vq = to_dev(vp), to_dev(vq)
        fd = (loss(P0 + h * Vp, Q0 + h * Vq, 1.0 + h * vA)[0]
              - loss(P0 - h * Vp, Q0 - h * Vq, 1.0 - h * vA)[0]) / (2 * h)
        ad = float(torch.real(torch.vdot(gp.flatten(), Vp.flatten()) + torch.vdot(gq.flatten(), Vq.flatten()))) + gA * vA
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-8 * L0), (fd, ad)


@pytest.mark.parametrize("grid", [STEP_GRIDS[0], STEP_GRIDS[1]])
def test_reverse_sweep_bitwise_invariant_to_segment_length(grid):
    lp, lq = W.random_state(grid["nth"], grid["nr"], seed=41)
    gw = to_dev(W.target_noise((6, grid["nth"]), 1.0, seed=42))
    outs = []
    for seg in (4, 8, 16):
        eng = gpu_engine(grid)
        eng.set_tuning(seg)
        gpu_source(eng, grid, SRC, 6)
        eng.adjoint_begin(6, to_dev(lp), to_dev(lq), gw=gw)
        eng.adjoint_step(6)
        p, q, dA = eng.adjoint_get()
        outs.append((host(p), host(q), dA))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
        assert abs(o[2] - outs[0][2]) <= 1e-13 * abs(outs[0][2])


def test_autograd_function_gradients():
    from paper_1001_3631_amd.autograd import evolve
    grid, n = _adjoint_case(60)
    g = T.Grid(**grid)
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    eng = gpu_engine(grid)
    gpu_source(eng, grid, SRC, n)
    P0 = to_dev(phi0).requires_grad_(True)
    Q0 = to_dev(pi0).requires_grad_(True)
    A = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    y = to_dev(W.target_noise((n, g.nth), 0.05, seed=4))
    w = evolve(P0, Q0, A, eng, n)
    L = torch.sum(torch.abs(w - y) ** 2)
    L.backward()
    # reference: the same adjoint driven by hand (torch forms d|w-y|^2/dw with
    # its own operation order, so agreement is to rounding, not bitwise)
    eng.adjoint_begin(n, gw=(2.0 * (w.detach() - y)).contiguous())
    eng.adjoint_step(n)
    gp, gq, gA = eng.adjoint_get()
    assert rel(host(P0.grad), host(gp)) <= 1e-13 and rel(host(Q0.grad), host(gq)) <= 1e-13
    assert abs(float(A.grad) - gA) <= 1e-13 * abs(gA)
