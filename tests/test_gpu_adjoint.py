"""GPU adjoint (teuk_adjoint_*) against the oracle's hand-transposed sweep,
the dot-product identity, central differences of the GPU forward, and the
torch.autograd wrapper."""

import ctypes

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


def test_reverse_steps_compose_and_zero_steps_do_nothing():
    """A reverse sweep taken as [n], or as [0, 37, 0, n - 37, 0] reverse
    iterations: the same lambda bit for bit and dL/dA to rounding (reading
    it mid-sweep sums its partials in other groups); a call of no
    iterations changes nothing."""
    grid, n = _adjoint_case(60)
    g = T.Grid(**grid)
    lp, lq = W.random_state(g.nth, g.nr, seed=91)
    gw = to_dev(W.target_noise((n, g.nth), 1.0, seed=92))
    outs = []
    for split in ([n], [0, 37, 0, n - 37, 0]):
        eng = gpu_engine(grid)
        gpu_source(eng, grid, SRC, n)
        eng.adjoint_begin(n, to_dev(lp), to_dev(lq), gw=gw)
        for k in split:
            before = eng.adjoint_get() if k == 0 else None
            eng.adjoint_step(k)
            if before is not None:
                after = eng.adjoint_get()
                assert torch.equal(after[0], before[0]) and torch.equal(after[1], before[1])
                assert after[2] == before[2]
        outs.append(eng.adjoint_get())
        eng.close()
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    assert abs(outs[0][2] - outs[1][2]) <= 1e-13 * abs(outs[0][2]), (outs[0][2], outs[1][2])


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
        eng.set_tuning(seg, 1, seg)
        assert eng.tuning["adj_seg_rows"] == seg
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


def test_autograd_function_matches_oracle_reverse_sweep():
    """torch.autograd through TeukEvolve against the oracle's own reverse
    sweep (not the engine's adjoint): the loss sum |w - y|^2 differentiated
    with respect to the initial data and the source amplitude."""
    from paper_1001_3631_amd.autograd import evolve
    grid, n = _adjoint_case(80)
    g = T.Grid(**grid)
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    y = W.target_noise((n, g.nth), 0.05, seed=4)
    src = oracle_source(g, SRC, n)
    w = T.evolve(g, phi0, pi0, n, src)[2]
    _, gw = T.waveform_loss(w, y)
    rgp, rgq, rdA = T.adjoint_evolve(g, gw, n, src)
    eng = gpu_engine(grid)
    gpu_source(eng, grid, SRC, n)
    P0 = to_dev(phi0).requires_grad_(True)
    Q0 = to_dev(pi0).requires_grad_(True)
    A = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = torch.sum(torch.abs(evolve(P0, Q0, A, eng, n) - to_dev(y)) ** 2)
    L.backward()
    e = (rel(host(P0.grad), rgp), rel(host(Q0.grad), rgq), abs(float(A.grad) - rdA) / abs(rdA))
    print("autograd vs oracle reverse sweep (grad Phi0, grad Pi0, dL/dA):", e)
    assert max(e) <= 1e-12, e


def test_checkpointed_autograd_refuses_snapshots_of_a_later_forward():
    """Two checkpointed forwards on one engine: the engine holds the second
    one's snapshots, so the first node's backward must refuse to run, and
    the second node's backward still gives the right gradient."""
    from paper_1001_3631_amd.autograd import TeukEvolveCheckpointed
    grid, n = _adjoint_case(40)
    g = T.Grid(**grid)
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    eng = gpu_engine(grid)
    gpu_source(eng, grid, SRC, n)
    sl = dict(STATE_LOSS, n_lo=10, n_hi=30)
    A = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    P0 = to_dev(phi0).requires_grad_(True)
    Q0 = to_dev(pi0).requires_grad_(True)
    _, ls1 = TeukEvolveCheckpointed.apply(P0, Q0, A, eng, n, sl, 0)
    P1 = to_dev(0.5 * phi0).requires_grad_(True)
    Q1 = to_dev(0.5 * pi0).requires_grad_(True)
    _, ls2 = TeukEvolveCheckpointed.apply(P1, Q1, A, eng, n, sl, 0)
    with pytest.raises(RuntimeError, match="another checkpointed forward"):
        ls1.backward()
    ls2.backward()
    # reference: the same loss and engine, one forward and one backward
    eng2 = gpu_engine(grid)
    gpu_source(eng2, grid, SRC, n)
    P2 = to_dev(0.5 * phi0).requires_grad_(True)
    Q2 = to_dev(0.5 * pi0).requires_grad_(True)
    A2 = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    _, ls3 = TeukEvolveCheckpointed.apply(P2, Q2, A2, eng2, n, sl, 0)
    ls3.backward()
    assert torch.equal(P1.grad, P2.grad) and torch.equal(Q1.grad, Q2.grad)


# ---------------------------------------------------------------------------
# Checkpointed gradient (snapshots + recompute) for losses on the states
# ---------------------------------------------------------------------------

STATE_LOSS = dict(weight=0.7, i0=40, i1=121, j0=5, j1=21, n_lo=30, n_hi=100)


def _masked(phi, sl):
    out = np.zeros_like(phi)
    out[sl["j0"]:sl["j1"], sl["i0"]:sl["i1"]] = phi[sl["j0"]:sl["j1"], sl["i0"]:sl["i1"]]
    return out


def test_checkpoint_recompute_equals_residual_only_bitwise():
    grid, n = _adjoint_case()
    g = T.Grid(**grid)
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    y = to_dev(W.target_noise((n, g.nth), 0.05, seed=4))
    eng = gpu_engine(grid)
    gpu_source(eng, grid, SRC, n)
    eng.set_state(to_dev(phi0), to_dev(pi0))
    w = eng.step(n)
    gw = (2.0 * (w - y)).contiguous()
    eng.adjoint_begin(n, gw=gw)
    eng.adjoint_step(n)
    gp0, gq0, dA0 = eng.adjoint_get()
    for interval in (0, 7, n):
        eng.set_state(to_dev(phi0), to_dev(pi0))
        w2, _ = eng.forward_checkpointed(n, interval=interval, force_recompute=True)
        assert torch.equal(w2, w)
        gp, gq, dA = eng.backward_checkpointed(gw)
        assert torch.equal(gp, gp0) and torch.equal(gq, gq0) and dA == dA0


@pytest.mark.parametrize("snapshots", [1, 2, 3, 6, 200])
def test_binomial_schedule_gradient_equals_uniform_bitwise(snapshots):
    """The binomial schedule runs the same reverse iterations with the same
    forward states as the uniform one, only recomputed in another order: the
    state loss, the waveform and every gradient are bitwise equal, from one
    slot (every reverse iteration restarts at u^0) to more slots than
    iterations."""
    grid, n = _adjoint_case(90)
    g = T.Grid(**grid)
    sl = dict(STATE_LOSS, n_lo=5, n_hi=80)
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    y = to_dev(W.target_noise((n, g.nth), 0.05, seed=4))
    eng = gpu_engine(grid)
    gpu_source(eng, grid, SRC, n)
    out = []
    for snaps in (0, snapshots):
        eng.set_state(to_dev(phi0), to_dev(pi0))
        w, ls = eng.forward_checkpointed(n, state_loss=sl, snapshots=snaps)
        gp, gq, dA = eng.backward_checkpointed((2.0 * (w - y)).contiguous(), 1.0)
        out.append((w, ls, gp, gq, dA))
    (w0, ls0, gp0, gq0, dA0), (w1, ls1, gp1, gq1, dA1) = out
    assert torch.equal(w0, w1) and ls0 == ls1
    assert torch.equal(gp0, gp1) and torch.equal(gq0, gq1) and dA0 == dA1
    # forced recomputation without a state loss: the residual-only sweep's gradient
    gw = (2.0 * (w0 - y)).contiguous()
    eng.set_state(to_dev(phi0), to_dev(pi0))
    eng.forward_checkpointed(n, snapshots=snapshots, force_recompute=True)
    gpf, gqf, dAf = eng.backward_checkpointed(gw)
    eng.set_state(to_dev(phi0), to_dev(pi0))
    eng.step(n, waveform=False)
    eng.adjoint_begin(n, gw=gw)
    eng.adjoint_step(n)
    gpr, gqr, dAr = eng.adjoint_get()
    assert torch.equal(gpf, gpr) and torch.equal(gqf, gqr) and dAf == dAr


def test_binomial_plan_buffer_is_checked():
    grid, n = _adjoint_case(40)
    eng = gpu_engine(grid)
    nb = eng.checkpoint_bytes(n, snapshots=3)
    assert eng.checkpoint_bytes(n, snapshots=4) > nb
    assert eng.snapshots_for_budget(n, nb) == 3
    assert eng.snapshots_for_budget(n, 10 * nb) >= 9
    from paper_1001_3631_amd import _lib as L
    plan = eng._make_plan(n, 0, None, False, 3)
    small = torch.empty(nb - 256, dtype=torch.uint8, device="cuda")
    plan.ckpt_dev, plan.ckpt_bytes = small.data_ptr(), small.numel()
    assert eng._lib.teuk_forward_checkpointed(eng.ctx, ctypes.byref(plan), None, None) == L.TEUK_ENOMEM
    plan = eng._make_plan(n, 5, None, False, 3)          # interval and snapshots together
    assert eng._lib.teuk_checkpoint_size(eng.ctx, ctypes.byref(plan), ctypes.byref(ctypes.c_size_t())) == \
        L.TEUK_EINVAL


def test_checkpointed_state_loss_gradient_matches_oracle():
    grid, n = _adjoint_case()
    g = T.Grid(**grid)
    sl = STATE_LOSS
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    y = W.target_noise((n, g.nth), 0.05, seed=4)
    src = oracle_source(g, SRC, n)
    snaps = {k: None for k in range(sl["n_lo"], sl["n_hi"] + 1)}
    w = T.evolve(g, phi0, pi0, n, src, snapshots=snaps)[2]
    rls = sl["weight"] * sum(np.sum(np.abs(_masked(snaps[k][0], sl)) ** 2) for k in snaps)
    _, gw = T.waveform_loss(w, y)
    z = np.zeros_like(phi0)
    sg = lambda k: (2 * sl["weight"] * _masked(snaps[k][0], sl), z) if k in snaps else None
    rgp, rgq, rdA = T.adjoint_evolve(g, gw, n, src, state_grad=sg)
    eng = gpu_engine(grid)
    gpu_source(eng, grid, SRC, n)
    eng.set_state(to_dev(phi0), to_dev(pi0))
    wg, ls = eng.forward_checkpointed(n, interval=0, state_loss=sl)
    assert abs(ls - rls) <= 1e-12 * rls
    gp, gq, dA = eng.backward_checkpointed((2.0 * (wg - to_dev(y))).contiguous(), 1.0)
    e = (rel(host(gp), rgp), rel(host(gq), rgq), abs(dA - rdA) / abs(rdA))
    print("checkpointed state-loss gradient vs oracle:", e)
    assert max(e) <= 1e-12, e


def test_checkpointed_gradient_central_differences_and_interval_invariance():
    grid, n = _adjoint_case()
    g = T.Grid(**grid)
    sl = STATE_LOSS
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    y = to_dev(W.target_noise((n, g.nth), 0.05, seed=4))
    eng = gpu_engine(grid)
    gpu_source(eng, grid, SRC, n)

    def loss(p, q, A, interval=0):
        eng.set_amplitude(A)
        eng.set_state(p, q)
        w, ls = eng.forward_checkpointed(n, interval=interval, state_loss=sl)
        return float(torch.sum(torch.abs(w - y) ** 2)) + ls, w

    P0, Q0 = to_dev(phi0), to_dev(pi0)
    grads = []
    for interval in (0, 13, n):
        L0, w = loss(P0, Q0, 1.0, interval)
        grads.append(eng.backward_checkpointed((2.0 * (w - y)).contiguous(), 1.0))
    for gr in grads[1:]:
        assert torch.equal(gr[0], grads[0][0]) and torch.equal(gr[1], grads[0][1]) and gr[2] == grads[0][2]
    gp, gq, gA = grads[0]
    h = 1e-3 * np.sqrt(float(torch.sum(torch.abs(P0) ** 2) + torch.sum(torch.abs(Q0) ** 2) + 1.0))
    for vp, vq, vA in W.fd_directions(g.nth, g.nr, ndir=4, seed=45):
        Vp, Vq = to_dev(vp), to_dev(vq)
        fd = (loss(P0 + h * Vp, Q0 + h * Vq, 1.0 + h * vA)[0] - loss(P0 - h * Vp, Q0 - h * Vq, 1.0 - h * vA)[0]) / (2 * h)
        ad = float(torch.real(torch.vdot(gp.flatten(), Vp.flatten()) + torch.vdot(gq.flatten(), Vq.flatten()))) + gA * vA
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-8 * L0), (fd, ad)


def test_autograd_checkpointed_function():
    from paper_1001_3631_amd.autograd import TeukEvolveCheckpointed
    grid, n = _adjoint_case(60)
    g = T.Grid(**grid)
    sl = dict(STATE_LOSS, n_lo=10, n_hi=50)
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    eng = gpu_engine(grid)
    gpu_source(eng, grid, SRC, n)
    P0 = to_dev(phi0).requires_grad_(True)
    Q0 = to_dev(pi0).requires_grad_(True)
    A = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    y = to_dev(W.target_noise((n, g.nth), 0.05, seed=4))
    w, ls = TeukEvolveCheckpointed.apply(P0, Q0, A, eng, n, sl, 0)
    L = torch.sum(torch.abs(w - y) ** 2) + 3.0 * ls
    L.backward()
    eng.set_state(to_dev(phi0), to_dev(pi0))
    w2, _ = eng.forward_checkpointed(n, 0, sl)
    gp, gq, gA = eng.backward_checkpointed((2.0 * (w2 - y)).contiguous(), 3.0)
    assert rel(host(P0.grad), host(gp)) <= 1e-13 and rel(host(Q0.grad), host(gq)) <= 1e-13
    assert abs(float(A.grad) - gA) <= 1e-13 * abs(gA)


# ---------------------------------------------------------------------------
# Full-size adjoint workload: 3200 x 64, a = 0.7, 20000 iterations
# ---------------------------------------------------------------------------

def _adjoint_fullsize():
    cfg = W.ADJOINT
    grid, n = cfg["grid"], cfg["steps"]
    eng = gpu_engine(grid)
    gpu_source(eng, grid, cfg["source"], n)
    return cfg, grid, n, eng


def test_adjoint_fullsize_one_reverse_iteration_against_oracle():
    """A reverse sweep of 200 iterations from a seeded lambda on the GPU, then
    one more GPU reverse iteration against one oracle reverse iteration
    applied to the same GPU lambda (whole field and dL/dA)."""
    cfg, grid, n, eng = _adjoint_fullsize()
    g = T.Grid(**grid)
    lp, lq = W.random_state(g.nth, g.nr, seed=51)
    m0 = 5000
    eng.adjoint_begin(m0 + 200, to_dev(lp), to_dev(lq))
    eng.adjoint_step(200)
    p0, q0, _ = eng.adjoint_get(want_dA=False)
    p0, q0 = host(p0), host(q0)
    eng.adjoint_begin(m0, to_dev(p0), to_dev(q0))
    eng.adjoint_step(1)
    p1, q1, dA = eng.adjoint_get()
    src = oracle_source(g, cfg["source"], n)
    rp, rq, rdA = T.adjoint_step(g, p0, q0, m0 - 1, src)
    assert rel(host(p1), rp) <= 1e-13 and rel(host(q1), rq) <= 1e-13
    assert abs(dA - rdA) <= 1e-12 * abs(rdA)


def test_adjoint_fullsize_gradient_vs_central_differences_32_directions():
    """Loss sum |w - y|^2 against a target from the same system with A = 1.25
    and the pulse at 52M plus 1 % seeded noise; the adjoint gradient with
    respect to all initial data and A against central differences along 32
    seeded unit directions, h = 1e-3 |x| (the loss is quadratic, so the
    differences are exact up to rounding)."""
    cfg, grid, n, eng = _adjoint_fullsize()
    nth, nr = grid["nth"], grid["nr"]
    tg = cfg["target"]
    eng.init_pulse(tg["center"], cfg["pulse"]["width"], cfg["pulse"]["amplitude"])
    eng.set_amplitude(tg["amplitude"])
    y = eng.step(n)
    rms = float(torch.sqrt(torch.mean(torch.abs(y) ** 2)))
    y = y + to_dev(W.target_noise((n, nth), tg["noise_rel"] * rms, seed=tg["seed"]))
    eng.init_pulse(**cfg["pulse"])
    P0, Q0 = [t.clone() for t in eng.get_state()]

    def loss(p, q, A):
        eng.set_amplitude(A)
        eng.set_state(p, q)
        w = eng.step(n)
        return float(torch.sum(torch.abs(w - y) ** 2)), w

    L0, w = loss(P0, Q0, 1.0)
    gw = (2.0 * (w - y)).contiguous()
    eng.adjoint_begin(n, gw=gw)
    eng.adjoint_step(n)
    gp, gq, gA = eng.adjoint_get()
    h = 1e-3 * float(torch.sqrt(torch.sum(torch.abs(P0) ** 2) + torch.sum(torch.abs(Q0) ** 2) + 1.0))
    worst = 0.0
    for vp, vq, vA in W.fd_directions(nth, nr, ndir=cfg["fd"]["ndir"], seed=cfg["fd"]["seed"]):
        Vp, Vq = to_dev(vp), to_dev(vq)
        fd = (loss(P0 + h * Vp, Q0 + h * Vq, 1.0 + h * vA)[0] - loss(P0 - h * Vp, Q0 - h * Vq, 1.0 - h * vA)[0]) / (2 * h)
        ad = float(torch.real(torch.vdot(gp.flatten(), Vp.flatten()) + torch.vdot(gq.flatten(), Vq.flatten()))) + gA * vA
        worst = max(worst, abs(fd - ad) / max(abs(ad), 1e-300))
    print("adjoint_3200x64: worst relative |FD - adjoint| over 32 directions:", worst)
    assert worst <= 1e-6


def test_adjoint_segment_setting():
    """teuk_tuning.adj_seg_rows: default 4 on a small grid and 16 where
    16-row segments give more waves than SIMDs, 0 keeps the current value,
    the stepper's own settings do not touch it, invalid values are refused."""
    from paper_1001_3631_amd import _lib as L
    nsimd = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    for grid, waves16 in ((W.KERR_EMRI["grid"], 104 * 8), (W.SCALE_GRID["grid"], 207 * 16)):
        big = gpu_engine(grid)
        assert big.tuning["adj_seg_rows"] == (16 if waves16 > nsimd else 4)
        big.close()
    eng = gpu_engine(STEP_GRIDS[0])
    assert eng.tuning["adj_seg_rows"] == 4
    eng.set_tuning(8, 1, 16)
    assert eng.tuning == {"seg_rows": 8, "k_steps": 1, "adj_seg_rows": 16}
    eng.set_tuning(4, 2)
    assert eng.tuning == {"seg_rows": 4, "k_steps": 2, "adj_seg_rows": 16}
    with pytest.raises(L.TeukError):
        eng.set_tuning(8, 1, 5)
    assert eng.tuning == {"seg_rows": 4, "k_steps": 2, "adj_seg_rows": 16}
    eng.close()


@pytest.mark.parametrize("adj_seg", [4, 8])
@pytest.mark.parametrize("th_cells", [None, 2.5, 124.5], ids=["equator", "near_theta0", "near_theta_pi"])
def test_split_reverse_iteration_against_oracle(th_cells, adj_seg):
    """On a grid of more adjoint waves than SIMDs (6400 x 128: 3328 waves at
    segments of 4, 1664 at 8) the reverse iteration with a source is split: with the
    windows away from the poles every wave runs without source terms and
    dL/dA comes from the windows alone; with a window that reaches the pole
    rows the waves near it run in a launch of their own.  Both against one
    oracle reverse iteration on the same lambda, whole field and dL/dA; the
    particle sits on the equator or two and a half cells from a pole (an
    orbit table given to both sides)."""
    grid = W.KERR_EMRI["grid"]
    g = T.Grid(**grid)
    n = 8
    th_p = 0.5 * np.pi if th_cells is None else th_cells * g.hth
    t = np.arange(2 * n + 1) * 0.5 * g.dt
    rs_p = 12.7834
    orbit = {"rs": np.full(t.shape, rs_p), "th": np.full(t.shape, th_p), "phi": 0.0307 * t}
    eng = gpu_engine(grid)
    eng.set_tuning(8, 1, adj_seg)
    eng.set_source(np.stack([orbit["rs"], orbit["th"], orbit["phi"]], axis=1), 1.0, 2.0, 2.0, 8.0)
    src = T.Source(g, orbit, 1.0, 2.0, 2.0, 8.0)
    lp, lq = W.random_state(g.nth, g.nr, seed=61)
    m0 = n - 2
    eng.adjoint_begin(m0, to_dev(lp), to_dev(lq))
    eng.adjoint_step(1)
    p1, q1, dA = eng.adjoint_get()
    rp, rq, rdA = T.adjoint_step(g, lp, lq, m0 - 1, src)
    e = (rel(host(p1), rp), rel(host(q1), rq), abs(dA - rdA) / abs(rdA))
    print("split reverse iteration", th_cells, adj_seg, e)
    assert e[0] <= 1e-13 and e[1] <= 1e-13 and e[2] <= 1e-12, e


@pytest.mark.parametrize("adj_seg", [4, 8])
@pytest.mark.parametrize("th_cells", [None, 2.5, 60.5], ids=["equator", "near_theta0", "near_theta_pi"])
def test_small_grid_reverse_iteration_against_oracle(th_cells, adj_seg):
    """On a grid of fewer adjoint waves than SIMDs (3200 x 64: 832 waves at
    segments of 4) the reverse iteration with a source is one launch: with
    the windows clear of the poles every wave runs without source terms and
    dL/dA comes from the windows; with a window that reaches the pole rows
    every body runs in the one launch.  Against one oracle reverse
    iteration on the same lambda, whole field and dL/dA."""
    grid = W.ADJOINT["grid"]
    g = T.Grid(**grid)
    n = 8
    th_p = 0.5 * np.pi if th_cells is None else th_cells * g.hth
    t = np.arange(2 * n + 1) * 0.5 * g.dt
    orbit = {"rs": np.full(t.shape, 12.7834), "th": np.full(t.shape, th_p), "phi": 0.0307 * t}
    eng = gpu_engine(grid)
    eng.set_tuning(4, 1, adj_seg)
    eng.set_source(np.stack([orbit["rs"], orbit["th"], orbit["phi"]], axis=1), 1.0, 2.0, 2.0, 8.0)
    src = T.Source(g, orbit, 1.0, 2.0, 2.0, 8.0)
    lp, lq = W.random_state(g.nth, g.nr, seed=63)
    m0 = n - 2
    eng.adjoint_begin(m0, to_dev(lp), to_dev(lq))
    eng.adjoint_step(1)
    p1, q1, dA = eng.adjoint_get()
    rp, rq, rdA = T.adjoint_step(g, lp, lq, m0 - 1, src)
    e = (rel(host(p1), rp), rel(host(q1), rq), abs(dA - rdA) / abs(rdA))
    print("small-grid reverse iteration", th_cells, adj_seg, e)
    assert e[0] <= 1e-13 and e[1] <= 1e-13 and e[2] <= 1e-12, e


@pytest.mark.parametrize("th_cells", [None, 2.5], ids=["equator", "near_theta0"])
def test_large_grid_reverse_sweep_bitwise_across_segments(th_cells):
    """6400 x 128 with a source: the reverse sweep at adjoint segments of 4,
    8 and 16 rows (split launches with window dL/dA, split launches with
    a launch for the waves near a pole window, one launch) gives the same
    lambda bit for bit; dL/dA, summed from differently grouped partials,
    agrees to rounding."""
    grid = W.KERR_EMRI["grid"]
    g = T.Grid(**grid)
    n = 6
    th_p = 0.5 * np.pi if th_cells is None else th_cells * g.hth
    t = np.arange(2 * n + 3) * 0.5 * g.dt
    orbit = np.stack([np.full(t.shape, 12.7834), np.full(t.shape, th_p), 0.0307 * t], axis=1)
    lp, lq = W.random_state(g.nth, g.nr, seed=71)
    gw = to_dev(W.target_noise((n, g.nth), 1.0, seed=72))
    outs = []
    for seg in (4, 8, 16):
        eng = gpu_engine(grid)
        eng.set_tuning(8, 1, seg)
        eng.set_source(orbit, 1.0, 2.0, 2.0, 8.0)
        eng.adjoint_begin(n, to_dev(lp), to_dev(lq), gw=gw)
        eng.adjoint_step(n)
        p, q, dA = eng.adjoint_get()
        outs.append((p, q, dA))
        eng.close()
    for p, q, dA in outs[1:]:
        assert torch.equal(p, outs[0][0]) and torch.equal(q, outs[0][1])
        assert abs(dA - outs[0][2]) <= 1e-13 * abs(outs[0][2]), (dA, outs[0][2])


@pytest.mark.parametrize("adj_seg", [4, 8, 16])
def test_large_grid_reverse_iteration_without_source_against_oracle(adj_seg):
    """Without a source on 6400 x 128 (more waves than SIMDs at 4 and 8
    rows: the general-form waves dispatched first), one reverse iteration
    with the waveform residual against the oracle's, every point."""
    grid = W.KERR_EMRI["grid"]
    g = T.Grid(**grid)
    lp, lq = W.random_state(g.nth, g.nr, seed=81)
    gw = W.target_noise((3, g.nth), 1.0, seed=82)
    eng = gpu_engine(grid)
    eng.set_tuning(8, 1, adj_seg)
    eng.adjoint_begin(3, to_dev(lp), to_dev(lq), gw=to_dev(gw))
    eng.adjoint_step(1)
    p1, q1, _ = eng.adjoint_get(want_dA=False)
    mp, mq = lp.copy(), lq.copy()
    mp[:, g.i_ext] += gw[2]
    rp, rq, _ = T.adjoint_step(g, mp, mq, 2, None)
    rp[:, g.i_ext] += gw[1]        # the residual of iteration 2, added after the step
    e = (rel(host(p1), rp), rel(host(q1), rq))
    print("large grid, no source, adj seg", adj_seg, e)
    assert max(e) <= 1e-13, e
    eng.close()
