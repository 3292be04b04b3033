"""Eccentric-orbit sources: the HIP path with the library's orbit table
against the oracle with its own (independently built) orbit, for the field,
the waveform and the gradient; and the 16-instance 12800 x 256 workload's
forward + checkpointed adjoint checked at full size through properties that
hold at any size (dL/dA in closed form, the adjoint identity along seeded
directions; the split adjoint launch against the single one)."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import teuk_oracle as T
from paper_1001_3631_amd import workloads as W
from test_gpu_parity import gpu_engine, host, rel, to_dev

SMALL = dict(M=1.0, a=0.9, s=-2, m=2, nr=200, nth=41, rs_min=-40.0, rs_max=60.0, cfl=0.5,
             rs_extract=40.0, ko_eps=0.5)
SRC = dict(amplitude=1.0, sigma_r_cells=2.0, sigma_th_cells=2.0, cutoff_sigmas=8.0)

CASES = [
    (SMALL, dict(p=10.0, e=0.4, chi0=0.7)),
    (dict(SMALL, a=0.3, m=3, nth=37, cfl=0.25), dict(p=8.0, e=0.5, chi0=2.0)),
]


def _gpu(grid, orb, n):
    eng = gpu_engine(grid)
    table = eng.orbit_eccentric(orb["p"], orb["e"], 2 * n + 1, M=grid["M"], a=grid["a"], chi0=orb["chi0"])
    eng.set_source(table, SRC["amplitude"], SRC["sigma_r_cells"], SRC["sigma_th_cells"], SRC["cutoff_sigmas"])
    return eng


def _oracle_source(g, orb, n):
    table = T.eccentric_orbit(g.M, g.a, orb["p"], orb["e"], orb["chi0"], g.dt, n)
    return T.Source(g, table, SRC["amplitude"], SRC["sigma_r_cells"], SRC["sigma_th_cells"],
                    SRC["cutoff_sigmas"])


@pytest.mark.parametrize("grid,orb", CASES)
def test_eccentric_source_evolution_matches_oracle(grid, orb):
    n = 240
    g = T.Grid(**grid)
    phi0, pi0 = T.initial_pulse(g, 20.0, 4.0)
    rp, rq, rw = T.evolve(g, phi0, pi0, n, _oracle_source(g, orb, n))
    eng = _gpu(grid, orb, n)
    eng.set_state(to_dev(phi0), to_dev(pi0))
    w = eng.step(n)
    p, q = eng.get_state()
    e = (rel(host(p), rp), rel(host(q), rq), rel(host(w), rw))
    print(f"eccentric source {grid['nr']}x{grid['nth']} {orb}: rel L2 (Phi, Pi, w) = {e}")
    assert max(e) <= 1e-12, e
    eng.close()


@pytest.mark.parametrize("grid,orb", CASES[:1])
def test_eccentric_source_gradient_matches_oracle(grid, orb):
    n = 160
    g = T.Grid(**grid)
    phi0, pi0 = T.initial_pulse(g, 20.0, 4.0)
    src = _oracle_source(g, orb, n)
    y = W.target_noise((n, g.nth), 0.05, seed=4)
    w = T.evolve(g, phi0, pi0, n, src)[2]
    _, gw = T.waveform_loss(w, y)
    rgp, rgq, rdA = T.adjoint_evolve(g, gw, n, src)
    eng = _gpu(grid, orb, n)
    eng.set_state(to_dev(phi0), to_dev(pi0))
    wg = eng.step(n)
    gwg = (2.0 * (wg - to_dev(y))).contiguous()
    eng.adjoint_begin(n, gw=gwg)
    eng.adjoint_step(n)
    p, q, dA = eng.adjoint_get()
    e = (rel(host(p), rgp), rel(host(q), rgq), abs(dA - rdA) / abs(rdA))
    print("eccentric source gradient vs oracle (grad Phi0, grad Pi0, dL/dA):", e)
    assert max(e) <= 1e-12, e
    eng.close()


def test_adjoint_at_scale_instance_full_size():
    """The most eccentric, fastest-spinning instance of the 16 (12800 x 256,
    a = 0.949, m = 3, e = 0.467) in the configuration the benchmark runs:
    forward keeping snapshots every ceil(sqrt(N)) iterations, backward
    recomputing every segment.  The extraction radius is moved in to
    r* = 30M so that the short run here sees the signal.  Loss sum |w - y|^2
    with y = 0.9 w (zero initial data: w is linear in A), so
    dL/dA = 0.2 |w|^2; and for the initial data the adjoint identity
    Re<dL/du0, v> = 2 Re<w - y, G v>, with G v the waveform of a forward run
    from v with the source off, along two seeded directions."""
    cfg = W.ADJOINT_AT_SCALE
    inst = W.adjoint_at_scale_instances(cfg["seed"], cfg["instances"])[9]
    grid, orb = dict(inst["grid"], rs_extract=30.0), inst["orbit"]
    assert grid["nr"] == 12800 and grid["nth"] == 256 and orb["e"] > 0.45 and grid["a"] > 0.94
    n = 6000
    eng = _gpu(grid, orb, n)
    eng.autotune(None)
    z = torch.zeros((grid["nth"], grid["nr"]), dtype=torch.complex128, device="cuda")
    eng.set_state(z, z)
    w, _ = eng.forward_checkpointed(n, interval=0, force_recompute=True)
    eng.check_finite()
    wn2 = float(torch.sum(torch.abs(w) ** 2))
    assert wn2 > 0.0
    r = (1.0 - cfg["target_amplitude"]) * w               # w - y
    gp, gq, dA = eng.backward_checkpointed((2.0 * r).contiguous(), 0.0)
    e_dA = abs(dA - 2.0 * (1.0 - cfg["target_amplitude"]) * wn2) / (2.0 * (1.0 - cfg["target_amplitude"]) * wn2)
    worst = 0.0
    eng.set_amplitude(0.0)
    for vp, vq, _ in W.fd_directions(grid["nth"], grid["nr"], ndir=2, seed=45):
        Vp, Vq = to_dev(vp), to_dev(vq)
        eng.set_state(Vp, Vq)
        Gv = eng.step(n)
        lhs = float(torch.real(torch.vdot(gp.flatten(), Vp.flatten()) + torch.vdot(gq.flatten(), Vq.flatten())))
        rhs = 2.0 * float(torch.real(torch.vdot(r.flatten(), Gv.flatten())))
        worst = max(worst, abs(lhs - rhs) / max(abs(rhs), 1e-300))
    print(f"adjoint at scale (instance 9, {n} iterations): dL/dA rel {e_dA:.3e}, "
          f"adjoint identity worst rel {worst:.3e}")
    assert e_dA <= 1e-10
    assert worst <= 1e-9
    eng.close()


@pytest.mark.parametrize("adj_seg", [4, 8, 16])
def test_adjoint_at_scale_one_reverse_iteration_against_oracle(adj_seg):
    """One GPU reverse iteration on 12800 x 256 (13248, 6624 or 3312 waves) with
    the eccentric source, from a lambda made by 20 GPU reverse iterations
    from a seeded state, against one oracle reverse iteration on the same
    lambda: every point, including the strip seams inside the source window."""
    cfg = W.ADJOINT_AT_SCALE
    inst = W.adjoint_at_scale_instances(cfg["seed"], cfg["instances"])[9]
    grid, orb = inst["grid"], inst["orbit"]
    g = T.Grid(**grid)
    m0 = 150
    eng = _gpu(grid, orb, m0 + 40)
    eng.set_tuning(8, 1, adj_seg)
    lp, lq = W.random_state(g.nth, g.nr, seed=52)
    eng.adjoint_begin(m0 + 20, to_dev(lp), to_dev(lq))
    eng.adjoint_step(20)
    p0, q0, _ = eng.adjoint_get(want_dA=False)
    p0, q0 = host(p0), host(q0)
    eng.adjoint_begin(m0, to_dev(p0), to_dev(q0))
    eng.adjoint_step(1)
    p1, q1, dA = eng.adjoint_get()
    rp, rq, rdA = T.adjoint_step(g, p0, q0, m0 - 1, _oracle_source(g, orb, m0 + 40))
    e = (rel(host(p1), rp), rel(host(q1), rq), abs(dA - rdA) / abs(rdA))
    print(f"adjoint at scale, one reverse iteration, adj seg {adj_seg}: {e}")
    assert e[0] <= 1e-13 and e[1] <= 1e-13 and e[2] <= 1e-12, e
    eng.close()


def test_adjoint_split_launch_bitwise_equal_to_single_launch():
    """On 12800 x 256 with a source, adjoint segments of 4 rows run as two
    launches (waves without the source window, then waves with it); 8 and 16
    rows run as one.  The same reverse sweep from a seeded lambda gives the
    same bits either way, and dL/dA to the reduction's rounding."""
    cfg = W.ADJOINT_AT_SCALE
    inst = W.adjoint_at_scale_instances(cfg["seed"], cfg["instances"])[9]
    grid, orb = inst["grid"], inst["orbit"]
    lp, lq = W.random_state(grid["nth"], grid["nr"], seed=53)
    gw = to_dev(W.target_noise((8, grid["nth"]), 1.0, seed=54))
    outs = []
    for seg in (4, 8, 16):
        eng = _gpu(grid, orb, 40)
        eng.set_tuning(8, 1, seg)
        eng.adjoint_begin(8, to_dev(lp), to_dev(lq), gw=gw)
        eng.adjoint_step(8)
        p, q, dA = eng.adjoint_get()
        outs.append((host(p), host(q), dA))
        eng.close()
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
        assert abs(o[2] - outs[0][2]) <= 1e-13 * abs(outs[0][2])
