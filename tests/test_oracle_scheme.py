"""Pins for the oracle's discrete scheme (Sec. 3.2, Eqs. (lw1)-(lw2) and the
boundary conditions), against facts that hold independently of it:

* exact linearity / superposition of the iteration (it is linear in u and F);
* boundary conditions hold after every step;
* the adjoint sweep is the transpose: dot-product identity, and equality with
  the conjugate transpose of the step matrix assembled column by column;
* the loss is exactly quadratic in (u0, A), so central differences of it equal
  the adjoint gradient up to rounding;
* second-order self-convergence under simultaneous refinement of h_r*,
  h_theta and dt, with and without the theta dissipation;
* a manufactured solution is reproduced to second order.
"""

import numpy as np
import pytest

from oracle import teuk_oracle as T


def small_grid(a=0.6, m=2, nr=23, nth=11, ko=0.5, s=-2):
    return T.Grid(M=1.0, a=a, s=s, m=m, nr=nr, nth=nth, rs_min=-20.0, rs_max=40.0,
                  cfl=0.5, rs_extract=10.0, ko_eps=ko)


def rand_state(g, rng):
    z = lambda: rng.standard_normal((g.nth, g.nr)) + 1j * rng.standard_normal((g.nth, g.nr))
    return z(), z()


def vdot(x, y):
    return np.vdot(x[0], y[0]) + np.vdot(x[1], y[1])


@pytest.mark.parametrize("m,a,ko", [(2, 0.6, 0.5), (1, 0.9, 0.5), (3, 0.0, 0.0), (2, 0.0, 0.5), (4, 0.99, 0.5)])
def test_linearity_and_bc(m, a, ko):
    g = small_grid(a=a, m=m, ko=ko)
    rng = np.random.default_rng(1)
    u, v = rand_state(g, rng), rand_state(g, rng)
    al, be = 0.3 - 1.7j, 2.1 + 0.4j
    lhs = T.step(g, al * u[0] + be * v[0], al * u[1] + be * v[1], 0)
    su, sv = T.step(g, *u, 0), T.step(g, *v, 0)
    for k in range(2):
        ref = al * su[k] + be * sv[k]
        assert np.max(np.abs(lhs[k] - ref)) <= 1e-13 * np.max(np.abs(ref))
    for f in lhs:
        assert np.all(f[:, 0] == 0) and np.all(f[:, -1] == 0)
        if g.even:
            np.testing.assert_allclose(f[0, 1:-1], (4 * f[1, 1:-1] - f[2, 1:-1]) / 3, rtol=0, atol=1e-14 * np.abs(f).max())
        else:
            assert np.all(f[0] == 0) and np.all(f[-1] == 0)


@pytest.mark.parametrize("m,a,ko", [(2, 0.6, 0.5), (1, 0.9, 0.5), (3, 0.3, 0.0), (2, 0.0, 0.0)])
def test_adjoint_dot_product(m, a, ko):
    g = small_grid(a=a, m=m, ko=ko)
    rng = np.random.default_rng(2)
    x, y = rand_state(g, rng), rand_state(g, rng)
    Gx = T.step(g, *x, 0)
    GTy = T.adjoint_step(g, *y, 0)[:2]
    lhs, rhs = vdot(Gx, y), vdot(x, GTy)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("m,a,ko", [(2, 0.6, 0.5), (1, 0.8, 0.5), (2, 0.0, 0.0)])
def test_adjoint_equals_bruteforce_transpose(m, a, ko):
    """Assemble G column by column on a 9x7 grid; G^H must equal the
    matrix-free adjoint applied to unit vectors."""
    g = small_grid(a=a, m=m, nr=9, nth=7, ko=ko)
    G = T.assemble_step_matrix(g)
    npt = g.nth * g.nr
    GH = np.zeros_like(G)
    for k in range(2 * npt):
        e = np.zeros(2 * npt, dtype=np.complex128)
        e[k] = 1.0
        p, q, _ = T.adjoint_step(g, e[:npt].reshape(g.nth, g.nr), e[npt:].reshape(g.nth, g.nr), 0)
        GH[:, k] = np.concatenate([p.ravel(), q.ravel()])
    assert np.max(np.abs(GH - G.conj().T)) <= 1e-14 * np.max(np.abs(G))


def _config4_like(nsteps=25):
    g = T.Grid(M=1.0, a=0.7, s=-2, m=2, nr=41, nth=13, rs_min=-20.0, rs_max=40.0,
               cfl=0.5, rs_extract=12.0, ko_eps=0.5)
    orbit = T.circular_orbit(g.M, g.a, 10.0, g.dt, nsteps)
    src = T.Source(g, orbit, amplitude=1.0)
    return g, src


def test_gradient_matches_central_differences():
    """L(u0, A) = sum |w - y|^2 is exactly quadratic, so central differences
    equal the directional derivative up to rounding."""
    nsteps = 25
    g, src = _config4_like(nsteps)
    rng = np.random.default_rng(4)
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    A0 = 1.0
    y = 0.01 * (rng.standard_normal((nsteps, g.nth)) + 1j * rng.standard_normal((nsteps, g.nth)))

    def loss(p, q, A):
        w = T.evolve(g, p, q, nsteps, src, amplitude=A)[2]
        return T.waveform_loss(w, y)

    L0, gw = loss(phi0, pi0, A0)
    gphi, gpi, gA = T.adjoint_evolve(g, gw, nsteps, src)
    for trial in range(6):
        vp, vq = rand_state(g, rng)
        vA = rng.standard_normal()
        nrm = np.sqrt(np.sum(np.abs(vp) ** 2) + np.sum(np.abs(vq) ** 2) + vA ** 2)
        vp, vq, vA = vp / nrm, vq / nrm, vA / nrm
        h = 1e-3
        Lp = loss(phi0 + h * vp, pi0 + h * vq, A0 + h * vA)[0]
        Lm = loss(phi0 - h * vp, pi0 - h * vq, A0 - h * vA)[0]
        fd = (Lp - Lm) / (2 * h)
        ad = np.real(np.vdot(gphi, vp) + np.vdot(gpi, vq)) + gA * vA
        assert abs(fd - ad) <= 1e-7 * max(abs(ad), 1e-3 * L0), (fd, ad)


def test_source_amplitude_is_linear():
    nsteps = 20
    g, src = _config4_like(nsteps)
    z = np.zeros((g.nth, g.nr), np.complex128)
    w1 = T.evolve(g, z, z, nsteps, src, amplitude=1.0)[2]
    w3 = T.evolve(g, z, z, nsteps, src, amplitude=3.0)[2]
    assert np.max(np.abs(w3 - 3.0 * w1)) <= 1e-14 * np.max(np.abs(w3))
    assert np.max(np.abs(w1)) > 0


def test_state_loss_gradient_through_adjoint():
    """A loss on intermediate states: L = sum_{n in S} |Phi^n|^2 over the grid.
    The adjoint with state_grad injection agrees with central differences."""
    nsteps = 12
    g, src = _config4_like(nsteps)
    phi0, pi0 = T.initial_pulse(g, 15.0, 4.0)
    S = [4, 9, 12]

    def loss(p, q):
        snaps = {k: None for k in S}
        pN, qN, _ = T.evolve(g, p, q, nsteps, snapshots=snaps)
        return sum(np.sum(np.abs(snaps[k][0]) ** 2) for k in S), snaps

    L0, snaps = loss(phi0, pi0)
    z = np.zeros_like(phi0)
    sg = lambda n: (2 * snaps[n][0], z) if n in S and n < nsteps else None
    gphi, gpi, _ = T.adjoint_evolve(g, np.zeros((nsteps, g.nth)), nsteps, None,
                                   lam_phi_N=2 * snaps[nsteps][0], state_grad=sg)
    rng = np.random.default_rng(9)
    vp, vq = rand_state(g, rng)
    h = 1e-4
    fd = (loss(phi0 + h * vp, pi0 + h * vq)[0] - loss(phi0 - h * vp, pi0 - h * vq)[0]) / (2 * h)
    ad = np.real(np.vdot(gphi, vp) + np.vdot(gpi, vq))
    assert abs(fd - ad) <= 1e-8 * abs(ad)


def _run_to_time(a, m, level, ko, T_end=12.0):
    nr = 60 * 2 ** level + 1
    nth = 8 * 2 ** level + 1
    g = T.Grid(M=1.0, a=a, s=-2, m=m, nr=nr, nth=nth, rs_min=-15.0, rs_max=45.0,
               cfl=0.5, ko_eps=ko)
    # fix dt across levels: the coarse dt halved per level (same ratio dt/h)
    g0 = T.Grid(M=1.0, a=a, s=-2, m=m, nr=61, nth=9, rs_min=-15.0, rs_max=45.0, cfl=0.5)
    g.dt = g0.dt / 2 ** level
    nsteps = int(round(T_end / g.dt))
    assert abs(nsteps * g.dt - T_end) < 1e-9
    phi, pi = T.initial_pulse(g, 10.0, 3.0)
    phi, pi, _ = T.evolve(g, phi, pi, nsteps)
    return g, phi


@pytest.mark.slow
@pytest.mark.parametrize("ko", [0.0, 0.5])
def test_second_order_self_convergence(ko):
    a, m = 0.5, 2
    # pick T so that it is a whole number of coarse steps
    g0 = T.Grid(M=1.0, a=a, s=-2, m=m, nr=61, nth=9, rs_min=-15.0, rs_max=45.0, cfl=0.5)
    T_end = 40 * g0.dt
    sols = [_run_to_time(a, m, L, ko, T_end) for L in range(3)]
    # common points: coarse nodes
    f0 = sols[0][1]
    f1 = sols[1][1][::2, ::2]
    f2 = sols[2][1][::4, ::4]
    e01 = np.sqrt(np.sum(np.abs(f0 - f1) ** 2))
    e12 = np.sqrt(np.sum(np.abs(f1 - f2) ** 2))
    order = np.log2(e01 / e12)
    print('self-convergence order', order)
    assert 1.85 <= order <= 2.3, order


class _Manufactured:
    """Forcing F for the exact solution Phi = e^{-i om t} g(r*) P(theta) of the
    continuous system; F = Pi_t - b Pi_r* + c_t Pi - m_r Phi_r* - C_0 Phi - w Ang[Phi]
    with Pi = Phi_t + b Phi_r*, derivatives of g and P analytic, of b by
    centred differences in r* at h = 1e-4 (error far below the scheme's)."""

    def __init__(self, g, om=0.4, c=10.0, sig=3.0):
        self.g, self.om, self.c, self.sig = g, om, c, sig
        self.P = lambda th: T.angular_profile(th, g.s, g.m)

    def _fields(self, t, rs, th):
        g, om, c, sig = self.g, self.om, self.c, self.sig
        G = np.exp(-(rs - c) ** 2 / (2 * sig * sig))
        G1 = -(rs - c) / sig ** 2 * G
        G2 = ((rs - c) ** 2 / sig ** 4 - 1 / sig ** 2) * G
        P = self.P(th)
        hth = 1e-5
        P1 = (self.P(th + hth) - self.P(th - hth)) / (2 * hth)
        P2 = (self.P(th + hth) - 2 * P + self.P(th - hth)) / hth ** 2
        x = T.x_of_tortoise(rs, g.M, g.a)
        cf = T.coefficients(x[None, :], th[:, None], g.M, g.a, g.s, g.m)
        xp = T.x_of_tortoise(rs + 1e-4, g.M, g.a)
        xm = T.x_of_tortoise(rs - 1e-4, g.M, g.a)
        b_rs = (T.coefficients(xp[None, :], th[:, None], g.M, g.a, g.s, g.m)["b"]
                - T.coefficients(xm[None, :], th[:, None], g.M, g.a, g.s, g.m)["b"]) / 2e-4
        e = np.exp(-1j * om * t)
        Phi = e * P[:, None] * G[None, :]
        Phi_t = -1j * om * Phi
        Phi_r = e * P[:, None] * G1[None, :]
        Phi_rr = e * P[:, None] * G2[None, :]
        Phi_tr = -1j * om * Phi_r
        b = cf["b"]
        Pi = Phi_t + b * Phi_r
        Pi_t = -1j * om * Pi
        Pi_r = Phi_tr + b_rs * Phi_r + b * Phi_rr
        V = T.angular_potential(th, g.s, g.m)
        with np.errstate(divide="ignore", invalid="ignore"):   # pole rows are not used
                ang = e * (P2 + np.cos(th) / np.sin(th) * P1 - V * P)[:, None] * G[None, :]
        F = Pi_t - b * Pi_r + cf["ct"] * Pi - cf["mr"] * Phi_r - cf["C0"] * Phi - cf["w"] * ang
        return Phi, Pi, F

    def field(self, k, rs, th, amplitude=None):
        t = k * 0.5 * self.g.dt
        th_safe = np.clip(th, 1e-3, np.pi - 1e-3)
        F = self._fields(t, rs, th_safe)[2]
        return F


@pytest.mark.slow
def test_manufactured_solution_second_order():
    """a = 0.5, m = 1 (odd: Dirichlet at the poles, where the manufactured
    profile sin(1+cos) vanishes).  Error vs the exact solution drops ~4x per
    refinement."""
    errs = []
    for L in range(3):
        nr, nth = 40 * 2 ** L + 1, 8 * 2 ** L + 1
        g = T.Grid(M=1.0, a=0.5, s=-2, m=1, nr=nr, nth=nth, rs_min=-10.0, rs_max=30.0,
                   cfl=0.5, ko_eps=0.5)
        g0 = T.Grid(M=1.0, a=0.5, s=-2, m=1, nr=41, nth=9, rs_min=-10.0, rs_max=30.0, cfl=0.5)
        g.dt = g0.dt / 2 ** L
        nsteps = 30 * 2 ** L
        man = _Manufactured(g)
        phi, pi, _ = man._fields(0.0, g.rs, g.th)
        phi, pi = phi.copy(), pi.copy()
        T.apply_bc(g, phi, pi)
        phi, pi, _ = T.evolve(g, phi, pi, nsteps, source=man)
        ex = man._fields(nsteps * g.dt, g.rs, g.th)[0]
        inner = (slice(1, -1), slice(4 * 2 ** L, -4 * 2 ** L))   # away from the radial walls
        errs.append(np.sqrt(np.mean(np.abs(phi[inner][:, ::2 ** L] - ex[inner][:, ::2 ** L]) ** 2)))
    o1, o2 = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    print('MMS orders', o1, o2)
    assert o1 > 1.7 and o2 > 1.8, errs
