"""Stability of the literal Lax-Wendroff scheme and of the dissipation reading.

The paper asserts stable evolutions with the two-step Lax-Wendroff scheme
(Sec. 3.2) without giving dt.  With dt = cfl min(h_r, r(r*_min) h_theta) the
angular term w Ang[Phi] is integrated by the scheme's midpoint rule, whose
amplification for an oscillation of frequency omega is
|1 + i z - z^2/2| = sqrt(1 + z^4/4) > 1, z = omega dt.  The stiffest mode sits
on the row next to a pole where (m + s cos)^2/sin^2 ~ (m -+ s)^2/h^2.

* frozen-coefficient analysis of r-smooth modes (which the radial
  Lax-Wendroff dissipation does not touch), with the physical c_t and C_0
  terms removed so that only the numerical mode is measured: the literal
  scheme grows, a fourth-difference theta dissipation of strength 0.5 makes
  it neutral for every configured (a, m, grid, cfl);
* the literal config-1 run blows up on the theta = pi pole row within its
  2000 steps; with the dissipation it does not.
"""

import numpy as np
import pytest

from oracle import teuk_oracle as T
from paper_1001_3631_amd import workloads as W


def assemble_d4(nth, even):
    """Fourth theta-difference on the interior rows 1..nth-2 as a matrix over
    all nth rows, written entry by entry: stencil (1, -4, 6, -4, 1), and a
    ghost row beyond a pole reflected onto the row next to it with the sign of
    the pole condition (+ even |m|, where d_theta u = 0; - odd |m|, where
    u = 0)."""
    n2 = nth - 2
    sig = 1.0 if even else -1.0
    D4 = np.zeros((n2, nth))
    for k, j in enumerate(range(1, nth - 1)):
        for d, c in zip(range(-2, 3), (1, -4, 6, -4, 1)):
            jj = j + d
            if jj == -1:
                D4[k, 1] += sig * c
            elif jj == nth:
                D4[k, nth - 2] += sig * c
            else:
                D4[k, jj] += c
    return D4


def frozen_numerical_rho(M, a, s, m, nth, dt, eps, xs):
    """max over radii of the spectral radius of one iteration restricted to
    r-smooth modes, with c_t = C_0 = 0 (pure numerical amplification)."""
    th = np.arange(nth) * np.pi / (nth - 1)
    h = th[1]
    even = abs(m) % 2 == 0
    J = np.arange(1, nth - 1)
    n2 = nth - 2
    cot = np.cos(th[J]) / np.sin(th[J])
    V = T.angular_potential(th[J], s, m)
    Ang = np.zeros((n2, nth))
    for k, j in enumerate(J):
        Ang[k, j + 1] += 1 / h ** 2 + cot[k] / (2 * h)
        Ang[k, j] += -2 / h ** 2 - V[k]
        Ang[k, j - 1] += 1 / h ** 2 - cot[k] / (2 * h)
    B = np.zeros((nth, n2))
    B[J, np.arange(n2)] = 1.0
    if even:
        B[0, 0], B[0, 1], B[-1, -1], B[-1, -2] = 4 / 3, -1 / 3, 4 / 3, -1 / 3
    D4 = assemble_d4(nth, even)
    Sel = np.zeros((n2, nth))
    Sel[np.arange(n2), J] = 1.0
    Z = np.zeros((n2, nth))
    out = 0.0
    for x in xs:
        w = T.coefficients(x, th[J], M, a, s, m)["w"]
        Hpi = np.hstack([0.5 * dt * np.diag(w) @ Ang, Sel])
        Hphi = np.hstack([Sel, 0.5 * dt * Sel])
        hphi, hpi = B @ Hphi, B @ Hpi
        Uphi = np.hstack([Sel, Z]) + dt * (Sel @ hpi) - eps / 16 * np.hstack([D4, Z])
        Upi = np.hstack([Z, Sel]) + dt * (np.diag(w) @ Ang @ hphi) - eps / 16 * np.hstack([Z, D4])
        G = np.vstack([B @ Uphi, B @ Upi])
        out = max(out, np.max(np.abs(np.linalg.eigvals(G))))
    return out


def _cases():
    cases = []
    for cfg in (W.SCHWARZSCHILD_PULSE, W.KERR_EMRI, W.ADJOINT):
        g = cfg["grid"]
        cases.append((cfg["name"], g["a"], g["m"], g["nth"], g["nr"], g["rs_min"], g["rs_max"], g["cfl"]))
    # batched instances: the corners of the (a, m, level) draw
    for a in (0.0, 0.99):
        for m in (1, 2, 3, 4):
            for lvl in (0, 2):
                cases.append((f"batch a={a} m={m} lvl={lvl}", a, m, 32 * 2 ** lvl, 1600 * 2 ** lvl,
                              -200.0, 600.0, 0.25))
    return cases


def _dt(a, nr, nth, rs_min, rs_max, cfl):
    rp, _ = T.horizons(1.0, a)
    r0 = rp + T.x_of_tortoise(rs_min, 1.0, a)[0]
    return cfl * min((rs_max - rs_min) / (nr - 1), r0 * np.pi / (nth - 1))


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_dissipation_neutralises_the_stiff_pole_mode(case):
    name, a, m, nth, nr, rs_min, rs_max, cfl = case
    dt = _dt(a, nr, nth, rs_min, rs_max, cfl)
    xs = np.geomspace(0.05, 60.0, 25)
    rho = frozen_numerical_rho(1.0, a, -2, m, nth, dt, W.KO_EPS, xs)
    assert rho <= 1.0 + 2e-6, (name, rho)


def test_literal_scheme_is_unstable_at_config1_dt():
    g = W.SCHWARZSCHILD_PULSE["grid"]
    dt = _dt(g["a"], g["nr"], g["nth"], g["rs_min"], g["rs_max"], g["cfl"])
    xs = np.geomspace(0.05, 60.0, 25)
    assert frozen_numerical_rho(1.0, 0.0, -2, 2, g["nth"], dt, 0.0, xs) > 1.04
    # and at cfl 0.5 the m = 4, a = 0 mode is beyond what any eps <= 1 can hold,
    # which is why the batched instances run at cfl 0.25
    dt4 = _dt(0.0, 3200, 64, -200.0, 600.0, 0.5)
    assert frozen_numerical_rho(1.0, 0.0, -2, 4, 64, dt4, 1.0, xs) > 1.05


@pytest.mark.slow
def test_literal_config1_run_blows_up_and_dissipated_run_does_not():
    cfg = W.SCHWARZSCHILD_PULSE
    res = {}
    for eps in (0.0, W.KO_EPS):
        g = T.Grid(**dict(cfg["grid"], ko_eps=eps))
        p, q = T.initial_pulse(g, **cfg["pulse"])
        p, q, _ = T.evolve(g, p, q, cfg["steps"])
        res[eps] = np.max(np.abs(p[-2]))      # row next to theta = pi
    assert res[0.0] > 1e6 * res[W.KO_EPS], res
    assert np.isfinite(res[W.KO_EPS]) and res[W.KO_EPS] < 1e6


@pytest.mark.parametrize("m", [1, 2])
def test_dissipation_term_is_the_assembled_fourth_difference(m):
    """The oracle's dissipation term (ghost rows reflected by the pole
    condition) equals the fourth-difference matrix assembled entry by entry
    above, on a random state, for even and odd |m|."""
    g = T.Grid(M=1.0, a=0.5, s=-2, m=m, nr=11, nth=13, rs_min=-10.0, rs_max=20.0, ko_eps=0.5)
    rng = np.random.default_rng(m)
    u = rng.standard_normal((g.nth, g.nr)) + 1j * rng.standard_normal((g.nth, g.nr))
    ref = assemble_d4(g.nth, g.even) @ u
    np.testing.assert_allclose(T._ko_delta4(g, u), ref, rtol=0, atol=1e-13 * np.max(np.abs(ref)))


def test_weaker_dissipation_leaves_a_configured_grid_unstable():
    """eps = 0.5 is the smallest of {0.02, 0.05, 0.1, 0.2, 0.3, 0.5} that holds
    every configured grid: the next smaller value, 0.3, leaves at least one
    of them growing."""
    xs = np.geomspace(0.05, 60.0, 25)
    worst = 0.0
    for name, a, m, nth, nr, rs_min, rs_max, cfl in _cases():
        dt = _dt(a, nr, nth, rs_min, rs_max, cfl)
        worst = max(worst, frozen_numerical_rho(1.0, a, -2, m, nth, dt, 0.3, xs))
    assert worst > 1.0 + 2e-6, worst


def _late_growth_rate(g, nu, T_end=20.0, seed=0):
    """Growth rate per unit time of a seeded random state over the second
    half of [0, T_end], with dt set to nu h_r / max b (radial Courant number
    nu)."""
    bmax = max(np.max(g.node["b"]), np.max(g.half["b"]))
    g.dt = nu * g.hr / bmax
    rng = np.random.default_rng(seed)
    p = rng.standard_normal((g.nth, g.nr)) + 1j * rng.standard_normal((g.nth, g.nr))
    q = rng.standard_normal((g.nth, g.nr)) + 1j * rng.standard_normal((g.nth, g.nr))
    T.apply_bc(g, p, q)
    n = int(round(T_end / g.dt))
    norms = []
    for k in range(n):
        p, q = T.step(g, p, q, k)
        norms.append(np.sqrt(np.sum(np.abs(p) ** 2) + np.sum(np.abs(q) ** 2)))
    return np.log(norms[-1] / norms[n // 2]) / (g.dt * (n - 1 - n // 2))


@pytest.mark.parametrize("eps", [0.0, 0.5, 1.0])
def test_radial_courant_limit(eps):
    """CFL limit of the iteration.  For the checkerboard mode in r* (k h = pi)
    the two-step Lax-Wendroff factor is 1 - 2 nu^2 (nu = b dt / h_r); the
    dissipation adds -eps mu/16, mu the largest eigenvalue of the assembled
    fourth difference (at most 16).  So |1 - 2 nu^2 - eps mu/16| <= 1 needs
    nu <= sqrt(1 - eps mu/32): 1 for the literal scheme, 0.87 at eps = 0.5.
    Below that limit a random state grows no faster than the equation itself
    lets it; above it, the state blows up."""
    g = T.Grid(M=1.0, a=0.0, s=-2, m=2, nr=201, nth=17, rs_min=-5.0, rs_max=15.0, ko_eps=eps)
    mu = np.max(np.linalg.eigvalsh(assemble_d4(g.nth, g.even)[:, 1:-1]))
    assert 15.0 < mu <= 16.0
    lim = np.sqrt(1.0 - eps * mu / 32.0)
    slow = _late_growth_rate(g, 0.5)
    below = _late_growth_rate(g, lim - 0.03)
    above = _late_growth_rate(g, lim + 0.03)
    print("eps", eps, "limit", lim, "rates (0.5, below, above)", slow, below, above)
    assert abs(slow) < 0.05 and below < 0.05, (slow, below)
    assert above > 0.3, above
    # every configured grid runs well inside the limit of the scheme it uses
    for cfg in (W.SCHWARZSCHILD_PULSE, W.KERR_EMRI, W.ADJOINT):
        gc = cfg["grid"]
        cg = T.Grid(**dict(gc, nr=41, nth=gc["nth"]))
        nu = gc["cfl"] * max(np.max(cg.node["b"]), np.max(cg.half["b"]))
        assert nu < np.sqrt(1.0 - gc["ko_eps"] * 16.0 / 32.0) - 0.2
