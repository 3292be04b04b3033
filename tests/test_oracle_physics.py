"""Pins of the oracle against facts that the physics and the mathematics fix.

* The a = 0, l = 2 Schwarzschild quasinormal ringdown (Sec. 3.2 evolution,
  Eq. (1) at a = 0): the late signal of the 801 x 33 pulse run, seen at
  r* = 20M, is a damped sinusoid whose complex frequency approaches the
  textbook fundamental mode omega M = 0.37367 - 0.08896 i (Leaver 1985;
  Chandrasekhar & Detweiler 1975) at second order in the grid spacing.
* The synthetic source (it stands in for T of Eq. (1)): the smeared particle
  carries exactly the amplitude A e^{-i m phi~_p} (its Gaussians are
  normalised, so their sums over the grid are quadratures of unit integrals,
  exact to rounding for a width of two cells), it vanishes beyond the
  cutoff, and the forced response of the linear, time-invariant iteration
  to a circular orbit oscillates at the orbit's frequency m Omega.
* Time-symmetric initial data: Pi(0) = b d_r* Phi(0) makes d_t Phi = 0 at
  t = 0, so one iteration changes Phi by O(dt^2), not O(dt).
"""

import numpy as np
import pytest
from scipy.optimize import least_squares

from oracle import teuk_oracle as T
from paper_1001_3631_amd import workloads as W

QNM_L2 = 0.37367 - 0.08896j   # Schwarzschild l = 2, n = 0, in units of 1/M


def fit_damped_sinusoid(t, y, t0, t1):
    """Complex frequency omega_R - i gamma of y ~ A e^{-gamma t} cos(omega_R t + ph)
    on [t0, t1]: a two-pole linear prediction (Prony) for the start, then
    nonlinear least squares with residuals scaled by the decaying envelope so
    that late samples weigh as much as early ones."""
    sel = (t >= t0) & (t <= t1)
    tt, yy = t[sel], y[sel]
    c = np.linalg.lstsq(np.column_stack([yy[1:-1], yy[:-2]]), yy[2:], rcond=None)[0]
    s = np.log(np.roots([1.0, -c[0], -c[1]]).astype(complex)) / (tt[1] - tt[0])
    s0 = s[np.argmax(s.imag)]
    amp = np.max(np.abs(yy))

    def res(v):
        A, ph, om, ga = v
        model = A * np.exp(-ga * (tt - t0)) * np.cos(om * (tt - t0) + ph)
        return (model - yy) * np.exp(-s0.real * (tt - t0)) / amp

    best = None
    for ph in np.linspace(0.0, 2.0 * np.pi, 8, endpoint=False):
        r = least_squares(res, [amp, ph, s0.imag, -s0.real], x_scale=[amp, 1.0, 0.1, 0.01],
                          xtol=1e-15, ftol=1e-15)
        if best is None or r.cost < best.cost:
            best = r
    return best.x[2] - 1j * best.x[3]


def ringdown_frequency(level):
    """Config 1 (a = 0, s = -2, m = 2, pulse at 50M of width 4M) refined
    `level` times (h_r, h_theta and dt halved each time), observed at
    r* = 20M on the equator; fitted on t in [120, 200]M, after the overtones
    have decayed and before any wall reflection returns."""
    base = W.SCHWARZSCHILD_PULSE
    k = 2 ** level
    grid = dict(base["grid"], nr=800 * k + 1, nth=32 * k + 1, rs_extract=20.0)
    g = T.Grid(**grid)
    n = int(round(200.0 / g.dt))
    p, q = T.initial_pulse(g, **base["pulse"])
    _, _, w = T.evolve(g, p, q, n)
    t = g.dt * np.arange(1, n + 1)
    y = w[:, g.nth // 2]
    assert np.all(y.imag == 0.0)        # a = 0: the operator and the data are real
    return fit_damped_sinusoid(t, y.real, 120.0, 200.0)


@pytest.mark.slow
def test_schwarzschild_l2_quasinormal_ringdown():
    w0 = ringdown_frequency(0)
    w1 = ringdown_frequency(1)
    e0, e1 = abs(w0 - QNM_L2) / abs(QNM_L2), abs(w1 - QNM_L2) / abs(QNM_L2)
    rich = (4.0 * w1 - w0) / 3.0       # second-order Richardson extrapolation
    print("801x33", w0, e0, "1601x65", w1, e1, "extrapolated", rich)
    assert e0 <= 0.01, (w0, e0)
    assert e1 <= e0 / 3.0, (e0, e1)      # second order: about 4x per refinement
    assert abs(rich - QNM_L2) / abs(QNM_L2) <= 1e-3, rich


# ---------------------------------------------------------------------------
# Synthetic source
# ---------------------------------------------------------------------------

def _source_grid(a=0.6, m=2):
    return T.Grid(M=1.0, a=a, s=-2, m=m, nr=400, nth=61, rs_min=-20.0, rs_max=80.0, cfl=0.5, ko_eps=0.5)


@pytest.mark.parametrize("m,phase,rs_p,th_p", [(2, 0.7, 12.3, 0.5 * np.pi), (3, -2.1, 20.04, 1.2),
                                               (1, 4.0, 5.5, 1.9)])
def test_source_carries_its_amplitude(m, phase, rs_p, th_p):
    """Sum over the grid of F h_r h_theta = A e^{-i m phi~_p}: each Gaussian is
    normalised to unit integral, and a uniform sum of a Gaussian two cells
    wide is its integral to within 2 e^{-8 pi^2} (Poisson summation), less
    the tails beyond the 8-sigma cutoff (erfc(8/sqrt 2) ~ 1e-15)."""
    g = _source_grid(m=m)
    orbit = {"rs": np.array([rs_p]), "th": np.array([th_p]), "phi": np.array([phase])}
    A = 1.7
    src = T.Source(g, orbit, amplitude=A)
    for rs in (g.rs, g.rs_half):
        F = src.field(0, rs, g.th)
        total = np.sum(F) * g.hr * g.hth
        assert abs(total - A * np.exp(-1j * m * phase)) <= 1e-13 * A, total


def test_source_cutoff():
    g = _source_grid()
    rs_p, th_p = 30.0 + 0.3 * g.hr, 1.4
    orbit = {"rs": np.array([rs_p]), "th": np.array([th_p]), "phi": np.array([0.0])}
    src = T.Source(g, orbit)
    F = src.field(0, g.rs, g.th)
    dr = np.abs(g.rs - rs_p)[None, :] / src.sr
    dth = np.abs(g.th - th_p)[:, None] / src.sth
    inside = (dr <= 8.0) & (dth <= 8.0)
    assert np.all(F[~inside] == 0.0)
    assert np.all(F[inside] != 0.0)
    # two cells wide in each direction, as configured
    assert src.sr == 2.0 * g.hr and src.sth == 2.0 * g.hth


def test_forced_response_oscillates_at_the_orbit_frequency():
    """From zero data a circular orbit drives the linear, time-invariant
    iteration with e^{-i m Omega t}; once the switch-on transient has rung
    down, the waveform advances in phase by -m Omega dt per iteration with a
    constant modulus.  The walls are far enough away that no reflection
    reaches the observer (r* = 30M) before t = 300M."""
    g = T.Grid(M=1.0, a=0.5, s=-2, m=2, nr=611, nth=21, rs_min=-130.0, rs_max=175.0, cfl=0.5,
               rs_extract=30.0, ko_eps=0.5)
    n = int(300.0 / g.dt)
    orbit = T.circular_orbit(g.M, g.a, 10.0, g.dt, n)
    src = T.Source(g, orbit)
    z = np.zeros((g.nth, g.nr), np.complex128)
    _, _, w = T.evolve(g, z, z, n, src)
    seg = w[int(200.0 / g.dt):, g.nth // 2]
    adv = np.angle(seg[1:] / seg[:-1])
    expect = -g.m * orbit["Omega"] * g.dt
    print("phase advance", np.median(adv), "expected", expect)
    assert abs(np.median(adv) - expect) <= 1e-3 * abs(expect)
    amp = np.abs(seg)
    assert np.std(amp) / np.mean(amp) < 0.01


# ---------------------------------------------------------------------------
# Initial data
# ---------------------------------------------------------------------------

def _first_step_change(level, pi_sign):
    k = 2 ** level
    g = T.Grid(M=1.0, a=0.7, s=-2, m=2, nr=60 * k + 1, nth=12 * k + 1, rs_min=-10.0, rs_max=50.0,
               cfl=0.5, ko_eps=0.5)
    p, q = T.initial_pulse(g, 20.0, 3.0)
    p1, _ = T.step(g, p, pi_sign * q, 0)
    return np.sqrt(np.mean(np.abs(p1 - p) ** 2)) / np.sqrt(np.mean(np.abs(p) ** 2))


def test_initial_data_is_time_symmetric():
    """With Pi(0) = b d_r* Phi(0) the first iteration moves Phi by O(dt^2): the
    change drops about 4x when h_r, h_theta and dt are halved.  With the sign
    of Pi(0) flipped (d_t Phi = -2 b d_r* Phi) it is O(dt) and drops 2x, which
    shows that the check can tell the two apart."""
    d = [_first_step_change(L, 1.0) for L in range(3)]
    r1, r2 = d[0] / d[1], d[1] / d[2]
    assert r1 > 3.5 and r2 > 3.5, d
    f = [_first_step_change(L, -1.0) for L in range(3)]
    assert 1.8 < f[1] / f[2] < 2.2, f
    assert d[2] < 0.05 * f[2]
