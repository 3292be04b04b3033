"""Pins of the oracle's radiated fluxes (energy, linear momentum, z angular
momentum carried off by the waves, Sec. 3.2 closing paragraph; standard
psi_4 formulas) against facts that do not depend on how they are coded:

* an analytic outgoing mode, w = A e^{-i w t} P(theta): H, K and hence
  dE/dt, dJ_z/dt and E(t) have closed forms in t (P's angular integrals in
  closed form too); the trapezoidal rules converge to them at second order;
* the mode sums equal brute-force quadratures over the sphere of the
  definitions (|H|^2, cos |H|^2, sin e^{i phi} |H|^2, conj(H) d_phi K) with
  the field rebuilt on a phi grid; this fixes every factor, conjugation and
  the (m, m+1) pairing of the transverse momentum;
* symmetry: a single m radiates no transverse momentum, and a field whose
  |H|^2 is symmetric about the equator none along z.
"""

import numpy as np
import pytest

from oracle import teuk_oracle as T


def _modes(nth, nt, ms, seed):
    """Smooth random waveforms: a few damped oscillations per mode with
    random angular profiles built from low harmonics in theta."""
    rng = np.random.default_rng(seed)
    th = np.arange(nth) * np.pi / (nth - 1)
    t = np.arange(nt)
    out = []
    for m in ms:
        prof = sum((rng.standard_normal() + 1j * rng.standard_normal()) * np.sin(th) ** k * np.cos(th) ** l
                   for k in range(3) for l in range(2))
        om = 0.2 + 0.3 * rng.random()
        out.append(np.exp(-1j * om * 0.05 * t - 0.001 * t)[:, None] * prof[None, :])
    return out


def test_analytic_outgoing_mode_converges_to_closed_form():
    """w = A e^{-i om t} (1 + cos)^2: with H = (iA/om)(e^{-i om t} - 1) P and
    K = (iA/om)((e^{-i om t} - 1)/(-i om) - t) P, int P^2 sin = 32/5 and
    int P^2 cos sin = 64/15: dE/dt = (16/5)|h|^2, dP_z/dt = (32/15)|h|^2 and
    dJ_z/dt = (m/2)(32/5) Im(conj(h) k) with h, k the time factors."""
    A, om, m = 0.7 - 0.4j, 0.37, 2
    tend = 30.0
    errs = []
    for lvl in range(3):
        nth = 64 * 2 ** lvl + 1
        nt = 600 * 2 ** lvl + 1
        dt = tend / (nt - 1)
        th = np.arange(nth) * np.pi / (nth - 1)
        t = np.arange(nt) * dt
        P = (1 + np.cos(th)) ** 2
        w = A * np.exp(-1j * om * t)[:, None] * P[None, :]
        out = T.radiated_flux([m], [w], dt, th[1])
        h = (1j * A / om) * (np.exp(-1j * om * t) - 1)
        k = (1j * A / om) * ((np.exp(-1j * om * t) - 1) / (-1j * om) - t)
        dE = 0.5 * np.abs(h) ** 2 * 32 / 5
        dJ = 0.5 * m * np.imag(np.conj(h) * k) * 32 / 5
        dPz = 0.5 * np.abs(h) ** 2 * 64 / 15
        E = 0.5 * 32 / 5 * (np.abs(A) ** 2 / om ** 2) * (2 * t - 2 * np.sin(om * t) / om)
        errs.append(max(np.max(np.abs(out[:, 0] - dE)) / np.max(dE), np.max(np.abs(out[:, 4] - dJ)) / np.max(np.abs(dJ)),
                        np.max(np.abs(out[:, 5] - E)) / np.max(E), np.max(np.abs(out[:, 3] - dPz)) / np.max(dPz)))
        assert np.all(out[:, 1:3] == 0.0)      # a single m carries no transverse momentum
    print("closed-form errors per level", errs)
    assert errs[0] < 1e-3
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_mode_sums_equal_quadrature_over_the_sphere():
    ms = [1, 2, 3]
    nth, nt, dt = 41, 200, 0.05
    hth = np.pi / (nth - 1)
    waves = _modes(nth, nt, ms, seed=5)
    out = T.radiated_flux(ms, waves, dt, hth)
    # rebuild H and K on (t, theta, phi) and integrate the definitions
    nph = 64
    ph = np.arange(nph) * 2 * np.pi / nph

    def tint(f):
        o = np.zeros_like(f)
        o[1:] = np.cumsum(0.5 * dt * (f[1:] + f[:-1]), axis=0)
        return o

    H = sum(tint(w)[:, :, None] * np.exp(1j * m * ph)[None, None, :] for m, w in zip(ms, waves))
    dK = sum(1j * m * tint(tint(w))[:, :, None] * np.exp(1j * m * ph)[None, None, :] for m, w in zip(ms, waves))
    th = np.arange(nth) * hth
    wq = np.full(nth, hth)
    wq[0] = wq[-1] = 0.5 * hth
    dOm = (wq * np.sin(th))[None, :, None] * (2 * np.pi / nph)
    quad = lambda f: np.sum(f * dOm, axis=(1, 2)) / (4 * np.pi)
    H2 = np.abs(H) ** 2
    ref = [quad(H2), quad(np.sin(th)[None, :, None] * np.exp(1j * ph)[None, None, :] * H2),
           quad(np.cos(th)[None, :, None] * H2), -np.real(quad(np.conj(H) * dK))]
    for got, want in ((out[:, 0], ref[0]), (out[:, 1], ref[1].real), (out[:, 2], ref[1].imag),
                      (out[:, 3], ref[2]), (out[:, 4], ref[3])):
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(ref[0])), np.max(np.abs(got - want))
    assert np.max(np.abs(ref[1])) > 1e-3 * np.max(ref[0])     # the check has something to check


def test_symmetry_zeros():
    nth, nt, dt = 33, 100, 0.1
    hth = np.pi / (nth - 1)
    th = np.arange(nth) * hth
    t = np.arange(nt) * dt
    w = np.exp(-0.3j * t)[:, None] * np.sin(th)[None, :] ** 2     # |H|^2 symmetric about the equator
    out = T.radiated_flux([2], [w], dt, hth)
    assert np.all(out[:, 1] == 0.0) and np.all(out[:, 2] == 0.0)  # one m: no transverse momentum
    assert np.max(np.abs(out[:, 3])) <= 1e-14 * np.max(out[:, 0])
    two = T.radiated_flux([2, 4], [w, w], dt, hth)                # m and m + 2 do not pair either
    assert np.all(two[:, 1:3] == 0.0)
    np.testing.assert_allclose(two[:, 0], 2 * out[:, 0], rtol=1e-14)
