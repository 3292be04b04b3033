"""Pins of the oracle's orbit builder for the synthetic source: bound
equatorial Kerr geodesics parameterized by the relativistic anomaly chi,
r = p/(1 + e cos chi).  Each check compares against something the builder
does not compute itself: closed forms of the Schwarzschild and circular
limits, the normalization of the four-velocity, the turning points."""

import numpy as np
import pytest

from oracle import teuk_oracle as T


@pytest.mark.parametrize("p,e", [(8.0, 0.5), (9.0, 0.45), (12.0, 0.2), (14.0, 0.0)])
def test_schwarzschild_constants_closed_form(p, e):
    """a = 0: E^2 = ((p-2)^2 - 4e^2)/(p(p-3-e^2)), L^2 = p^2/(p-3-e^2),
    third root of R(r)/r at 2p/(p-4) (Cutler, Kennefick and Poisson 1994)."""
    E, L, r3 = T.equatorial_constants(0.0, p, e)
    assert abs(E - np.sqrt(((p - 2.0) ** 2 - 4.0 * e * e) / (p * (p - 3.0 - e * e)))) < 1e-14
    assert abs(L - p / np.sqrt(p - 3.0 - e * e)) < 1e-13
    assert abs(r3 - 2.0 * p / (p - 4.0)) < 1e-10


@pytest.mark.parametrize("p,e", [(8.0, 0.5), (9.0, 0.45), (13.0, 0.1)])
def test_schwarzschild_rates_closed_form(p, e):
    """a = 0: dt/dchi = p^2/((p-2-2e cos chi)(1+e cos chi)^2)
    sqrt(((p-2)^2-4e^2)/(p-6-2e cos chi)), dphi/dchi = sqrt(p/(p-6-2e cos chi))."""
    E, L, r3 = T.equatorial_constants(0.0, p, e)
    chi = np.linspace(0.0, 2.0 * np.pi, 37)
    vt, vphi, _ = T.equatorial_rates(0.0, p, e, E, L, r3, chi)
    c = np.cos(chi)
    ref_t = p * p / ((p - 2.0 - 2.0 * e * c) * (1.0 + e * c) ** 2) \
        * np.sqrt(((p - 2.0) ** 2 - 4.0 * e * e) / (p - 6.0 - 2.0 * e * c))
    ref_phi = np.sqrt(p / (p - 6.0 - 2.0 * e * c))
    np.testing.assert_allclose(vt, ref_t, rtol=1e-13)
    np.testing.assert_allclose(vphi, ref_phi, rtol=1e-13)


@pytest.mark.parametrize("a,r", [(0.0, 10.0), (0.6, 9.0), (0.9, 8.0), (0.95, 6.0)])
def test_circular_limit_bardeen_press_teukolsky(a, r):
    """e = 0: E = (1 - 2/r + a r^{-3/2})/sqrt(1 - 3/r + 2a r^{-3/2}),
    L = sqrt(r)(1 - 2a r^{-3/2} + a^2/r^2)/sqrt(1 - 3/r + 2a r^{-3/2}), and
    dphi/dt = 1/(r^{3/2} + a)."""
    E, L, r3 = T.equatorial_constants(a, r, 0.0)
    den = np.sqrt(1.0 - 3.0 / r + 2.0 * a / r ** 1.5)
    assert abs(E - (1.0 - 2.0 / r + a / r ** 1.5) / den) < 1e-13
    assert abs(L - np.sqrt(r) * (1.0 - 2.0 * a / r ** 1.5 + a * a / r ** 2) / den) < 1e-12
    vt, vphi, _ = T.equatorial_rates(a, r, 0.0, E, L, r3, np.array([0.3]))
    assert abs(vphi[0] / vt[0] - 1.0 / (r ** 1.5 + a)) < 1e-14 / r ** 1.5


def test_circular_limit_matches_circular_orbit():
    orb = T.eccentric_orbit(1.0, 0.7, 10.0, 0.0, 0.0, 0.0177, 200)
    ref = T.circular_orbit(1.0, 0.7, 10.0, 0.0177, 200)
    np.testing.assert_allclose(orb["rs"], ref["rs"], rtol=1e-14)
    np.testing.assert_allclose(orb["phi"], ref["phi"], rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("a,p,e", [(0.9, 10.0, 0.4), (0.95, 8.0, 0.5), (0.3, 14.0, 0.25)])
def test_kerr_four_velocity_is_normalized(a, p, e):
    """g_{mu nu} u^mu u^nu = -1 with the equatorial Kerr metric
    (g_tt = -(1 - 2/r), g_tphi = -2a/r, g_phiphi = r^2 + a^2 + 2a^2/r,
    g_rr = r^2/Delta) and u = (dt, dr, dphi)/dchi divided by dtau/dchi."""
    E, L, r3 = T.equatorial_constants(a, p, e)
    chi = np.linspace(0.0, 2.0 * np.pi, 41)
    vt, vphi, dtau = T.equatorial_rates(a, p, e, E, L, r3, chi)
    r = p / (1.0 + e * np.cos(chi))
    drdchi = p * e * np.sin(chi) / (1.0 + e * np.cos(chi)) ** 2
    ut, uph, ur = vt / dtau, vphi / dtau, drdchi / dtau
    delta = r * r - 2.0 * r + a * a
    norm = (-(1.0 - 2.0 / r) * ut * ut - 4.0 * a / r * ut * uph
            + (r * r + a * a + 2.0 * a * a / r) * uph * uph + r * r / delta * ur * ur)
    np.testing.assert_allclose(norm, -1.0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("a,p,e", [(0.9, 10.0, 0.4), (0.5, 8.0, 0.5)])
def test_orbit_turning_points_and_radial_period(a, p, e):
    """The sampled r stays in [p/(1+e), p/(1-e)], and r(t) repeats after the
    radial period T_r = integral of dt/dchi over one anomaly cycle."""
    from scipy.integrate import quad

    E, L, r3 = T.equatorial_constants(a, p, e)
    Tr = quad(lambda c: float(T.equatorial_rates(a, p, e, E, L, r3, c)[0]), 0.0, 2.0 * np.pi,
              epsabs=0.0, epsrel=2e-14, limit=200)[0]
    dt = Tr / 100.0          # one radial period = 200 samples
    orb = T.eccentric_orbit(1.0, a, p, e, 0.4, dt, 150)
    r = orb["r"]
    assert r.min() >= p / (1.0 + e) - 1e-12 and r.max() <= p / (1.0 - e) + 1e-12
    np.testing.assert_allclose(r[200:], r[:-200], rtol=1e-12)
    np.testing.assert_allclose(orb["chi"][200:] - orb["chi"][:-200], 2.0 * np.pi, rtol=1e-12)
