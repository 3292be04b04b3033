"""Pins for the oracle's continuous ingredients, against the paper's own
definitions evaluated independently in high precision (mpmath).

* Eq. (1) [teuk0] of Sec. 3.1, written out term by term in Boyer-Lindquist
  coordinates, applied to Psi = e^{i m phi~} r^3 Phi [eq:psiphi] of an
  arbitrary analytic test function Phi, must equal (up to the normalising
  factor) the oracle's second-order operator built from its coefficient
  fields b, w, c_t, C_r, C_0, V.  A dropped term, a wrong sign or a wrong
  power anywhere in the coefficient derivation fails this.
* The first-order form with Pi = d_t Phi + b d_r* Phi (Sec. 3.2) is equivalent
  iff m_r = b c_t + C_r - b d_r* b; d_r* b is taken numerically here.
* Tortoise coordinate: dr*/dr = (r^2+a^2)/Delta (Sec. 3.2), inversion
  round trip, and agreement with a high-precision root.
* Angular operator: the spin-weighted profiles are eigenfunctions with the
  textbook eigenvalues -(l-s)(l+s+1).
"""

import mpmath as mp
import numpy as np
import pytest

from oracle import teuk_oracle as T

mp.mp.dps = 40

CASES = [  # (M, a, s, m)
    (1.0, 0.0, -2, 2),
    (1.0, 0.9, -2, 2),
    (1.0, 0.7, -2, 3),
    (1.0, 0.5, 2, -1),
    (1.0, 0.99, -1, 4),
]


def _mp_geometry(M, a):
    M, a = mp.mpf(M), mp.mpf(a)
    d = mp.sqrt(M * M - a * a)
    rp, rm = M + d, M - d

    def rstar(r):
        return r + 2 * M * rp / (rp - rm) * mp.log((r - rp) / (2 * M)) \
            - 2 * M * rm / (rp - rm) * mp.log((r - rm) / (2 * M))

    def phit_shift(r):
        # phi~ - phi = int a/Delta dr = a/(r+ - r-) ln((r - r+)/(r - r-))
        return a / (rp - rm) * mp.log((r - rp) / (r - rm))

    return M, a, rp, rm, rstar, phit_shift


def _test_phi(t, rho, th):
    """Generic analytic complex test function Phi(t, r*, theta)."""
    return mp.exp(mp.mpc(0.07, 0.31) * t + mp.mpc(0.05, -0.02) * rho
                  + mp.mpc(0.0, 0.013) * rho * rho) * \
        (mp.mpf(1) + mp.mpf("0.4") * mp.cos(th) + mp.mpc(0, 0.3) * mp.sin(th) ** 2
         + mp.mpf("0.1") * mp.cos(3 * th))


@pytest.mark.parametrize("M,a,s,m", CASES)
def test_coefficients_satisfy_teukolsky_eq1(M, a, s, m):
    Mm, am, rp, rm, rstar, phit_shift = _mp_geometry(M, a)
    rng = np.random.default_rng(11)
    for _ in range(3):
        r0 = mp.mpf(rp) + mp.mpf(float(rng.uniform(0.3, 25.0)))
        th0 = mp.mpf(float(rng.uniform(0.3, 2.8)))
        t0 = mp.mpf(float(rng.uniform(-1, 1)))
        ph0 = mp.mpf(float(rng.uniform(0, 6)))

        def Psi(t, r, th, ph):
            return mp.exp(1j * m * (ph + phit_shift(r))) * r ** 3 * _test_phi(t, rstar(r), th)

        D = mp.diff
        Delta = r0 ** 2 - 2 * Mm * r0 + am ** 2
        st, ct_ = mp.sin(th0), mp.cos(th0)
        args = (t0, r0, th0, ph0)
        # Eq. (1), left-hand side, term by term
        lhs = -((r0 ** 2 + am ** 2) ** 2 / Delta - am ** 2 * st ** 2) * D(Psi, args, (2, 0, 0, 0))
        lhs += -(4 * Mm * am * r0 / Delta) * D(Psi, args, (1, 0, 0, 1))
        lhs += -2 * s * (r0 - Mm * (r0 ** 2 - am ** 2) / Delta + 1j * am * ct_) * D(Psi, args, (1, 0, 0, 0))
        # Delta^{-s} d_r (Delta^{s+1} d_r Psi)
        def flux(r):
            Dl = r ** 2 - 2 * Mm * r + am ** 2
            return Dl ** (s + 1) * D(lambda rr: Psi(t0, rr, th0, ph0), r)
        lhs += Delta ** (-s) * D(flux, r0)
        # (1/sin) d_th (sin d_th Psi)
        def tflux(th):
            return mp.sin(th) * D(lambda tt: Psi(t0, r0, tt, ph0), th)
        lhs += D(tflux, th0) / st
        lhs += (1 / st ** 2 - am ** 2 / Delta) * D(Psi, args, (0, 0, 0, 2))
        lhs += 2 * s * (am * (r0 - Mm) / Delta + 1j * ct_ / st ** 2) * D(Psi, args, (0, 0, 0, 1))
        lhs += -(s ** 2 * (ct_ / st) ** 2 - s) * Psi(*args)

        # normalised source that this Psi implies: F = -Delta lhs e^{-im phi~} / (Sigma^2 r^3)
        Sig2 = (r0 ** 2 + am ** 2) ** 2 - am ** 2 * Delta * st ** 2
        F = -Delta * lhs * mp.exp(-1j * m * (ph0 + phit_shift(r0))) / (Sig2 * r0 ** 3)

        # oracle's second-order operator on Phi
        rho0 = rstar(r0)
        c = T.coefficients(float(r0 - rp), float(th0), M, a, s, m)
        V = T.angular_potential(float(th0), s, m)
        phi = lambda t, rho, th: _test_phi(t, rho, th)
        a3 = (t0, rho0, th0)
        Phi = phi(*a3)
        Phi_t = D(phi, a3, (1, 0, 0))
        Phi_tt = D(phi, a3, (2, 0, 0))
        Phi_r = D(phi, a3, (0, 1, 0))
        Phi_rr = D(phi, a3, (0, 2, 0))
        Phi_th = D(phi, a3, (0, 0, 1))
        Phi_thth = D(phi, a3, (0, 0, 2))
        ang = Phi_thth + (ct_ / st) * Phi_th - V * Phi
        op = (Phi_tt - complex(c["b"]) ** 2 * Phi_rr + complex(c["ct"]) * Phi_t
              - complex(c["Cr"]) * Phi_r - complex(c["C0"]) * Phi - float(c["w"]) * ang)
        scale = max(abs(Phi_tt), abs(F), abs(complex(c["b"]) ** 2 * Phi_rr))
        assert abs(op - F) / scale < 1e-12, (r0, th0, abs(op - F) / scale)


@pytest.mark.parametrize("M,a,s,m", CASES)
def test_first_order_momentum_coefficient(M, a, s, m):
    """m_r = b c_t + C_r - b d_r* b, with d_r* b = (Delta/q) db/dr taken
    numerically from the definitions b = (r^2+a^2)/Sigma,
    Sigma^2 = (r^2+a^2)^2 - a^2 Delta sin^2 (Sec. 3.2)."""
    Mm, am, rp, rm, _, _ = _mp_geometry(M, a)
    for x in [0.01, 0.4, 3.0, 17.0]:
        for th in [0.2, 1.1, 2.5]:
            def b_of_r(r):
                Dl = r ** 2 - 2 * Mm * r + am ** 2
                return (r ** 2 + am ** 2) / mp.sqrt((r ** 2 + am ** 2) ** 2 - am ** 2 * Dl * mp.sin(th) ** 2)
            r0 = rp + mp.mpf(x)
            Dl = r0 ** 2 - 2 * Mm * r0 + am ** 2
            db_drs = Dl / (r0 ** 2 + am ** 2) * mp.diff(b_of_r, r0)
            c = T.coefficients(x, th, M, a, s, m)
            expect = complex(b_of_r(r0) * (mp.mpc(c["ct"]) ) + mp.mpc(c["Cr"]) - b_of_r(r0) * db_drs)
            assert abs(complex(c["mr"]) - expect) <= 1e-13 * max(1.0, abs(expect)) + 1e-15
            assert abs(complex(c["mr_def"]) - expect) <= 1e-13 * max(1.0, abs(expect)) + 1e-15


def test_schwarzschild_closed_forms():
    """a = 0, s = -2: b = 1, c_t = -4(r-3M)/r^2, m_r = 0, C_0 = -6M Delta/r^5,
    w = Delta/r^4 (the s=-2 Regge-Wheeler-like limit of the system)."""
    M = 1.0
    x = np.geomspace(1e-6, 300.0, 50)
    c = T.coefficients(x, 0.7, M, 0.0, -2, 2)
    r = 2.0 + x
    Delta = x * (x + 2 * M)          # r^2 - 2Mr without cancellation near r = 2M
    np.testing.assert_allclose(c["b"], 1.0, rtol=1e-15)
    np.testing.assert_allclose(c["ct"].real, -4 * (r - 3 * M) / r ** 2, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(c["ct"].imag, 0.0, atol=0)
    assert np.all(c["mr"] == 0.0)           # the cancellation-free form is exactly zero
    np.testing.assert_allclose(c["mr_def"], 0.0, atol=1e-13)
    np.testing.assert_allclose(c["C0"].real, -6 * M * Delta / r ** 5, rtol=1e-11, atol=1e-18)
    np.testing.assert_allclose(c["w"], Delta / r ** 4, rtol=1e-12)


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9, 0.99])
def test_tortoise_derivative_and_a0_form(a):
    M = 1.0
    rp, rm = T.horizons(M, a)
    x = np.geomspace(1e-3, 500.0, 40)
    h = 1e-6 * x
    num = (T.tortoise_of_x(x + h, M, a) - T.tortoise_of_x(x - h, M, a)) / (2 * h)
    r = rp + x
    np.testing.assert_allclose(num, (r * r + a * a) / ((r - rp) * (r - rm)), rtol=2e-7)
    if a == 0.0:
        far = x > 1.0          # r/2M - 1 loses digits close to the horizon
        np.testing.assert_allclose(T.tortoise_of_x(x[far], M, a),
                                   r[far] + 2 * M * np.log(r[far] / (2 * M) - 1), rtol=1e-13)


@pytest.mark.parametrize("a", [0.0, 0.7, 0.9, 0.99])
def test_tortoise_inversion(a):
    M = 1.0
    rs = np.linspace(-200.0, 600.0, 1601)
    x = T.x_of_tortoise(rs, M, a)
    assert np.all(x > 0)
    np.testing.assert_allclose(T.tortoise_of_x(x, M, a), rs, rtol=0, atol=1e-13 * 600)
    # independent high-precision roots at a few points
    _, _, rp, rm, rstar, _ = _mp_geometry(M, a)
    for k in [0, 200, 750, 1000, 1600]:
        # r* written in x = r - r_+ so that x ~ 1e-44 is not lost against r_+
        f = lambda yy: (rp + mp.exp(yy) + 2 * rp / (rp - rm) * (yy - mp.log(2))
                        - 2 * rm / (rp - rm) * mp.log((mp.exp(yy) + rp - rm) / 2) - mp.mpf(rs[k]))
        y = mp.findroot(f, mp.mpf(np.log(x[k])), tol=mp.mpf(10) ** -60, verify=False)
        assert abs(f(y)) < mp.mpf(10) ** -25
        assert abs(float(mp.exp(y)) / x[k] - 1.0) < 1e-12


@pytest.mark.parametrize("m,l", [(1, 2), (2, 2), (3, 3), (4, 4)])
def test_angular_profiles_are_spin_weighted_eigenfunctions(m, l):
    """Ang[P] = -(l-s)(l+s+1) P for s = -2 and the lowest l = max(|m|,|s|)."""
    s = -2
    written = {1: lambda t: mp.sin(t) * (1 + mp.cos(t)),
               2: lambda t: (1 + mp.cos(t)) ** 2,
               3: lambda t: mp.sin(t) * (1 + mp.cos(t)) ** 2,
               4: lambda t: mp.sin(t) ** 2 * (1 + mp.cos(t)) ** 2}[m]
    for th in [0.3, 1.0, 1.7, 2.6]:
        P = float(written(th))
        assert abs(T.angular_profile(th, s, m) - P) < 1e-14 * max(1, abs(P))
        V = T.angular_potential(th, s, m)
        ang = mp.diff(written, th, 2) + mp.cot(th) * mp.diff(written, th) - V * written(th)
        assert abs(float(ang) + (l - s) * (l + s + 1) * P) < 1e-12 * max(1.0, abs(P))
