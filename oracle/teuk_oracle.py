"""CPU FP64 oracle for the m-mode Teukolsky Lax-Wendroff evolution.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
HIP path is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library: coefficients, tortoise inversion,
initial data, source, stepping, boundary conditions, extraction and adjoint
are all written out here again, directly from the paper.

What it follows (Khanna & McKennon, "Numerical modeling of gravitational wave
sources accelerated by OpenCL"):

* Sec. 3.1, Eq. (1) [teuk0]: the Teukolsky master equation in Boyer-Lindquist
  coordinates.  The explicit first-order system is not printed in the paper
  (it refers to the literature); it is derived here from Eq. (1) with the
  tortoise coordinate, the azimuth phi~ and the ansatz of Sec. 3.2 [eq:psiphi],
  and the momentum Pi = d_t Phi + b d_r* Phi with b = (r^2+a^2)/Sigma and
  Sigma^2 = (r^2+a^2)^2 - a^2 Delta sin^2(theta) [pi_eq].  Dividing Eq. (1) by
  -Sigma^2 r^3 e^{i m phi~}/Delta gives

      Phi_tt - b^2 Phi_r*r* + c_t Phi_t - C_r Phi_r* - C_0 Phi - w Ang[Phi] = F

  and with Pi the system  d_t u + D d_r* u = S  of Sec. 3.2 [new_teu2,
  d_matrix], D = diag(b, -b) on (Phi, Pi):

      S_Phi = Pi
      S_Pi  = -c_t Pi + m_r d_r*Phi + C_0 Phi + w Ang[Phi] + F,
      m_r   = b c_t + C_r - b d_r* b.

* Sec. 3.2, Eqs. (lw1) and (lw2): the two-step Lax-Wendroff iteration, with
  second-order centred angular differences, and the boundary conditions of
  the same section (Phi = Pi = 0 on both radial ends; d_theta Phi = 0 at the
  poles for even |m|, Phi = 0 there for odd |m|).

Readings where the paper is silent (each one is listed with its reason in the
design notes): nodes include both ends in r* and theta; coefficients at the
half points are evaluated at r*_{i+1/2} (not averaged); S at a half point is
built from the averaged state and the same radial difference that multiplies
D; pole rows are never evolved, they are set from the boundary condition
(u_0 = (4u_1 - u_2)/3 for even |m|) for both the half-step and the full-step
values; the step is dt = cfl * min(h_r*, r(r*_min) h_theta); an optional
theta-direction fourth-difference dissipation (strength eps) is added in the
full step, because the literal scheme is weakly unstable for the stiff
angular modes next to the poles (see tests/test_oracle_stability.py).

Every function works on complex128 arrays laid out [theta row j][r* column i].
"""

import numpy as np

__all__ = [
    "horizons", "tortoise_of_x", "x_of_tortoise", "coefficients",
    "angular_potential", "Grid", "Source", "circular_orbit", "equatorial_constants",
    "equatorial_rates", "eccentric_orbit", "initial_pulse",
    "apply_bc", "step", "evolve", "adjoint_step", "adjoint_evolve",
    "waveform_loss", "assemble_step_matrix", "radiated_flux",
]


# ---------------------------------------------------------------------------
# Geometry (Sec. 3.2: tortoise coordinate and azimuth)
# ---------------------------------------------------------------------------

def horizons(M, a):
    """Outer and inner horizon radii r_+- = M +- sqrt(M^2 - a^2) (roots of Delta)."""
    d = np.sqrt(M * M - a * a)
    return M + d, M - d


def tortoise_of_x(x, M, a):
    """r*(r) written in x = r - r_+ (> 0).

    Integral of dr*/dr = (r^2 + a^2)/Delta (Sec. 3.2), with the standard
    integration constant: r* = r + 2M r_+/(r_+ - r_-) ln((r - r_+)/2M)
    - 2M r_-/(r_+ - r_-) ln((r - r_-)/2M).  At a = 0 this is
    r + 2M ln(r/2M - 1).
    """
    rp, rm = horizons(M, a)
    A = 2.0 * M * rp / (rp - rm)
    B = 2.0 * M * rm / (rp - rm)
    x = np.asarray(x, dtype=np.float64)
    return rp + x + A * np.log(x / (2.0 * M)) - B * np.log((x + rp - rm) / (2.0 * M))


def x_of_tortoise(rs, M, a):
    """Invert r*(r): return x = r - r_+ for each r* by bisection on y = ln x.

    r* is strictly increasing in y (dr*/dy = x (r^2+a^2)/Delta > 0), so
    bisection on a bracket [y_lo, y_hi] with r*(y_lo) < r* < r*(y_hi) is
    plainly correct.  Working in y keeps x to full relative precision near
    the horizon, where x ~ 1e-44 at r* = -200M for a = 0.
    """
    rs = np.atleast_1d(np.asarray(rs, dtype=np.float64))
    lo = np.full(rs.shape, -700.0)
    hi = np.log(np.abs(rs) + 10.0 * M) + 2.0
    assert np.all(tortoise_of_x(np.exp(lo), M, a) < rs), "r* below bracket"
    assert np.all(tortoise_of_x(np.exp(hi), M, a) > rs), "r* above bracket"
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        done = (mid == lo) | (mid == hi)
        if np.all(done):
            break
        above = tortoise_of_x(np.exp(mid), M, a) > rs
        hi = np.where(above & ~done, mid, hi)
        lo = np.where(~above & ~done, mid, lo)
    # pick the endpoint whose residual is smaller
    flo = np.abs(tortoise_of_x(np.exp(lo), M, a) - rs)
    fhi = np.abs(tortoise_of_x(np.exp(hi), M, a) - rs)
    return np.exp(np.where(flo <= fhi, lo, hi))


# ---------------------------------------------------------------------------
# Coefficients of the first-order system (derived from Eq. (1), Sec. 3.1-3.2)
# ---------------------------------------------------------------------------

def coefficients(x, theta, M, a, s, m):
    """Coefficient fields b, w, c_t, m_r, C_0 at points (x = r - r_+, theta).

    Derived from Eq. (1) [teuk0] with Psi = e^{i m phi~} r^3 Phi [eq:psiphi]
    and the tortoise coordinate; Sigma^2 and b as in [pi_eq]:

      Delta = r^2 - 2Mr + a^2,  q = r^2 + a^2,  Sigma^2 = q^2 - a^2 Delta sin^2
      b   = q / Sigma                      (principal radial speed, matrix D)
      w   = Delta / Sigma^2                (angular operator weight)
      c_t = [4iMamr + 2s(r Delta - M(r^2 - a^2)) + 2isa Delta cos] / Sigma^2
      C_r = [q s Delta' + 2r Delta + 2imaq + 6q Delta/r] / Sigma^2
      C_0 = [2imas Delta' + (3 Delta/r^2)(2 Delta + (1+s) r Delta' + 2imar)] / Sigma^2
      m_r = b c_t + C_r - b d_r* b            (from eliminating Phi_t with Pi)

    Polynomials that cancel at large r or vanish identically are evaluated in
    expanded, cancellation-free forms (the same fields); "mr_def" keeps m_r
    as written above for cross-checking.

    Arguments broadcast; x and theta may be arrays of compatible shapes.
    """
    rp, rm = horizons(M, a)
    x = np.asarray(x, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    r = rp + x
    Delta = x * (x + rp - rm)
    dDelta = 2.0 * (r - M)
    q = r * r + a * a
    sin2 = np.sin(theta) ** 2
    cos = np.cos(theta)
    Sig2 = q * q - a * a * Delta * sin2
    Sig = np.sqrt(Sig2)
    b = q / Sig
    w = Delta / Sig2
    # r Delta - M(r^2 - a^2) = r^2 (r - 3M) + a^2 (r + M)
    ct_re_num = 2.0 * s * (r * r * (r - 3.0 * M) + a * a * (r + M))
    ct = (ct_re_num + 1j * (4.0 * M * a * m * r + 2.0 * s * a * Delta * cos)) / Sig2
    Cr = (q * s * dDelta + 2.0 * r * Delta + 2j * m * a * q + 6.0 * q * Delta / r) / Sig2
    # 2 Delta + (1+s) r Delta' = 2(2+s) r^2 - 2(3+s) M r + 2 a^2
    C0 = (2j * m * a * s * dDelta
          + (3.0 * Delta / r ** 2) * (2.0 * (2.0 + s) * r * r - 2.0 * (3.0 + s) * M * r + 2.0 * a * a
                                      + 2j * m * a * r)) / Sig2
    # m_r by its definition, b c_t + C_r - b d_r* b, with d_r* b = (Delta/q) d/dr (q/Sigma)
    dSig_dr = (4.0 * r * q - a * a * dDelta * sin2) / (2.0 * Sig)
    db_drs = (Delta / q) * (2.0 * r / Sig - q * dSig_dr / Sig2)
    mr_def = b * ct + Cr - b * db_drs
    # The same field collected over Sigma^4 so that nothing cancels (for a = 0,
    # s = -2 it vanishes identically, and the definition above leaves ~1e-16
    # of rounding residue that the evolution amplifies):
    #   Re m_r Sigma^4 = q^2 Delta [4(s+2) r + 6 a^2/r]
    #                    - a^2 Delta sin^2 [q ct_re_num/(q + Sigma) + q((s + 1/2) Delta' + 6 Delta/r)]
    #   Im m_r = q (4Mamr + 2sa Delta cos)/Sigma^3 + 2maq/Sigma^2
    re = (q * q * Delta * (4.0 * (s + 2.0) * r + 6.0 * a * a / r)
          - a * a * Delta * sin2 * (q * ct_re_num / (q + Sig)
                                    + q * ((s + 0.5) * dDelta + 6.0 * Delta / r))) / (Sig2 * Sig2)
    im = q * (4.0 * M * a * m * r + 2.0 * s * a * Delta * cos) / (Sig2 * Sig) + 2.0 * m * a * q / Sig2
    mr = re + 1j * im
    return {"b": b, "w": w, "ct": ct, "Cr": Cr, "C0": C0, "mr": mr, "mr_def": mr_def,
            "r": r, "Delta": Delta, "q": q, "Sig2": Sig2}


def angular_potential(theta, s, m):
    """V(theta) = (m + s cos)^2 / sin^2 - s, so that the angular part of
    Eq. (1) acting on Phi is Ang[Phi] = Phi_thth + cot Phi_th - V Phi."""
    theta = np.asarray(theta, dtype=np.float64)
    return (m + s * np.cos(theta)) ** 2 / np.sin(theta) ** 2 - s


# ---------------------------------------------------------------------------
# Grid, time step, tables
# ---------------------------------------------------------------------------

class Grid:
    """Uniform (r*, theta) grid with its coefficient fields.

    Nodes r*_i = r*_min + i h_r (i = 0..nr-1, both ends included), half points
    r*_{i+1/2} = r*_i + h_r/2 (i = 0..nr-2), theta_j = j h_th (j = 0..nth-1,
    h_th = pi/(nth-1), poles included).  dt = cfl * min(h_r, r(r*_min) h_th).
    """

    def __init__(self, M, a, s, m, nr, nth, rs_min, rs_max, cfl=0.5,
                 rs_extract=None, ko_eps=0.0):
        if not (abs(a) < M):
            raise ValueError("need |a| < M")
        if nr < 5 or nth < 7:
            raise ValueError("need nr >= 5 and nth >= 7")
        self.M, self.a, self.s, self.m = float(M), float(a), int(s), int(m)
        self.nr, self.nth = int(nr), int(nth)
        self.rs_min, self.rs_max = float(rs_min), float(rs_max)
        self.cfl = float(cfl)
        self.ko_eps = float(ko_eps)
        self.hr = (self.rs_max - self.rs_min) / (self.nr - 1)
        self.hth = np.pi / (self.nth - 1)
        self.rs = self.rs_min + np.arange(self.nr) * self.hr
        self.rs_half = self.rs[:-1] + 0.5 * self.hr
        self.th = np.arange(self.nth) * self.hth
        self.x = x_of_tortoise(self.rs, self.M, self.a)
        self.x_half = x_of_tortoise(self.rs_half, self.M, self.a)
        rp, _ = horizons(self.M, self.a)
        self.r = rp + self.x
        self.dt = self.cfl * min(self.hr, self.r[0] * self.hth)
        self.even = (abs(self.m) % 2 == 0)
        th = self.th[:, None]
        self.node = coefficients(self.x[None, :], th, self.M, self.a, self.s, self.m)
        self.half = coefficients(self.x_half[None, :], th, self.M, self.a, self.s, self.m)
        jj = self.th[1:-1]
        self.cot = np.cos(jj) / np.sin(jj)
        self.V = angular_potential(jj, self.s, self.m)
        if rs_extract is None:
            rs_extract = self.rs_max
        self.rs_extract = float(rs_extract)
        self.i_ext = int(np.rint((self.rs_extract - self.rs_min) / self.hr))
        if not (0 <= self.i_ext < self.nr):
            raise ValueError("extraction radius outside the grid")

    def ang(self, f):
        """Second-order centred Ang[f] on the interior rows j = 1..nth-2
        (Sec. 3.2: angular derivatives by centred differences).  f has all
        rows; the result has nth-2 rows."""
        h = self.hth
        up, mid, dn = f[2:], f[1:-1], f[:-2]
        return ((up - 2.0 * mid + dn) / (h * h)
                + self.cot[:, None] * (up - dn) / (2.0 * h)
                - self.V[:, None] * mid)

    def ang_T(self, y):
        """Transpose of ang (real coefficients): maps nth-2 rows to nth rows."""
        h = self.hth
        alpha = 1.0 / (h * h) + self.cot / (2.0 * h)     # multiplies f_{j+1}
        beta = -2.0 / (h * h) - self.V                    # multiplies f_j
        gamma = 1.0 / (h * h) - self.cot / (2.0 * h)     # multiplies f_{j-1}
        out = np.zeros((self.nth,) + y.shape[1:], dtype=np.complex128)
        out[2:] += alpha[:, None] * y
        out[1:-1] += beta[:, None] * y
        out[:-2] += gamma[:, None] * y
        return out


# ---------------------------------------------------------------------------
# Synthetic point-particle source (stands in for T of Eq. (1))
# ---------------------------------------------------------------------------

def circular_orbit(M, a, r0, dt, nsteps):
    """Circular equatorial prograde orbit sampled at t_k = k dt/2,
    k = 0..2*nsteps: (r*_p, theta_p, phi~_p).  Omega = M^{1/2}/(r0^{3/2} + a M^{1/2});
    phi~_p = Omega t (phase zero at t = 0); r*_p = r*(r0)."""
    rp, _ = horizons(M, a)
    rs_p = float(tortoise_of_x(r0 - rp, M, a))
    Omega = np.sqrt(M) / (r0 ** 1.5 + a * np.sqrt(M))
    t = np.arange(2 * nsteps + 1) * (0.5 * dt)
    return {"rs": np.full(t.shape, rs_p), "th": np.full(t.shape, 0.5 * np.pi),
            "phi": Omega * t, "Omega": Omega}


def _kerr_R(r, E, L, a):
    """Equatorial radial geodesic potential (M = 1, Carter constant 0):
    R(r) = [E(r^2+a^2) - a L]^2 - Delta [r^2 + (L - a E)^2], with
    (r^2 dr/dtau)^2 = R(r)."""
    delta = r * r - 2.0 * r + a * a
    P = E * (r * r + a * a) - a * L
    return P * P - delta * (r * r + (L - a * E) ** 2)


def equatorial_constants(a, p, e):
    """Energy E, angular momentum L and third root r_3 of a bound prograde
    equatorial Kerr geodesic with periapsis p/(1+e) and apoapsis p/(1-e)
    (M = 1).  Defined by R vanishing at both turning points (for e = 0: a
    double root, R(p) = R'(p) = 0), solved by a library root finder started
    from the Schwarzschild values.  r_3 is the remaining positive root of
    R(r)/r, a cubic."""
    import warnings

    from scipy.optimize import fsolve

    rp_, ra_ = p / (1.0 + e), p / (1.0 - e)
    E0 = np.sqrt(((p - 2.0) ** 2 - 4.0 * e * e) / (p * (p - 3.0 - e * e)))
    L0 = p / np.sqrt(p - 3.0 - e * e)
    if e > 0.0:
        def eqs(v):
            return [_kerr_R(rp_, v[0], v[1], a) / rp_ ** 4, _kerr_R(ra_, v[0], v[1], a) / ra_ ** 4]
    else:
        def eqs(v):
            h = 1e-4 * p
            dR = (_kerr_R(p + h, v[0], v[1], a) - _kerr_R(p - h, v[0], v[1], a)) / (2.0 * h)
            return [_kerr_R(p, v[0], v[1], a) / p ** 4, dR / p ** 3]
    with warnings.catch_warnings():   # at full precision fsolve reports that it cannot improve
        warnings.simplefilter("ignore", RuntimeWarning)
        E, L = fsolve(eqs, [E0, L0], xtol=1e-15)
    if e == 0.0:
        # R'(p) by a central difference is exact for the quartic up to an
        # O(h^2) term that the double root makes vanish to rounding; polish
        # with the exact derivative.
        def eqs2(v):
            E_, L_ = v
            P = E_ * (p * p + a * a) - a * L_
            delta = p * p - 2.0 * p + a * a
            dR = 4.0 * E_ * p * P - (2.0 * p - 2.0) * (p * p + (L_ - a * E_) ** 2) - delta * 2.0 * p
            return [_kerr_R(p, E_, L_, a) / p ** 4, dR / p ** 3]
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", RuntimeWarning)
            E, L = fsolve(eqs2, [E, L], xtol=1e-15)
    # R(r)/r = (E^2-1) r^3 + 2 r^2 - (a^2 + x^2 + 2 a x E) r + 2 x^2, x = L - a E
    x = L - a * E
    roots = np.roots([E * E - 1.0, 2.0, -(a * a + x * x + 2.0 * a * x * E), 2.0 * x * x])
    roots = np.sort(np.real(roots[np.abs(np.imag(roots)) < 1e-6 * p]))
    r3 = float(roots[0])
    return float(E), float(L), r3


def equatorial_rates(a, p, e, E, L, r3, chi):
    """dt/dchi and dphi/dchi along the orbit r = p/(1 + e cos chi) (M = 1).
    From the geodesic equations r^2 dt/dtau = a(L - aE) + (r^2+a^2) P/Delta,
    r^2 dphi/dtau = (L - aE) + a P/Delta, P = E(r^2+a^2) - aL, and
    dtau/dchi = (dr/dchi) r^2/sqrt(R) with R = (1-E^2) r (r_a - r)(r - r_p)(r - r_3),
    in which (dr/dchi)/sqrt((r_a - r)(r - r_p)) = sqrt(1-e^2)/(1 + e cos chi)."""
    chi = np.asarray(chi, dtype=np.float64)
    den = 1.0 + e * np.cos(chi)
    r = p / den
    delta = r * r - 2.0 * r + a * a
    P = E * (r * r + a * a) - a * L
    dtau = r * r * np.sqrt(1.0 - e * e) / (den * np.sqrt((1.0 - E * E) * r * (r - r3)))
    vt = (a * (L - a * E) + (r * r + a * a) * P / delta) / (r * r) * dtau
    vphi = ((L - a * E) + a * P / delta) / (r * r) * dtau
    return vt, vphi, dtau


def eccentric_orbit(M, a, p, e, chi0, dt, nsteps):
    """Bound prograde equatorial Kerr orbit (semi-latus rectum p, eccentricity
    e, relativistic anomaly chi0 at t = 0, chi = 0 at periapsis) sampled at
    t_k = k dt/2, k = 0..2*nsteps: (r*_p, theta_p, phi~_p).

    t(chi) and phi(chi) are integrated by adaptive quadrature from sample to
    sample, and chi at each t_k is found by Newton's method on t(chi) - t_k
    (dt/dchi > 0).  phi~ = phi + a/(r_+ - r_-) ln((r - r_+)/(r - r_-)) is the
    azimuth of Sec. 3.2 (d phi~ = d phi + a/Delta dr), with phase zero at t = 0.
    Lengths and times in units of M."""
    from scipy.integrate import quad

    a_, p_ = a / M, p / M
    E, L, r3 = equatorial_constants(a_, p_, e)
    vt = lambda c: float(equatorial_rates(a_, p_, e, E, L, r3, c)[0])
    vp = lambda c: float(equatorial_rates(a_, p_, e, E, L, r3, c)[1])
    rp, rm = horizons(1.0, a_)

    def phitilde_shift(r):
        return a_ / (rp - rm) * np.log((r - rp) / (r - rm))

    n = 2 * nsteps + 1
    h = 0.5 * dt / M
    chis = np.empty(n)
    phis = np.empty(n)
    chis[0], phis[0] = chi0, 0.0
    for k in range(1, n):
        c0 = chis[k - 1]
        c = c0 + h / vt(c0)
        for _ in range(50):
            f = quad(vt, c0, c, epsabs=0.0, epsrel=2e-14, limit=200)[0] - h
            dc = f / vt(c)
            c -= dc
            if abs(dc) <= 1e-16 * max(1.0, abs(c)):
                break
        chis[k] = c
        phis[k] = phis[k - 1] + quad(vp, c0, c, epsabs=0.0, epsrel=2e-14, limit=200)[0]
    r = p_ / (1.0 + e * np.cos(chis))
    rs = tortoise_of_x((r - rp) * M, M, a)
    phit = phis + phitilde_shift(r) - phitilde_shift(r[0])
    return {"rs": np.asarray(rs, dtype=np.float64), "th": np.full(n, 0.5 * np.pi), "phi": phit,
            "chi": chis, "r": r * M, "E": E, "L": L, "r3": r3}


class Source:
    """Gaussian-smeared particle: F = A G(r*-r*_p; s_r) G(theta-theta_p; s_th)
    e^{-i m phi~_p}, G(x; s) = exp(-x^2/2s^2)/(sqrt(2 pi) s), zero where
    |x| > cutoff*s.  Enters the Pi row of S only.  Samples of the orbit are
    given at t_k = k dt/2 (k = 2n for the half step of iteration n, k = 2n+1
    for its full step)."""

    def __init__(self, grid, orbit, amplitude=1.0, sigma_r_cells=2.0,
                 sigma_th_cells=2.0, cutoff_sigmas=8.0):
        self.g = grid
        self.orbit = orbit
        self.A = float(amplitude)
        self.sr = sigma_r_cells * grid.hr
        self.sth = sigma_th_cells * grid.hth
        self.cut = float(cutoff_sigmas)

    @staticmethod
    def _gauss(x, sig, cut):
        val = np.exp(-x * x / (2.0 * sig * sig)) / (np.sqrt(2.0 * np.pi) * sig)
        return np.where(np.abs(x) <= cut * sig, val, 0.0)

    def field(self, k, rs, th, amplitude=None):
        """F at orbit sample k on the outer product th (rows) x rs (columns)."""
        A = self.A if amplitude is None else amplitude
        o = self.orbit
        gr = self._gauss(rs - o["rs"][k], self.sr, self.cut)
        gt = self._gauss(th - o["th"][k], self.sth, self.cut)
        return A * np.exp(-1j * self.g.m * o["phi"][k]) * gt[:, None] * gr[None, :]


# ---------------------------------------------------------------------------
# Initial data and boundary conditions
# ---------------------------------------------------------------------------

def angular_profile(theta, s, m):
    """Lowest-l spin-weighted profile 2^{(|m+s|+|m-s|)/2} sin^{|m+s|}(th/2)
    cos^{|m-s|}(th/2); for s = -2 it is (1+cos)^2 (m=2), sin(1+cos) (m=1),
    sin(1+cos)^2 (m=3), sin^2(1+cos)^2 (m=4)."""
    p, q = abs(m + s), abs(m - s)
    return (2.0 ** (0.5 * (p + q)) * np.sin(0.5 * theta) ** p * np.cos(0.5 * theta) ** q)


def apply_bc(g, phi, pi):
    """Boundary conditions of Sec. 3.2, in place: zero on the two radial end
    columns; pole rows zero (odd |m|) or (4u_1 - u_2)/3 (even |m|, one-sided
    second-order d_theta u = 0)."""
    for u in (phi, pi):
        u[:, 0] = 0.0
        u[:, -1] = 0.0
        if g.even:
            u[0, 1:-1] = (4.0 * u[1, 1:-1] - u[2, 1:-1]) / 3.0
            u[-1, 1:-1] = (4.0 * u[-2, 1:-1] - u[-3, 1:-1]) / 3.0
        else:
            u[0, :] = 0.0
            u[-1, :] = 0.0


def initial_pulse(g, center, width, amplitude=1.0):
    """Phi(0) = A exp(-(r*-c)^2/(2 width^2)) P(theta); time-symmetric data
    d_t Phi = 0, so Pi(0) = b d_r* Phi(0) = -b (r*-c)/width^2 Phi(0); then the
    boundary conditions."""
    rad = np.exp(-(g.rs - center) ** 2 / (2.0 * width * width))
    P = angular_profile(g.th, g.s, g.m)
    phi = (amplitude * P[:, None] * rad[None, :]).astype(np.complex128)
    pi = (-g.node["b"] * (g.rs[None, :] - center) / (width * width) * phi).astype(np.complex128)
    apply_bc(g, phi, pi)
    return phi, pi


# ---------------------------------------------------------------------------
# One Lax-Wendroff iteration, Eqs. (lw1)-(lw2)
# ---------------------------------------------------------------------------

def _ko_delta4(g, u):
    """Fourth theta-difference of u at interior rows, with ghost rows
    u_{-1} = sigma u_1 and u_{nth} = sigma u_{nth-2} (sigma = +1 even |m|,
    -1 odd |m|: the reflection the pole condition implies)."""
    sig = 1.0 if g.even else -1.0
    ext = np.concatenate([sig * u[1:2], u, sig * u[-2:-1]], axis=0)
    # ext index e = j + 1
    return ext[4:] - 4.0 * ext[3:-1] + 6.0 * ext[2:-2] - 4.0 * ext[1:-3] + ext[:-4]


def step(g, phi, pi, n, source=None, amplitude=None):
    """u^n -> u^{n+1}.  Source (if any) at orbit sample 2n for the half step
    (time t_n) and 2n+1 for the full step (t_n + dt/2)."""
    dt, hr, nth, nr = g.dt, g.hr, g.nth, g.nr
    J = slice(1, nth - 1)
    # ---- (lw1): half step at r*_{i+1/2}, interior rows ----
    pbar = 0.5 * (phi[:, 1:] + phi[:, :-1])
    qbar = 0.5 * (pi[:, 1:] + pi[:, :-1])
    dphi = (phi[:, 1:] - phi[:, :-1]) / hr
    dpi = (pi[:, 1:] - pi[:, :-1]) / hr
    c = g.half
    S_pi = (-c["ct"][J] * qbar[J] + c["mr"][J] * dphi[J] + c["C0"][J] * pbar[J]
            + c["w"][J] * g.ang(pbar))
    if source is not None:
        S_pi = S_pi + source.field(2 * n, g.rs_half, g.th, amplitude)[J]
    S_phi = qbar[J]
    hphi = np.zeros_like(pbar)
    hpi = np.zeros_like(qbar)
    hphi[J] = pbar[J] - 0.5 * dt * (c["b"][J] * dphi[J] - S_phi)
    hpi[J] = qbar[J] - 0.5 * dt * (-c["b"][J] * dpi[J] - S_pi)
    # pole rows of the half-step values from the boundary condition
    if g.even:
        for h in (hphi, hpi):
            h[0] = (4.0 * h[1] - h[2]) / 3.0
            h[-1] = (4.0 * h[-2] - h[-3]) / 3.0
    # ---- (lw2): full step at interior nodes i = 1..nr-2 ----
    I = slice(1, nr - 1)
    ptil = 0.5 * (hphi[:, 1:] + hphi[:, :-1])
    qtil = 0.5 * (hpi[:, 1:] + hpi[:, :-1])
    dhphi = (hphi[:, 1:] - hphi[:, :-1]) / hr
    dhpi = (hpi[:, 1:] - hpi[:, :-1]) / hr
    c = {k: v[:, I] for k, v in g.node.items()}
    S_pi = (-c["ct"][J] * qtil[J] + c["mr"][J] * dhphi[J] + c["C0"][J] * ptil[J]
            + c["w"][J] * g.ang(ptil))
    if source is not None:
        S_pi = S_pi + source.field(2 * n + 1, g.rs[I], g.th, amplitude)[J]
    S_phi = qtil[J]
    phi_new = phi.copy()
    pi_new = pi.copy()
    phi_new[J, I] = phi[J, I] - dt * (c["b"][J] * dhphi[J] - S_phi)
    pi_new[J, I] = pi[J, I] - dt * (-c["b"][J] * dhpi[J] - S_pi)
    if g.ko_eps != 0.0:
        phi_new[J, I] -= (g.ko_eps / 16.0) * _ko_delta4(g, phi)[:, I]
        pi_new[J, I] -= (g.ko_eps / 16.0) * _ko_delta4(g, pi)[:, I]
    apply_bc(g, phi_new, pi_new)
    return phi_new, pi_new


def evolve(g, phi0, pi0, nsteps, source=None, amplitude=None, snapshots=None):
    """Run nsteps iterations.  Returns (Phi^N, Pi^N, w) with w[n-1, j] =
    Phi^n(r*_{i_ext}, theta_j) for n = 1..N (extraction after every step).
    If `snapshots` is a dict, snapshots[n] = (Phi^n, Pi^n) for n in its keys."""
    phi = np.array(phi0, dtype=np.complex128, copy=True)
    pi = np.array(pi0, dtype=np.complex128, copy=True)
    w = np.empty((nsteps, g.nth), dtype=np.complex128)
    for n in range(nsteps):
        phi, pi = step(g, phi, pi, n, source, amplitude)
        w[n] = phi[:, g.i_ext]
        if snapshots is not None and (n + 1) in snapshots:
            snapshots[n + 1] = (phi.copy(), pi.copy())
    return phi, pi, w


# ---------------------------------------------------------------------------
# Adjoint: transpose of one iteration, written sub-step by sub-step
# ---------------------------------------------------------------------------

def adjoint_step(g, lphi, lpi, n, source=None):
    """lambda^{n+1} -> lambda^n = G^H lambda^{n+1}, plus the unit-amplitude
    source sensitivity Re<lambda^{n+1}, d u^{n+1}/dA>.

    The step is C-linear, so its transpose in the real inner product is the
    conjugate transpose: every complex coefficient is conjugated and every
    sub-step (boundary projection, full step, pole rows of the half step,
    half step) is transposed in reverse order.
    """
    dt, hr, nth, nr = g.dt, g.hr, g.nth, g.nr
    J = slice(1, nth - 1)
    I = slice(1, nr - 1)
    cj = np.conj
    # ---- transpose of the boundary conditions on u^{n+1} ----
    mphi = np.zeros_like(lphi)
    mpi = np.zeros_like(lpi)
    mphi[J, I] = lphi[J, I]
    mpi[J, I] = lpi[J, I]
    if g.even:
        for mu, lam in ((mphi, lphi), (mpi, lpi)):
            mu[1, I] += (4.0 / 3.0) * lam[0, I]
            mu[2, I] -= (1.0 / 3.0) * lam[0, I]
            mu[-2, I] += (4.0 / 3.0) * lam[-1, I]
            mu[-3, I] -= (1.0 / 3.0) * lam[-1, I]
    # ---- transpose of the full step (lw2) ----
    out_phi = mphi.copy()          # identity part u^n -> u^{n+1} on interior nodes
    out_pi = mpi.copy()
    if g.ko_eps != 0.0:
        sig = 1.0 if g.even else -1.0
        for out, mu in ((out_phi, mphi), (out_pi, mpi)):
            y = -(g.ko_eps / 16.0) * mu[J, I]          # (nth-2, nr-2)
            ext = np.zeros((nth + 2, nr - 2), dtype=np.complex128)
            ext[4:] += y
            ext[3:-1] += -4.0 * y
            ext[2:-2] += 6.0 * y
            ext[1:-3] += -4.0 * y
            ext[:-4] += y
            out[:, I] += ext[1:-1]
            out[1, I] += sig * ext[0]
            out[-2, I] += sig * ext[-1]
    c = {k: v[:, I] for k, v in g.node.items()}
    mP = mphi[J, I]
    mQ = mpi[J, I]
    l_dh_phi = -dt * c["b"][J] * mP + dt * cj(c["mr"][J]) * mQ
    l_dh_pi = dt * c["b"][J] * mQ
    l_qtil = np.zeros((nth, nr - 2), dtype=np.complex128)
    l_ptil = np.zeros((nth, nr - 2), dtype=np.complex128)
    l_qtil[J] = dt * mP - dt * cj(c["ct"][J]) * mQ
    l_ptil[J] = dt * cj(c["C0"][J]) * mQ
    l_ptil += g.ang_T(dt * c["w"][J] * mQ)
    dA = 0.0
    if source is not None:
        F = source.field(2 * n + 1, g.rs[I], g.th, 1.0)[J]
        dA += float(np.real(np.sum(np.conj(mQ) * dt * F)))
    lh_phi = np.zeros((nth, nr - 1), dtype=np.complex128)
    lh_pi = np.zeros((nth, nr - 1), dtype=np.complex128)
    lh_phi[:, :-1] += 0.5 * l_ptil
    lh_phi[:, 1:] += 0.5 * l_ptil
    lh_pi[:, :-1] += 0.5 * l_qtil
    lh_pi[:, 1:] += 0.5 * l_qtil
    lh_phi[J, 1:] += l_dh_phi / hr
    lh_phi[J, :-1] -= l_dh_phi / hr
    lh_pi[J, 1:] += l_dh_pi / hr
    lh_pi[J, :-1] -= l_dh_pi / hr
    # ---- transpose of the half-step pole rows ----
    for lh in (lh_phi, lh_pi):
        if g.even:
            lh[1] += (4.0 / 3.0) * lh[0]
            lh[2] -= (1.0 / 3.0) * lh[0]
            lh[-2] += (4.0 / 3.0) * lh[-1]
            lh[-3] -= (1.0 / 3.0) * lh[-1]
        lh[0] = 0.0
        lh[-1] = 0.0
    # ---- transpose of the half step (lw1) ----
    c = g.half
    hP = lh_phi[J]
    hQ = lh_pi[J]
    l_pbar = np.zeros((nth, nr - 1), dtype=np.complex128)
    l_qbar = np.zeros((nth, nr - 1), dtype=np.complex128)
    l_pbar[J] = hP + 0.5 * dt * cj(c["C0"][J]) * hQ
    l_pbar += g.ang_T(0.5 * dt * c["w"][J] * hQ)
    l_qbar[J] = 0.5 * dt * hP + hQ - 0.5 * dt * cj(c["ct"][J]) * hQ
    l_dphi = -0.5 * dt * c["b"][J] * hP + 0.5 * dt * cj(c["mr"][J]) * hQ
    l_dpi = 0.5 * dt * c["b"][J] * hQ
    if source is not None:
        F = source.field(2 * n, g.rs_half, g.th, 1.0)[J]
        dA += float(np.real(np.sum(np.conj(hQ) * 0.5 * dt * F)))
    out_phi[:, :-1] += 0.5 * l_pbar
    out_phi[:, 1:] += 0.5 * l_pbar
    out_pi[:, :-1] += 0.5 * l_qbar
    out_pi[:, 1:] += 0.5 * l_qbar
    out_phi[J, 1:] += l_dphi / hr
    out_phi[J, :-1] -= l_dphi / hr
    out_pi[J, 1:] += l_dpi / hr
    out_pi[J, :-1] -= l_dpi / hr
    return out_phi, out_pi, dA


def adjoint_evolve(g, gw, nsteps, source=None, lam_phi_N=None, lam_pi_N=None,
                   state_grad=None):
    """Reverse sweep for a loss L(w_1..w_N, u^N [, states]).

    gw[n-1] = dL/dw_n as a complex gradient (dL/dRe + i dL/dIm), n = 1..N.
    lam_*_N: dL/du^N from terms other than the waveform (default zero).
    state_grad(n) -> (gphi, gpi) or None: extra dL/du^n for n = 1..N-1
    (used for losses on intermediate states).
    Returns (dL/dPhi^0, dL/dPi^0, dL/dA) where A is the source amplitude.
    """
    nth, nr = g.nth, g.nr
    lphi = np.zeros((nth, nr), np.complex128) if lam_phi_N is None else np.array(lam_phi_N, np.complex128)
    lpi = np.zeros((nth, nr), np.complex128) if lam_pi_N is None else np.array(lam_pi_N, np.complex128)
    lphi[:, g.i_ext] += gw[nsteps - 1]
    dA = 0.0
    for n in range(nsteps - 1, -1, -1):
        lphi, lpi, d = adjoint_step(g, lphi, lpi, n, source)
        dA += d
        if n >= 1:
            lphi[:, g.i_ext] += gw[n - 1]
            if state_grad is not None:
                sg = state_grad(n)
                if sg is not None:
                    lphi += sg[0]
                    lpi += sg[1]
    return lphi, lpi, dA


def waveform_loss(w, y):
    """L = sum_n sum_j |w_n[j] - y_n[j]|^2 and its complex gradient 2(w - y)."""
    d = w - y
    return float(np.sum(np.abs(d) ** 2)), 2.0 * d


def assemble_step_matrix(g):
    """Dense complex matrix of the homogeneous step on a tiny grid, built
    column by column from unit inputs (brute force, for checking the
    adjoint).  Flattening is (Phi rows, then Pi rows), row-major [j][i]."""
    nth, nr = g.nth, g.nr
    npt = nth * nr
    G = np.zeros((2 * npt, 2 * npt), dtype=np.complex128)
    for k in range(2 * npt):
        e = np.zeros(2 * npt, dtype=np.complex128)
        e[k] = 1.0
        phi = e[:npt].reshape(nth, nr)
        pi = e[npt:].reshape(nth, nr)
        p1, q1 = step(g, phi, pi, 0)
        G[:, k] = np.concatenate([p1.ravel(), q1.ravel()])
    return G


# ---------------------------------------------------------------------------
# Energy, momentum and angular momentum carried off by the extracted waves
# ---------------------------------------------------------------------------

def radiated_flux(ms, waves, dt, hth):
    """Radiated energy, linear momentum and z angular momentum, per unit time
    and accumulated, from the extracted waveforms of several m modes.

    Sec. 3.2 (closing paragraph, and the figure of the recoil) describes the
    waves as carrying energy, linear and angular momentum away from the
    binary; it prints no formula.  The standard ones are used (Newman-Penrose
    psi_4 at large r; e.g. Ruiz, Alcubierre, Nunez & Takahashi 2008): with
    r psi_4 -> sum_m Phi_m(t, theta) e^{i m phi} (for s = -2, Psi = rho^-4 psi_4
    and the ansatz Psi = e^{i m phi~} r^3 Phi), H = int_0^t r psi_4 dt' and
    K = int_0^t H dt',

      dE/dt          = (1/4pi) oint |H|^2 dOmega
      dP_z/dt        = (1/4pi) oint cos(theta) |H|^2 dOmega
      d(P_x+iP_y)/dt = (1/4pi) oint sin(theta) e^{i phi} |H|^2 dOmega
      dJ_z/dt        = -(1/4pi) Re oint conj(H) d_phi K dOmega.

    The phi integrals are done exactly on the Fourier modes:
      dE/dt = 1/2 sum_m int |H_m|^2 sin,  dP_z/dt = 1/2 sum_m int |H_m|^2 cos sin,
      d(P_x+iP_y)/dt = 1/2 sum_m int H_m conj(H_{m+1}) sin^2,
      dJ_z/dt = 1/2 sum_m m Im int conj(H_m) K_m sin.
    Time integrals by the trapezoidal rule from t = 0, theta integrals by the
    trapezoidal rule on the grid's rows (both poles included).

    ms: the m of each waveform (distinct); waves[k]: (N+1, nth) complex,
    row n = Phi at the extraction column at t = n dt (n = 0 is the initial
    state).  Returns (N+1, 10) real: dE/dt, dP_x/dt, dP_y/dt, dP_z/dt,
    dJ_z/dt, then E, P_x, P_y, P_z, J_z accumulated by the trapezoidal rule
    (the recoil velocity is -P/M for a final mass M)."""
    waves = [np.asarray(w, dtype=np.complex128) for w in waves]
    nt, nth = waves[0].shape
    th = np.arange(nth) * hth
    wq = np.full(nth, hth)             # trapezoid weights in theta
    wq[0] = wq[-1] = 0.5 * hth

    def tint(f):                       # cumulative trapezoid in t along axis 0
        out = np.zeros_like(f)
        out[1:] = np.cumsum(0.5 * dt * (f[1:] + f[:-1]), axis=0)
        return out

    H = {m: tint(w) for m, w in zip(ms, waves)}
    K = {m: tint(H[m]) for m in ms}
    sin, cos = np.sin(th), np.cos(th)
    dE = sum(0.5 * (np.abs(H[m]) ** 2) @ (wq * sin) for m in ms)
    dPz = sum(0.5 * (np.abs(H[m]) ** 2) @ (wq * cos * sin) for m in ms)
    dPxy = np.zeros(nt, dtype=np.complex128)
    for m in ms:
        if m + 1 in H:
            dPxy += 0.5 * (H[m] * np.conj(H[m + 1])) @ (wq * sin * sin)
    dJz = sum(0.5 * m * np.imag((np.conj(H[m]) * K[m]) @ (wq * sin)) for m in ms)
    rates = np.stack([dE, dPxy.real, dPxy.imag, dPz, dJz], axis=1)
    return np.concatenate([rates, tint(rates)], axis=1)
