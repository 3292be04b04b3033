// Orbit tables for the synthetic point-particle source: bound prograde
// equatorial Kerr geodesics sampled at uniform coordinate time, in the
// coordinates of Sec. 3.2 (tortoise r*, azimuth phi~ with
// d phi~ = d phi + a/Delta dr).  Host code.
#include <cmath>
#include <vector>

#include "ctx.h"
#include "geometry.h"
#include "teuk.h"

namespace {

using teuk_detail::fail;

// Lengths and times in units of M.
struct Equatorial {
    double a, p, e;
    double E, x, beta, r3;   // energy, x = L - a E, beta = 1 - E^2, third root of R(r)/r
};

// Constants of the orbit with turning points p/(1+e) and p/(1-e).  With
// Carter constant 0, R(r)/r = (E^2-1) r^3 + 2 r^2 - (a^2 + x^2 + 2 a x E) r + 2 x^2,
// and matching its roots to p/(1 +- e) and r3 gives
//   1 - E^2 = (1-e^2)/p (1 - x^2 (1-e^2)/p^2),   r3 = 2/(1-E^2) - 2p/(1-e^2),
//   2 a x E = p - a^2 - x^2 (p - 3 - e^2)/p.
// Squaring the last one leaves a quadratic F X^2 + N X + C = 0 in X = x^2
// (the form of Glampedakis and Kennefick 2002, multiplied by p^3); the
// prograde orbit is the root whose unsquared relation holds with x > 0.
bool equatorial_constants(double a, double p, double e, Equatorial& o) {
    const double u = 1.0 - e * e;
    const double q = p - 3.0 - e * e;
    const double F = p * q * q - 4.0 * a * a * u * u;
    const double N = -2.0 * p * p * (p * p - (3.0 + e * e - a * a) * p + a * a * (1.0 + 3.0 * e * e));
    const double C = p * p * p * (p - a * a) * (p - a * a);
    if (!(F > 0.0) || !(N < 0.0)) return false;
    double disc = N * N - 4.0 * F * C;
    if (disc < 0.0) {
        if (disc < -1e-12 * N * N) return false;
        disc = 0.0;   // a = 0: a double root, up to rounding
    }
    const double sq = std::sqrt(disc);
    const double X[2] = {2.0 * C / (-N + sq), (-N + sq) / (2.0 * F)};
    double best = INFINITY;
    for (double Xc : X) {
        const double beta = u / p * (1.0 - Xc * u / (p * p));
        if (!(Xc > 0.0) || !(beta > 0.0) || !(beta < 1.0)) continue;
        const double E = std::sqrt(1.0 - beta);
        const double x = std::sqrt(Xc);
        const double res = std::fabs(2.0 * a * x * E - (p - a * a - Xc * q / p));
        if (res < best) {
            best = res;
            o = Equatorial{a, p, e, E, x, beta, 2.0 / beta - 2.0 * p / u};
        }
    }
    if (!(best <= 1e-9 * p)) return false;
    return o.r3 < p / (1.0 + e);   // bound and stable: r3 below the periapsis
}

// dt/dchi and dphi/dchi on r = p/(1 + e cos chi):
//   r^2 dt/dtau = a x + (r^2+a^2) P/Delta,   r^2 dphi/dtau = x + a P/Delta,
//   P = E(r^2+a^2) - a L = E r^2 - a x,
//   dtau/dchi = r^2 sqrt(1-e^2) / ((1 + e cos chi) sqrt((1-E^2) r (r - r3)))
// (R = (1-E^2) r (r_a - r)(r - r_p)(r - r3), and dr/dchi divided by
// sqrt((r_a - r)(r - r_p)) is sqrt(1-e^2)/(1 + e cos chi)).
void rates(const Equatorial& o, double chi, double& vt, double& vphi) {
    const double den = 1.0 + o.e * std::cos(chi);
    const double r = o.p / den;
    const double delta = r * r - 2.0 * r + o.a * o.a;
    const double P = o.E * r * r - o.a * o.x;
    const double dtau = r * r * std::sqrt(1.0 - o.e * o.e) / (den * std::sqrt(o.beta * r * (r - o.r3)));
    vt = (o.a * o.x + (r * r + o.a * o.a) * P / delta) / (r * r) * dtau;
    vphi = (o.x + o.a * P / delta) / (r * r) * dtau;
}

// A smooth even 2 pi-periodic rate V(chi) = A0 + sum_k A_k cos(k chi) and
// its integral.  The coefficients come from the trapezoidal rule on kNq
// points, which for an analytic periodic V converges geometrically (the
// nearest complex singularity, 1 + e cos chi = 0, gives |A_k| ~
// ((1 - sqrt(1-e^2))/e)^k: below 1e-16 of A0 after 28 terms at e = 0.5).
struct CosSeries {
    static constexpr int kNq = 256;
    double a0 = 0.0;
    std::vector<double> ak;   // ak[k-1] = A_k, k = 1..K

    void fit(const double* v) {
        std::vector<double> cs(kNq);
        for (int j = 0; j < kNq; ++j) cs[j] = std::cos(2.0 * M_PI * j / kNq);
        double s = 0.0;
        for (int j = 0; j < kNq; ++j) s += v[j];
        a0 = s / kNq;
        std::vector<double> c(kNq / 2);
        int K = 0;
        for (int k = 1; k < kNq / 2; ++k) {
            double acc = 0.0;
            for (int j = 0; j < kNq; ++j) acc += v[j] * cs[(k * j) % kNq];
            c[k - 1] = 2.0 * acc / kNq;
            // terms below the rounding of A0 are noise of the quadrature
            if (std::fabs(c[k - 1]) > 1e-16 * std::fabs(a0)) K = k;
        }
        ak.assign(c.begin(), c.begin() + K);
    }
    // integral from 0: A0 chi + sum A_k sin(k chi)/k, and the rate itself
    void eval(double chi, double& integral, double& rate) const {
        const double s1 = std::sin(chi), c1 = std::cos(chi);
        double sk = s1, ck = c1, I = a0 * chi, V = a0;
        for (size_t k = 1; k <= ak.size(); ++k) {
            I += ak[k - 1] * sk / static_cast<double>(k);
            V += ak[k - 1] * ck;
            const double sn = sk * c1 + ck * s1;
            ck = ck * c1 - sk * s1;
            sk = sn;
        }
        integral = I;
        rate = V;
    }
};

}  // namespace

int teuk_orbit_eccentric(double M, double a, double p, double e, double chi0, double dt, int64_t nsamples,
                         double* out) {
    if (out == nullptr || nsamples < 0) return fail(TEUK_EINVAL, "bad orbit output");
    if (!(M > 0.0) || !(std::fabs(a) < M)) return fail(TEUK_EINVAL, "need M > 0 and |a| < M");
    if (!(e >= 0.0 && e <= 0.9)) return fail(TEUK_EINVAL, "eccentricity must be in [0, 0.9]");
    if (!(dt > 0.0) || !std::isfinite(chi0) || !std::isfinite(p)) return fail(TEUK_EINVAL, "bad dt, p or chi0");
    Equatorial o{};
    if (!equatorial_constants(a / M, p / M, e, o))
        return fail(TEUK_EINVAL, "no bound stable prograde equatorial orbit with this p and e");

    const int nq = CosSeries::kNq;
    std::vector<double> vt(nq), vp(nq);
    for (int j = 0; j < nq; ++j) rates(o, 2.0 * M_PI * j / nq, vt[j], vp[j]);
    CosSeries T, Ph;
    T.fit(vt.data());
    Ph.fit(vp.data());

    const double ah = a / M;
    const double rp = 1.0 + std::sqrt(1.0 - ah * ah), rm = 1.0 - std::sqrt(1.0 - ah * ah);
    auto shift = [&](double r) { return ah / (rp - rm) * std::log((r - rp) / (r - rm)); };
    double t0, ph0, rate;
    T.eval(chi0, t0, rate);
    Ph.eval(chi0, ph0, rate);
    const double h = 0.5 * dt / M;
    double chi = chi0, shift0 = 0.0;
    for (int64_t k = 0; k < nsamples; ++k) {
        const double tk = static_cast<double>(k) * h;
        if (k > 0) {
            // Newton on t(chi) = tk from the previous sample (t is increasing)
            double I, V;
            T.eval(chi, I, V);
            chi += h / V;
            // Newton converges quadratically; it is done once the step is at
            // the rounding level of the residual, or stops shrinking there
            bool done = false;
            double dprev = INFINITY;
            for (int it = 0; it < 40 && !done; ++it) {
                T.eval(chi, I, V);
                const double d = (I - t0 - tk) / V;
                chi -= d;
                const double tol = 1e-15 * (std::fabs(chi) + (std::fabs(I) + std::fabs(t0) + tk) / V);
                done = std::fabs(d) <= tol || (std::fabs(d) >= 0.5 * dprev && std::fabs(d) <= 64.0 * tol);
                dprev = std::fabs(d);
            }
            if (!done) return fail(TEUK_EINVAL, "orbit time inversion did not converge");
        }
        double phi, V;
        Ph.eval(chi, phi, V);
        const double r = o.p / (1.0 + e * std::cos(chi));   // units of M
        if (k == 0) shift0 = shift(r);
        out[3 * k + 0] = teuk::tortoise_of_x((r - rp) * M, M, a);
        out[3 * k + 1] = 0.5 * M_PI;
        out[3 * k + 2] = (phi - ph0) + shift(r) - shift0;
    }
    return TEUK_OK;
}
