// Host-side geometry: tortoise inversion and coefficient tables.
// See geometry.h for the factorisation of the coefficient fields.
#include <cmath>
#include <string>

#include "geometry.h"

namespace teuk {

namespace {

struct Horizon {
    double rp, rm, A, B, ln2M;
};

Horizon horizon(double M, double a) {
    Horizon h;
    const double d = std::sqrt(M * M - a * a);
    h.rp = M + d;
    h.rm = M - d;
    h.A = 2.0 * M * h.rp / (h.rp - h.rm);
    h.B = 2.0 * M * h.rm / (h.rp - h.rm);
    h.ln2M = std::log(2.0 * M);
    return h;
}

// r* as a function of y = ln x, and its derivative dr*/dy = q/(r - r_-).
inline double rstar_y(double y, double M, const Horizon& h) {
    const double x = std::exp(y);
    return h.rp + x + h.A * (y - h.ln2M) - h.B * std::log((x + h.rp - h.rm) / (2.0 * M));
}

inline double drstar_dy(double y, double a, const Horizon& h) {
    const double x = std::exp(y);
    const double r = h.rp + x;
    return (r * r + a * a) / (x + h.rp - h.rm);
}

}  // namespace

double tortoise_of_x(double x, double M, double a) {
    const Horizon h = horizon(M, a);
    return rstar_y(std::log(x), M, h);
}

double x_of_tortoise(double rs, double M, double a) {
    const Horizon h = horizon(M, a);
    // bracket in y; r*(y) is strictly increasing
    double lo = -740.0, hi = std::log(std::fabs(rs) + 10.0 * M) + 2.0;
    while (rstar_y(hi, M, h) < rs) hi += 1.0;
    // initial guess: horizon side r* ~ r_+ + A (y - ln 2M) + const; far side x ~ r* - r_+
    double y;
    if (rs < h.rp + 2.0 * M) {
        y = (rs - h.rp + h.B * std::log((h.rp - h.rm) / (2.0 * M))) / h.A + h.ln2M;
    } else {
        y = std::log(rs - h.rp);
    }
    if (!(y > lo && y < hi)) y = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        const double f = rstar_y(y, M, h) - rs;
        if (f > 0) hi = y; else lo = y;
        double yn = y - f / drstar_dy(y, a, h);
        if (!(yn > lo && yn < hi)) yn = 0.5 * (lo + hi);   // keep inside the bracket
        const double dy = yn - y;
        y = yn;
        if (std::fabs(dy) <= 1e-16 * std::fmax(1.0, std::fabs(y))) break;
    }
    return std::exp(y);
}

std::string build_geometry(double M, double a, int s, int m, int nr, int nth,
                           double rs_min, double rs_max, double cfl, double rs_extract,
                           Geometry& G) {
    if (!(M > 0.0) || !(std::fabs(a) < M)) return "need M > 0 and |a| < M";
    if (s < -2 || s > 2) return "spin weight s must be in -2..2";
    if (nr < 5 || nth < 7) return "need nr >= 5 and nth >= 7";
    // the per-row kernels (initial data, finiteness check) launch one block
    // row per theta row, and a launch has at most 65535 of them
    if (nth > 65535) return "need nth <= 65535";
    if (!(rs_max > rs_min)) return "need rs_max > rs_min";
    if (!(cfl > 0.0 && cfl <= 1.0)) return "need 0 < cfl <= 1";
    const Horizon h = horizon(M, a);
    G.M = M; G.a = a; G.s = s; G.m = m; G.nr = nr; G.nth = nth;
    G.rs_min = rs_min; G.rs_max = rs_max;
    G.h_r = (rs_max - rs_min) / (nr - 1);
    G.h_th = M_PI / (nth - 1);
    G.r_plus = h.rp; G.r_minus = h.rm;
    const long ie = std::lround((rs_extract - rs_min) / G.h_r);
    if (ie < 0 || ie >= nr) return "extraction radius outside the grid";
    G.i_ext = static_cast<int>(ie);

    G.rnode.assign(static_cast<size_t>(RF_COUNT) * nr, 0.0);
    G.rhalf.assign(static_cast<size_t>(RF_COUNT) * nr, 0.0);
    auto fill = [&](std::vector<double>& tab, int idx, double rs) {
        const double x = x_of_tortoise(rs, M, a);
        const double r = h.rp + x;
        const double Delta = x * (x + h.rp - h.rm);
        const double dDelta = 2.0 * (r - M);
        const double q = r * r + a * a;
        double* col = tab.data();
        auto set = [&](RField f, double v) { col[static_cast<size_t>(f) * nr + idx] = v; };
        set(RF_Q, q);
        set(RF_Q2, q * q);
        set(RF_A2D, a * a * Delta);
        set(RF_DELTA, Delta);
        // c_t numerator: 2s(r Delta - M(r^2 - a^2)) + i(4 M a m r + 2 s a Delta cos),
        // with r Delta - M(r^2 - a^2) = r^2 (r - 3M) + a^2 (r + M)
        const double ct_re = 2.0 * s * (r * r * (r - 3.0 * M) + a * a * (r + M));
        set(RF_CT_RE, ct_re);
        set(RF_CT_I0, 4.0 * M * a * m * r);
        set(RF_CT_I1, 2.0 * s * a * Delta);
        // C_0 numerator: (3 Delta/r^2)(2 Delta + (1+s) r Delta') + i(2 m a s Delta' + 6 m a Delta / r),
        // with 2 Delta + (1+s) r Delta' = 2(2+s) r^2 - 2(3+s) M r + 2 a^2
        // C_0 numerators, halved (see ThetaRow)
        set(RF_C0_RE, 0.5 * ((3.0 * Delta / (r * r)) * (2.0 * (2.0 + s) * r * r - 2.0 * (3.0 + s) * M * r + 2.0 * a * a)));
        set(RF_C0_IM, 0.5 * (2.0 * m * a * s * dDelta + 6.0 * m * a * Delta / r));
        // m_r = b c_t + C_r - b d_r* b collected over Sigma^4:
        //   Re: q^2 Delta [4(s+2) r + 6 a^2/r] - a^2 Delta sin^2 [q ct_re/(q + Sigma) + q((s+1/2) Delta' + 6 Delta/r)]
        //   Im: b Im(c_t) + 2 m a q / Sigma^2
        set(RF_MR_P, q * q * Delta * (4.0 * (s + 2.0) * r + 6.0 * a * a / r));
        set(RF_MR_B, 2.0 * m * a * q);
        set(RF_MR_K1, q * ct_re);
        set(RF_MR_K2, q * ((s + 0.5) * dDelta + 6.0 * Delta / r));
        set(RF_RS, rs);
    };
    for (int i = 0; i < nr; ++i) fill(G.rnode, i, rs_min + i * G.h_r);
    for (int i = 0; i < nr - 1; ++i) fill(G.rhalf, i, rs_min + i * G.h_r + 0.5 * G.h_r);

    const double r0 = h.rp + x_of_tortoise(rs_min, M, a);
    G.dt = cfl * std::fmin(G.h_r, r0 * G.h_th);

    G.rows.assign(nth, ThetaRow{});
    const double hh = G.h_th;
    const int p = std::abs(m + s), qq = std::abs(m - s);
    for (int j = 0; j < nth; ++j) {
        ThetaRow& R = G.rows[j];
        const double th = j * hh;
        R.theta = th;
        R.inv_2h2 = 0.5 * (1.0 / (hh * hh));
        R.cos_th = std::cos(th);
        const double sn = std::sin(th);
        R.sin2 = sn * sn;
        if (j > 0 && j < nth - 1) {
            const double cot = R.cos_th / sn;
            const double V = (m + s * R.cos_th) * (m + s * R.cos_th) / (sn * sn) - s;
            R.cot4h = 0.5 * (cot / (2.0 * hh));
            R.V2 = 0.5 * V;
        }
        R.prof = std::pow(2.0, 0.5 * (p + qq)) * std::pow(std::sin(0.5 * th), p) *
                 std::pow(std::cos(0.5 * th), qq);
    }
    return std::string();
}

}  // namespace teuk
