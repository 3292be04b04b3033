// Device point updates of the two-step Lax-Wendroff iteration (Sec. 3.2,
// Eqs. (lw1) and (lw2)).  Every GPU variant (single step, temporally
// blocked, batched) evaluates a point through these functions and nothing
// else, so their results are bitwise identical.  The file is compiled with
// -ffp-contract=off: every fused multiply-add below is written out.
#pragma once

#include <hip/hip_runtime.h>

#include "geometry.h"

namespace teuk {

// Radial record of one column (node or half node), see geometry.h.
struct RCol {
    double q, q2, a2d, delta, ct_re, ct_i0, ct_i1, c0_re, c0_im, mr_p, mr_b, mr_k1, mr_k2;
};

__device__ __forceinline__ RCol load_rcol(const double* __restrict__ tab, int pitch, int i) {
    RCol r;
    r.q = tab[RF_Q * pitch + i];
    r.q2 = tab[RF_Q2 * pitch + i];
    r.a2d = tab[RF_A2D * pitch + i];
    r.delta = tab[RF_DELTA * pitch + i];
    r.ct_re = tab[RF_CT_RE * pitch + i];
    r.ct_i0 = tab[RF_CT_I0 * pitch + i];
    r.ct_i1 = tab[RF_CT_I1 * pitch + i];
    r.c0_re = tab[RF_C0_RE * pitch + i];
    r.c0_im = tab[RF_C0_IM * pitch + i];
    r.mr_p = tab[RF_MR_P * pitch + i];
    r.mr_b = tab[RF_MR_B * pitch + i];
    r.mr_k1 = tab[RF_MR_K1 * pitch + i];
    r.mr_k2 = tab[RF_MR_K2 * pitch + i];
    return r;
}

// x^(-1/2) for a positive normal x: the hardware estimate y refined by one
// second-order step of the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ...,
// e = 1 - x y^2.  (The library rsqrt adds a class test for 0, inf and NaN;
// the arguments here never are.)
__device__ __forceinline__ double rsqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// 1/x for a positive normal x: the hardware estimate refined by two
// Newton-Raphson steps r <- r + r (1 - x r) (within an ulp or two of the
// rounded quotient; the IEEE division adds scaling and a final correction).
__device__ __forceinline__ double recip_pos(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// Coefficient fields at one point.
struct Coef {
    double b, w;
    double2 ct, mr, c0;
};

// b = q g, w = Delta g^2, c_t, C_0 = numerators g^2, g = 1/Sigma (the C_0
// numerators, and so c.c0, are stored halved: see ThetaRow),
// Re m_r = [mr_p - a^2 Delta sin^2 (mr_k1/(q + Sigma) + mr_k2)] g^4,
// Im m_r = b Im c_t + mr_b g^2.  For a = 0 the bracket's second term is zero
// and the division is skipped; kerr (a != 0) is the same for every point of
// a grid, so the test is a uniform branch.  (Where a^2 Delta is 0 with
// a != 0 the term is an exact signed zero, so both forms agree bitwise.)
__device__ __forceinline__ Coef coef_at(const RCol& r, double cos_th, double sin2, bool kerr) {
    const double sig2 = fma(-r.a2d, sin2, r.q2);
    const double g = rsqrt_pos(sig2);
    const double g2 = g * g;
    const double g4 = g2 * g2;
    Coef c;
    c.b = r.q * g;
    c.w = r.delta * g2;
    c.ct.x = r.ct_re * g2;
    c.ct.y = fma(r.ct_i1, cos_th, r.ct_i0) * g2;
    c.c0.x = r.c0_re * g2;
    c.c0.y = r.c0_im * g2;
    double num = r.mr_p;
    if (kerr) {
        const double inv_qs = recip_pos(fma(sig2, g, r.q));   // 1/(q + Sigma), Sigma = Sigma^2 g
        num = fma(-r.a2d * sin2, fma(r.mr_k1, inv_qs, r.mr_k2), num);
    }
    c.mr.x = num * g4;
    c.mr.y = fma(c.b, c.ct.y, r.mr_b * g2);
    return c;
}

__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_scale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
// v where keep holds, else zero (component selects: a select of the whole
// pair can be lowered through a private-memory array).
__device__ __forceinline__ double2 masked(bool keep, double2 v) {
    return make_double2(keep ? v.x : 0.0, keep ? v.y : 0.0);
}

// One point of either half of the iteration.  Inputs are column sums and
// differences of the level being differenced (u^n for the half step, the
// half-step values for the full step) at rows j-1, j, j+1:
//   sPm, sP0, sPp : Phi_left + Phi_right   (rows j-1, j, j+1)
//   sQ0           : Pi_left + Pi_right     (row j)
//   dP0, dQ0      : right - left           (row j)
// With averages Phi~ = sP/2, Pi~ = sQ0/2 and differences dPhi = dP0/h_r,
// dPi = dQ0/h_r (the halvings of the C_0 and angular terms sit in the
// halved c.c0 and angular weights):
//   S_Pi  = -c_t Pi~ + m_r dPhi + C_0 Phi~ + w Ang_h[Phi~] + F
//   Phi'  = basePhi + tau (Pi~ - b dPhi)          (S_Phi = Pi~, D = diag(b, -b))
//   Pi'   = basePi  + tau (b dPi + S_Pi)
// Half step (lw1): tau = dt/2, base = (Phi~, Pi~).  Full step (lw2): tau = dt,
// base = u^n at the node.  Ang_h[f]_j = (f_{j+1} - 2 f_j + f_{j-1})/h^2
// + cot (f_{j+1} - f_{j-1})/(2h) - V f_j, differences taken first (the
// second difference of a smooth field is small; weighting first would cancel).
__device__ __forceinline__ void lw_point(const Coef& c, const ThetaRow& R,
                                         double2 sPm, double2 sP0, double2 sPp, double2 sQ0,
                                         double2 dP0, double2 dQ0, double2 F,
                                         double tau, double inv_hr,
                                         double2 basePhi, double2 basePi,
                                         double2& outPhi, double2& outPi) {
    const double2 Q = c_scale(0.5, sQ0);
    const double2 dP = c_scale(inv_hr, dP0);
    const double2 dQ = c_scale(inv_hr, dQ0);
    double2 ang;
    {
        // 2 sP0 is exact, so the fma rounds as the subtraction would
        const double d2x = fma(-2.0, sP0.x, sPp.x) + sPm.x, d2y = fma(-2.0, sP0.y, sPp.y) + sPm.y;
        const double d1x = sPp.x - sPm.x, d1y = sPp.y - sPm.y;
        ang.x = fma(-R.V2, sP0.x, fma(R.cot4h, d1x, d2x * R.inv_2h2));
        ang.y = fma(-R.V2, sP0.y, fma(R.cot4h, d1y, d2y * R.inv_2h2));
    }
    double2 S;
    S.x = fma(c.w, ang.x, F.x);
    S.y = fma(c.w, ang.y, F.y);
    // -c_t Pi~
    S.x = fma(-c.ct.x, Q.x, S.x);
    S.x = fma(c.ct.y, Q.y, S.x);
    S.y = fma(-c.ct.x, Q.y, S.y);
    S.y = fma(-c.ct.y, Q.x, S.y);
    // + m_r dPhi
    S.x = fma(c.mr.x, dP.x, S.x);
    S.x = fma(-c.mr.y, dP.y, S.x);
    S.y = fma(c.mr.x, dP.y, S.y);
    S.y = fma(c.mr.y, dP.x, S.y);
    // + C_0 Phi~ = (C_0 / 2) sP0
    S.x = fma(c.c0.x, sP0.x, S.x);
    S.x = fma(-c.c0.y, sP0.y, S.x);
    S.y = fma(c.c0.x, sP0.y, S.y);
    S.y = fma(c.c0.y, sP0.x, S.y);
    outPhi.x = fma(tau, fma(-c.b, dP.x, Q.x), basePhi.x);
    outPhi.y = fma(tau, fma(-c.b, dP.y, Q.y), basePhi.y);
    outPi.x = fma(tau, fma(c.b, dQ.x, S.x), basePi.x);
    outPi.y = fma(tau, fma(c.b, dQ.y, S.y), basePi.y);
}

// Fourth theta-difference dissipation added in the full step:
// out -= (eps/16) (u_{j+2} - 4u_{j+1} + 6u_j - 4u_{j-1} + u_{j-2}).
__device__ __forceinline__ double2 ko_apply(double2 out, double ko_c, double2 um2, double2 um1,
                                            double2 u0, double2 up1, double2 up2) {
    double2 d;
    d.x = fma(-4.0, up1.x + um1.x, fma(6.0, u0.x, up2.x + um2.x));
    d.y = fma(-4.0, up1.y + um1.y, fma(6.0, u0.y, up2.y + um2.y));
    return make_double2(fma(-ko_c, d.x, out.x), fma(-ko_c, d.y, out.y));
}

// Pole rows from the boundary condition: (4 u_1 - u_2)/3 (even |m|), 0 (odd |m|).
// The third is a multiplication by the rounded 1/3 (a division would expand
// into a long instruction sequence).
__device__ __forceinline__ double2 pole_value(bool even, double2 u1, double2 u2) {
    if (!even) return make_double2(0.0, 0.0);
    const double third = 0.33333333333333331483;   // nearest double to 1/3
    return make_double2(fma(4.0, u1.x, -u2.x) * third, fma(4.0, u1.y, -u2.y) * third);
}

// Synthetic source value at (t, r*, theta): amplitude G_r G_th e^{-i m phi~_p}.
__device__ __forceinline__ double gauss_cut(double x, double sig, double cut) {
    if (fabs(x) > cut * sig) return 0.0;
    return exp(-x * x / (2.0 * sig * sig)) / (2.5066282746310002 * sig);
}

}  // namespace teuk
