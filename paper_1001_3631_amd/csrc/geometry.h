// Host-side geometry and coefficient tables of the m-mode Teukolsky system.
//
// The coefficient fields of the first-order system d_t u + D d_r* u = S
// (Sec. 3.2; derived from Eq. (1) of Sec. 3.1 with the tortoise coordinate,
// the azimuth phi~ and Psi = e^{i m phi~} r^3 Phi) depend on (r, theta) only
// through radial functions and Sigma^2 = (r^2+a^2)^2 - a^2 Delta sin^2(theta).
// With g = 1/Sigma:
//   b   = q g                                   (q = r^2 + a^2)
//   w   = Delta g^2
//   c_t = [ct_re + i (ct_i0 + ct_i1 cos)] g^2
//   C_0 = [c0_re + i c0_im] g^2   (the record holds half of c0_re, c0_im)
//   Re m_r = [mr_p - a^2 Delta sin^2 (mr_k1/(q + Sigma) + mr_k2)] g^4
//   Im m_r = b Im c_t + mr_b g^2
// so the device keeps one radial record per node / half node and one angular
// record per row, and forms the 2D fields on the fly.  The numerators are
// written in expanded forms that do not cancel: m_r vanishes identically for
// a = 0, s = -2, and cancellation residue there is amplified by the evolution.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace teuk {

// Fields of one radial record (struct-of-arrays on the device, in this order).
enum RField {
    RF_Q = 0, RF_Q2, RF_A2D, RF_DELTA, RF_CT_RE, RF_CT_I0, RF_CT_I1,
    RF_C0_RE, RF_C0_IM, RF_MR_P, RF_MR_B, RF_MR_K1, RF_MR_K2, RF_RS,
    RF_COUNT
};

// One angular record per row (array-of-structs, 8 doubles = 64 bytes).
// Pole rows (j = 0, nth-1) leave cot4h and V2 at zero: they are never evolved.
// The angular operator's weights are stored halved, and so is C_0 in the
// radial record: the stencil applies them to column sums (twice the
// averages), and scaling by a power of two commutes with rounding, so the
// products are the same numbers without the multiplications by 1/2.
struct ThetaRow {
    double cos_th;   // cos(theta_j)
    double sin2;     // sin^2(theta_j)
    double cot4h;    // cot(theta_j) / (4 h_th), half the first-difference weight
    double V2;       // half the angular potential ((m + s cos)^2 / sin^2 - s) / 2
    double inv_2h2;  // 1 / (2 h_th^2), half the second-difference weight
    double theta;    // theta_j
    double prof;     // initial angular profile P(theta_j)
    double pad;      // keeps the record at 64 bytes
};

struct Geometry {
    double M, a;
    int s, m;
    int nr, nth;
    double rs_min, rs_max, h_r, h_th, dt;
    double r_plus, r_minus;
    int i_ext;
    // radial tables: field-major, nodes have nr entries, half points nr-1
    std::vector<double> rnode;   // RF_COUNT * nr
    std::vector<double> rhalf;   // RF_COUNT * (nr - 1)  (stored with pitch nr)
    std::vector<ThetaRow> rows;  // nth
};

// r*(x) with x = r - r_+ (integral of dr*/dr = (r^2+a^2)/Delta).
double tortoise_of_x(double x, double M, double a);
// Inverse: x(r*) by safeguarded Newton on y = ln x.
double x_of_tortoise(double rs, double M, double a);

// Build everything; returns an empty string on success, else a message.
std::string build_geometry(double M, double a, int s, int m, int nr, int nth,
                           double rs_min, double rs_max, double cfl, double rs_extract,
                           Geometry& G);

}  // namespace teuk
