// Device helpers shared by the stepping kernels: wave shifts, the source
// window test, the XCD-aware work-item order, and stream_level, one level
// of the streaming Lax-Wendroff stencil (Sec. 3.2, Eqs. (lw1), (lw2)) used
// by the temporally blocked and batched kernels.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "lw_point.h"

namespace teuk {

// Rows of u^n the single-step kernel fetches ahead of their use.
#ifndef TEUK_PREFETCH_ROWS
#define TEUK_PREFETCH_ROWS 2
#endif
constexpr int kPrefetchRows = TEUK_PREFETCH_ROWS;

namespace {

// Cross-lane moves with DPP wave shifts (no LDS traffic): from_next gives lane
// l the value of lane l+1 (lane 63 gets zero), from_prev the value of lane
// l-1 (lane 0 gets zero).  Lanes 0 and 63 are halo lanes whose results are
// never stored, so the fill value is free; zero fill (bound_ctrl) needs no
// copy of the old value in front of each move.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double2 from_next(double2 v) {
    return make_double2(dpp_move<0x130>(v.x), dpp_move<0x130>(v.y));   // wave_shl:1
}
__device__ __forceinline__ double2 from_prev(double2 v) {
    return make_double2(dpp_move<0x138>(v.x), dpp_move<0x138>(v.y));   // wave_shr:1
}

// A pointer that reaches a kernel through memory (an instance table) rather
// than as an argument is generic to the compiler: loads and stores through it
// become flat instructions, which also count against the scalar-memory
// counter, so each wait for an angular record (a scalar load) would also wait
// for every row in flight.  Rebuilding the pointer in the global address
// space (device pass only; the address is the same) makes them global
// instructions.
template <typename T>
__device__ __forceinline__ T* global_ptr(T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
    using G = __attribute__((address_space(1))) T*;
    return (T*)(G)(reinterpret_cast<unsigned long long>(p));
#else
    return p;
#endif
}

// The same for a table that nothing writes while the kernel runs (the
// angular records), rebuilt in the constant address space: its wave-uniform
// reads become scalar loads even after the kernel's own stores, which the
// compiler cannot otherwise rule out as aliasing it.
template <typename T>
__device__ __forceinline__ const T* constant_ptr(const T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
    using C = __attribute__((address_space(4))) const T*;
    return (const T*)(C)(reinterpret_cast<unsigned long long>(p));
#else
    return p;
#endif
}

// Source value at (col, row) of a window table with origin (c0, r0), zero
// outside it.
__device__ __forceinline__ double2 window_value(const double2* __restrict__ tab, int c0, int r0, int win_r,
                                                int win_t, int col, int row) {
    const unsigned dc = static_cast<unsigned>(col - c0);
    const unsigned dr = static_cast<unsigned>(row - r0);
    if (dc < static_cast<unsigned>(win_r) && dr < static_cast<unsigned>(win_t)) return tab[dr * win_r + dc];
    return make_double2(0.0, 0.0);
}

// Whether the window [c0, c0 + win_r) x [r0, r0 + win_t) meets the columns
// [i0, i0 + 63] and rows [ja, jb] of a wave.  A wave that meets no window of
// its iteration takes the forms of its body without source lookups: a lookup
// is a conditional load, and the wait for its result (which cannot be told
// apart from the wait for every load issued before it) would also wait for
// the rows prefetched ahead, on every row.
__device__ __forceinline__ bool window_meets(int4 org2, bool node, int win_r, int win_t, int i0, int ja,
                                             int jb) {
    const int c0 = node ? org2.z : org2.x;
    const int r0 = node ? org2.w : org2.y;
    return c0 <= i0 + 63 && i0 < c0 + win_r && r0 <= jb && ja < r0 + win_t;
}

// Workgroups are handed to the 8 XCDs round robin; renumber them so that each
// XCD walks a contiguous range of work items (vertically adjacent segments of
// the same column strip share halo rows in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nwg) {
    const int per = nwg / 8;
    const int full = per * 8;
    if (b >= full) return b;
    return (b % 8) * per + (b / 8);
}

}  // namespace

// One level of the streaming stencil: a wave owns 64 columns (lane = column,
// column i = lane + offset) and produces the full-step rows [lo, hi) of one
// Lax-Wendroff iteration, streaming down theta: load input row jj, form the
// half-step row jj-1, then the full-step row jj-2.  Radial neighbours come
// from the adjacent lane; the theta window lives in registers (the loop is
// fully unrolled, NROW >= hi - lo).
//
// Input rows come from the planes P.phi/P.pi or (IN_LDS) from this wave's
// LDS buffer; output rows go to P.phi_out/P.pi_out (owner lanes only) or
// (OUT_LDS) back into the LDS buffer, every lane, in place: row r is read at
// the iteration that loads it and written two iterations later.  Lanes
// outside the grid read zeros and the Dirichlet columns are written as zero,
// so a buffered level feeds the next exactly as a plane would.  Lanes whose
// neighbours lie outside the wave produce values that no owner lane uses.
struct LevelArgs {
    int lo, hi;                    // full-step output rows of this level
    int lane, i;
    int halo;                      // owner lanes are halo .. 63 - halo
    const double2* fh;             // source windows of this iteration (or null)
    const double2* fn;
    int4 org;
    double2* wave;                 // extraction row of this iteration (or null)
    double2* lp;                   // LDS buffer of this wave: rows [lbase, ...) x 64 lanes
    double2* lq;
    int lbase;
};

// Parameters are taken by value: with references the compiler must assume
// that the output stores may alias them and re-reads fields after each store.
// rows is the kernel's __restrict__ argument where it has one (scalar loads).
//
// FAST_ROWS > 0 is the interior form, which the caller may choose when
// hi - lo == FAST_ROWS, lo >= 4, hi <= nth - 2 and every lane is an interior
// column (1 <= i <= nr - 2): every row and half row is then in range and no
// pole or ghost row is touched, so those tests become constants.  SRC adds
// the source lookups (A.fh, A.fn non-null; the caller chooses it when a
// window of the level meets the wave, window_meets).  Without it F = 0,
// which is what a lookup outside the window gives.  The arithmetic on every
// point is the same in all forms.
template <int NROW, bool IN_LDS, bool OUT_LDS, int PREFETCH = kPrefetchRows, int FAST_ROWS = 0, bool SRC = false>
__device__ __forceinline__ void stream_level(const StepParams P, const LevelArgs A, const RCol rn,
                                             const RCol rh, const ThetaRow* __restrict__ rows) {
    constexpr bool FAST = FAST_ROWS > 0;
    static_assert(FAST_ROWS <= NROW, "interior rows exceed the window");
    constexpr int NT = FAST ? FAST_ROWS + 4 : NROW + 4;   // input rows lo-2 .. hi+1
    const int nth = P.nth;
    const int ld = P.ld;
    const int i = A.i;
    const int lane = A.lane;
    const int lo = A.lo, hi = A.hi;
    const bool in_col = (i >= 0) && (i < P.nr);
    const bool owner = in_col && lane >= A.halo && lane <= 63 - A.halo;
    const bool interior_col = (i >= 1) && (i <= P.nr - 2);
    const double2 z = make_double2(0.0, 0.0);
    double2 uP[NROW + 4], uQ[NROW + 4];     // input level, own column, rows lo-2+t
    double2 sP[NROW + 4], sQ[NROW + 4], dP[NROW + 4], dQ[NROW + 4];
    double2 hP[NROW + 4], hQ[NROW + 4];     // half-step values at i+1/2, rows lo-2+t
    double2 gP[NROW + 4], gQ[NROW + 4];     // half-step values at i-1/2 (from lane-1)
    double2 oP1 = z, oQ1 = z;               // full-step row 1 (for the pole row 0)
    double2 oPp = z, oQp = z;               // previous full-step row (for the last pole row)

    double2* const wave = A.wave;
    auto store = [&](int row, double2 vp, double2 vq) {
        if (OUT_LDS) {
            A.lp[(row - A.lbase) * 64 + lane] = vp;
            A.lq[(row - A.lbase) * 64 + lane] = vq;
            if (wave != nullptr && owner && i == P.i_ext) wave[row] = vp;
        } else if (owner) {
            P.phi_out[static_cast<size_t>(row) * ld + i] = vp;
            P.pi_out[static_cast<size_t>(row) * ld + i] = vq;
            if (wave != nullptr && i == P.i_ext) wave[row] = vp;
        }
    };

    // Rows read from the planes are fetched PREFETCH iterations ahead at
    // clamped addresses (as in lw_step_kernel); LDS rows are read in place.
    constexpr int PF = IN_LDS ? 0 : PREFETCH;
    double2 fP[NROW + 4], fQ[NROW + 4];
    const int icl = min(max(i, 0), P.nr - 1);
    auto fetch = [&](int t) {
        const int jc = FAST ? lo - 2 + t : min(max(lo - 2 + t, 0), nth - 1);
        fP[t] = P.phi[static_cast<size_t>(jc) * ld + icl];
        fQ[t] = P.pi[static_cast<size_t>(jc) * ld + icl];
    };
#pragma unroll
    for (int t = 0; t < PF && t < NT; ++t) fetch(t);

    // Angular records: the half step of iteration t uses row lo-3+t, the full
    // step of iteration t the row of the half step of t-1.  Each is read
    // once, one iteration before its first use.
    ThetaRow Rh[NROW + 4];
    auto fetch_row = [&](int t) {
        const int jr = FAST ? lo - 3 + t : min(max(lo - 3 + t, 0), nth - 1);
        Rh[t] = rows[jr];
    };
    if (2 < NT) fetch_row(2);

#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (!IN_LDS && t + PF < NT) fetch(t + PF);
        if (t >= 1 && t + 1 < NT) fetch_row(t + 1);
        const int jj = lo - 2 + t;
        if (FAST || jj <= hi + 1) {
            // ---- row jj of the input level and its column sums/differences ----
            double2 p = z, q = z;
            if (IN_LDS) {
                if (FAST || (jj >= 0 && jj < nth)) {
                    p = A.lp[(jj - A.lbase) * 64 + lane];
                    q = A.lq[(jj - A.lbase) * 64 + lane];
                }
            } else if (FAST || (jj >= 0 && jj < nth && in_col)) {
                p = fP[t];
                q = fQ[t];
            }
            uP[t] = p;
            uQ[t] = q;
            const double2 pN = from_next(p), qN = from_next(q);
            sP[t] = c_add(p, pN);
            sQ[t] = c_add(q, qN);
            dP[t] = c_sub(pN, p);
            dQ[t] = c_sub(qN, q);

            // ---- half step (lw1) at (i+1/2, jh), jh = jj - 1 ----
            if (t >= 2) {
                const int jh = jj - 1;
                hP[t - 1] = z;
                hQ[t - 1] = z;
                if (FAST || (jh >= 1 && jh <= nth - 2)) {
                    const ThetaRow& R = Rh[t];
                    const Coef c = coef_at(rh, R.cos_th, R.sin2, P.kerr != 0);
                    const double2 F = SRC ? window_value(A.fh, A.org.x, A.org.y, P.win_r, P.win_t, i, jh) : z;
                    lw_point(c, R, sP[t - 2], sP[t - 1], sP[t], sQ[t - 1],
                             dP[t - 1], dQ[t - 1], F, 0.5 * P.dt, P.inv_hr, c_scale(0.5, sP[t - 1]),
                             c_scale(0.5, sQ[t - 1]), hP[t - 1], hQ[t - 1]);
                } else if (jh == nth - 1 && t >= 4) {
                    hP[t - 1] = pole_value(P.even, hP[t - 2], hP[t - 3]);
                    hQ[t - 1] = pole_value(P.even, hQ[t - 2], hQ[t - 3]);
                }
                if (!FAST && jh == 2 && t >= 5) {   // pole row 0 of the half step, now that rows 1, 2 exist
                    hP[t - 3] = pole_value(P.even, hP[t - 2], hP[t - 1]);
                    hQ[t - 3] = pole_value(P.even, hQ[t - 2], hQ[t - 1]);
                    gP[t - 3] = from_prev(hP[t - 3]);
                    gQ[t - 3] = from_prev(hQ[t - 3]);
                }
                gP[t - 1] = from_prev(hP[t - 1]);
                gQ[t - 1] = from_prev(hQ[t - 1]);
            }

            // ---- full step (lw2) at (i, jf), jf = jj - 2 ----
            if (t >= 4) {
                const int jf = jj - 2;
                if (FAST || (jf >= lo && jf < hi)) {
                    double2 oP = z, oQ = z;
                    const bool pole = !FAST && ((jf == 0) || (jf == nth - 1));
                    if (FAST || (!pole && interior_col)) {
                        const ThetaRow& R = Rh[t - 1];
                        const Coef c = coef_at(rn, R.cos_th, R.sin2, P.kerr != 0);
                        const double2 F = SRC ? window_value(A.fn, A.org.z, A.org.w, P.win_r, P.win_t, i, jf) : z;
                        // sums/differences of the half values at i+1/2 (own) and i-1/2 (lane-1)
                        const double2 sPm = c_add(hP[t - 3], gP[t - 3]);
                        const double2 sP0 = c_add(hP[t - 2], gP[t - 2]);
                        const double2 sPp = c_add(hP[t - 1], gP[t - 1]);
                        const double2 sQ0 = c_add(hQ[t - 2], gQ[t - 2]);
                        const double2 dP0 = c_sub(hP[t - 2], gP[t - 2]);
                        const double2 dQ0 = c_sub(hQ[t - 2], gQ[t - 2]);
                        lw_point(c, R, sPm, sP0, sPp, sQ0, dP0, dQ0, F,
                                 P.dt, P.inv_hr, uP[t - 2], uQ[t - 2], oP, oQ);
                        if (P.ko_c != 0.0) {
                            const double sg = P.even ? 1.0 : -1.0;
                            // rows jf-2 .. jf+2; ghost rows -1 and nth reflect row 1 / nth-2
                            const bool lo_ghost = !FAST && jf == 1;
                            const bool hi_ghost = !FAST && jf == nth - 2;
                            const double2 pm2 = lo_ghost ? c_scale(sg, uP[t - 2]) : uP[t - 4];
                            const double2 qm2 = lo_ghost ? c_scale(sg, uQ[t - 2]) : uQ[t - 4];
                            const double2 pp2 = hi_ghost ? c_scale(sg, uP[t - 2]) : uP[t];
                            const double2 qp2 = hi_ghost ? c_scale(sg, uQ[t - 2]) : uQ[t];
                            oP = ko_apply(oP, P.ko_c, pm2, uP[t - 3], uP[t - 2], uP[t - 1], pp2);
                            oQ = ko_apply(oQ, P.ko_c, qm2, uQ[t - 3], uQ[t - 2], uQ[t - 1], qp2);
                        }
                    }
                    if (!pole) {
                        store(jf, oP, oQ);
                        if (!FAST) {
                            if (jf == 1) { oP1 = oP; oQ1 = oQ; }
                            if (jf == 2 && lo == 0) {   // pole row 0 from rows 1, 2
                                store(0, masked(interior_col, pole_value(P.even, oP1, oP)),
                                      masked(interior_col, pole_value(P.even, oQ1, oQ)));
                            }
                            if (jf == nth - 2 && hi == nth) {   // last pole row from rows nth-2, nth-3
                                store(nth - 1, masked(interior_col, pole_value(P.even, oP, oPp)),
                                      masked(interior_col, pole_value(P.even, oQ, oQp)));
                            }
                            oPp = oP;
                            oQp = oQ;
                        }
                    }
                }
            }
        }
    }
}

}  // namespace teuk
