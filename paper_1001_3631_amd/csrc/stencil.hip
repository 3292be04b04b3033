// Device kernels of the engine: the single-step streaming stencil, the
// compact source pass, initial data, and small utilities.
//
// Layout in HBM: Phi and Pi are two planes of double2 (complex, interleaved)
// [nth][ld], r* contiguous, ld = nr rounded up to 16 elements (256-byte rows).
// Coefficients are never stored as 2D fields: each wave keeps the radial
// records of its 64 columns in registers and forms b, w, c_t, m_r, C_0 per
// point from them and one angular record per row (see geometry.h).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "lw_point.h"

namespace teuk {

// Rows of u^n the single-step kernel fetches ahead of their use.
#ifndef TEUK_PREFETCH_ROWS
#define TEUK_PREFETCH_ROWS 2
#endif
constexpr int kPrefetchRows = TEUK_PREFETCH_ROWS;
// The batched kernel holds more state per wave (instance fields); with the
// prefetch its register count would leave one wave per SIMD.
#ifndef TEUK_BATCH_PREFETCH_ROWS
#define TEUK_BATCH_PREFETCH_ROWS 0
#endif
constexpr int kBatchPrefetchRows = TEUK_BATCH_PREFETCH_ROWS;

namespace {

// Cross-lane moves with DPP wave shifts (no LDS traffic): from_next gives lane
// l the value of lane l+1 (lane 63 keeps its own), from_prev the value of lane
// l-1 (lane 0 keeps its own).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double2 from_next(double2 v) {
    return make_double2(dpp_move<0x130>(v.x), dpp_move<0x130>(v.y));   // wave_shl:1
}
__device__ __forceinline__ double2 from_prev(double2 v) {
    return make_double2(dpp_move<0x138>(v.x), dpp_move<0x138>(v.y));   // wave_shr:1
}



__device__ __forceinline__ double2 src_lookup(const double2* __restrict__ tab, int c0, int r0,
                                              int win_r, int win_t, int col, int row) {
    if (tab == nullptr) return make_double2(0.0, 0.0);
    const unsigned dc = static_cast<unsigned>(col - c0);
    const unsigned dr = static_cast<unsigned>(row - r0);
    if (dc < static_cast<unsigned>(win_r) && dr < static_cast<unsigned>(win_t))
        return tab[dr * win_r + dc];
    return make_double2(0.0, 0.0);
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
template <int NROW, bool IN_LDS, bool OUT_LDS, int PREFETCH = kPrefetchRows>
__device__ __forceinline__ void stream_level(const StepParams P, const LevelArgs A, const RCol rn,
                                             const RCol rh, const ThetaRow* __restrict__ rows) {
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
        const int jc = min(max(lo - 2 + t, 0), nth - 1);
        fP[t] = P.phi[static_cast<size_t>(jc) * ld + icl];
        fQ[t] = P.pi[static_cast<size_t>(jc) * ld + icl];
    };
#pragma unroll
    for (int t = 0; t < PF && t < NROW + 4; ++t) fetch(t);

#pragma unroll
    for (int t = 0; t < NROW + 4; ++t) {
        if (!IN_LDS && t + PF < NROW + 4) fetch(t + PF);
        const int jj = lo - 2 + t;
        if (jj <= hi + 1) {
            // ---- row jj of the input level and its column sums/differences ----
            double2 p = z, q = z;
            if (IN_LDS) {
                if (jj >= 0 && jj < nth) {
                    p = A.lp[(jj - A.lbase) * 64 + lane];
                    q = A.lq[(jj - A.lbase) * 64 + lane];
                }
            } else if (jj >= 0 && jj < nth && in_col) {
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
                if (jh >= 1 && jh <= nth - 2) {
                    const ThetaRow R = rows[jh];
                    const Coef c = coef_at(rh, R.cos_th, R.sin2, P.kerr != 0);
                    const double2 F = src_lookup(A.fh, A.org.x, A.org.y, P.win_r, P.win_t, i, jh);
                    lw_point(c, R, sP[t - 2], sP[t - 1], sP[t], sQ[t - 1],
                             dP[t - 1], dQ[t - 1], F, 0.5 * P.dt, P.inv_hr, c_scale(0.5, sP[t - 1]),
                             c_scale(0.5, sQ[t - 1]), hP[t - 1], hQ[t - 1]);
                } else if (jh == nth - 1 && t >= 4) {
                    hP[t - 1] = pole_value(P.even, hP[t - 2], hP[t - 3]);
                    hQ[t - 1] = pole_value(P.even, hQ[t - 2], hQ[t - 3]);
                }
                if (jh == 2 && t >= 5) {   // pole row 0 of the half step, now that rows 1, 2 exist
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
                if (jf >= lo && jf < hi) {
                    double2 oP = z, oQ = z;
                    const bool pole = (jf == 0) || (jf == nth - 1);
                    if (!pole && interior_col) {
                        const ThetaRow R = rows[jf];
                        const Coef c = coef_at(rn, R.cos_th, R.sin2, P.kerr != 0);
                        const double2 F = src_lookup(A.fn, A.org.z, A.org.w, P.win_r, P.win_t, i, jf);
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
                            const double2 pm2 = (jf == 1) ? c_scale(sg, uP[t - 2]) : uP[t - 4];
                            const double2 qm2 = (jf == 1) ? c_scale(sg, uQ[t - 2]) : uQ[t - 4];
                            const double2 pp2 = (jf == nth - 2) ? c_scale(sg, uP[t - 2]) : uP[t];
                            const double2 qp2 = (jf == nth - 2) ? c_scale(sg, uQ[t - 2]) : uQ[t];
                            oP = ko_apply(oP, P.ko_c, pm2, uP[t - 3], uP[t - 2], uP[t - 1], pp2);
                            oQ = ko_apply(oQ, P.ko_c, qm2, uQ[t - 3], uQ[t - 2], uQ[t - 1], qp2);
                        }
                    }
                    if (!pole) {
                        store(jf, oP, oQ);
                        if (jf == 1) { oP1 = oP; oQ1 = oQ; }
                        if (jf == 2 && lo == 0) {   // pole row 0 from rows 1, 2
                            const double2 p0 = pole_value(P.even, oP1, oP);
                            const double2 q0 = pole_value(P.even, oQ1, oQ);
                            store(0, interior_col ? p0 : z, interior_col ? q0 : z);
                        }
                        if (jf == nth - 2 && hi == nth) {   // last pole row from rows nth-2, nth-3
                            const double2 pl = pole_value(P.even, oP, oPp);
                            const double2 ql = pole_value(P.even, oQ, oQp);
                            store(nth - 1, interior_col ? pl : z, interior_col ? ql : z);
                        }
                        oPp = oP;
                        oQp = oQ;
                    }
                }
            }
        }
    }
}

// One Lax-Wendroff iteration.  Each wave owns a strip of 64 columns (62
// written, one halo column on each side) and a segment of theta rows, and
// streams down the rows: load row jj of u^n, form the half-step row jj-1,
// then the full-step row jj-2.  Radial neighbours come from the adjacent
// lane; the theta window lives in registers (the loop is fully unrolled).
// This is the sequence of stream_level for one level from and to the planes,
// written out in the kernel itself: the compiler schedules it about 8 %
// faster than the same code reached through the inlined template (same
// instructions on every point, so the results are bitwise identical).
template <int SEG>
__global__ void __launch_bounds__(256) lw_step_kernel(StepParams P, const ThetaRow* __restrict__ rows) {
    const int lane = threadIdx.x & 63;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    // the wave's work item, in a scalar register: everything derived from it
    // (segment rows, row branches, angular-record addresses) is then known to
    // be wave-uniform, so the row branches are scalar and the records are
    // fetched through the scalar cache
    const int item = __builtin_amdgcn_readfirstlane(wg * 4 + (threadIdx.x >> 6));
    if (item >= P.nstrips * P.nseg) return;   // uniform per wave
    const int strip = item / P.nseg;
    const int seg = item - strip * P.nseg;
    const int i = strip * 62 - 1 + lane;
    const bool in_col = (i >= 0) && (i < P.nr);
    const bool writer = in_col && lane >= 1 && lane <= 62;
    const bool interior_col = (i >= 1) && (i <= P.nr - 2);
    const int jlo = seg * SEG;
    const int jhi = (seg == P.nseg - 1) ? P.nth : jlo + SEG;
    const int nth = P.nth;
    const int ld = P.ld;

    int4 org = make_int4(0, 0, 0, 0);
    if (P.org != nullptr) org = *P.org;
    const int ic = min(max(i, 0), P.nr - 1);
    const int ih = min(max(i, 0), P.nr - 2);
    const RCol rn = load_rcol(P.rnode, P.rpitch, ic);
    const RCol rh = load_rcol(P.rhalf, P.rpitch, ih);

    const double2 z = make_double2(0.0, 0.0);
    double2 uP[SEG + 6], uQ[SEG + 6];     // u^n, own column, rows jlo-2+t
    double2 sP[SEG + 6], sQ[SEG + 6], dP[SEG + 6], dQ[SEG + 6];
    double2 hP[SEG + 6], hQ[SEG + 6];     // half-step values at i+1/2, rows jlo-2+t
    double2 gP[SEG + 6], gQ[SEG + 6];     // half-step values at i-1/2 (from lane-1)
    double2 oP1 = z, oQ1 = z;             // full-step row 1 (for the pole row 0)
    double2 oPp = z, oQp = z;             // previous full-step row (for the last pole row)

    // Software prefetch: row t of u^n is fetched PF iterations before it is
    // used, at a clamped (always valid) address and unconditionally, so its
    // latency overlaps the arithmetic of the rows in between; out-of-range
    // rows and columns are masked to zero where they are used.
    constexpr int PF = kPrefetchRows;
    double2 fP[SEG + 6], fQ[SEG + 6];
    const int icl = min(max(i, 0), P.nr - 1);
    auto fetch = [&](int t) {
        const int jc = min(max(jlo - 2 + t, 0), nth - 1);
        fP[t] = P.phi[static_cast<size_t>(jc) * ld + icl];
        fQ[t] = P.pi[static_cast<size_t>(jc) * ld + icl];
    };
#pragma unroll
    for (int t = 0; t < PF && t < SEG + 6; ++t) fetch(t);

#pragma unroll
    for (int t = 0; t < SEG + 6; ++t) {
        if (t + PF < SEG + 6) fetch(t + PF);
        const int jj = jlo - 2 + t;
        if (jj <= jhi + 1) {
            // ---- row jj of u^n and its column sums/differences ----
            double2 p = z, q = z;
            if (jj >= 0 && jj < nth && in_col) {
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
                if (jh >= 1 && jh <= nth - 2) {
                    const ThetaRow R = rows[jh];
                    const Coef c = coef_at(rh, R.cos_th, R.sin2, P.kerr != 0);
                    const double2 F = src_lookup(P.fh, org.x, org.y, P.win_r, P.win_t, i, jh);
                    lw_point(c, R, sP[t - 2], sP[t - 1], sP[t], sQ[t - 1],
                             dP[t - 1], dQ[t - 1], F, 0.5 * P.dt, P.inv_hr, c_scale(0.5, sP[t - 1]),
                             c_scale(0.5, sQ[t - 1]), hP[t - 1], hQ[t - 1]);
                } else if (jh == nth - 1 && t >= 4) {
                    hP[t - 1] = pole_value(P.even, hP[t - 2], hP[t - 3]);
                    hQ[t - 1] = pole_value(P.even, hQ[t - 2], hQ[t - 3]);
                }
                if (jh == 2 && t >= 5) {   // pole row 0 of the half step, now that rows 1, 2 exist
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
                if (jf >= jlo && jf < jhi) {
                    double2 oP = z, oQ = z;
                    const bool pole = (jf == 0) || (jf == nth - 1);
                    if (!pole && interior_col) {
                        const ThetaRow R = rows[jf];
                        const Coef c = coef_at(rn, R.cos_th, R.sin2, P.kerr != 0);
                        const double2 F = src_lookup(P.fn, org.z, org.w, P.win_r, P.win_t, i, jf);
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
                            const double2 pm2 = (jf == 1) ? c_scale(sg, uP[t - 2]) : uP[t - 4];
                            const double2 qm2 = (jf == 1) ? c_scale(sg, uQ[t - 2]) : uQ[t - 4];
                            const double2 pp2 = (jf == nth - 2) ? c_scale(sg, uP[t - 2]) : uP[t];
                            const double2 qp2 = (jf == nth - 2) ? c_scale(sg, uQ[t - 2]) : uQ[t];
                            oP = ko_apply(oP, P.ko_c, pm2, uP[t - 3], uP[t - 2], uP[t - 1], pp2);
                            oQ = ko_apply(oQ, P.ko_c, qm2, uQ[t - 3], uQ[t - 2], uQ[t - 1], qp2);
                        }
                    }
                    if (!pole) {
                        if (writer) {
                            P.phi_out[static_cast<size_t>(jf) * ld + i] = oP;
                            P.pi_out[static_cast<size_t>(jf) * ld + i] = oQ;
                            if (P.wave != nullptr && i == P.i_ext) P.wave[jf] = oP;
                        }
                        if (jf == 1) { oP1 = oP; oQ1 = oQ; }
                        if (jf == 2) {   // pole row 0 from rows 1, 2
                            const double2 p0 = pole_value(P.even, oP1, oP);
                            const double2 q0 = pole_value(P.even, oQ1, oQ);
                            if (writer) {
                                P.phi_out[i] = interior_col ? p0 : z;
                                P.pi_out[i] = interior_col ? q0 : z;
                                if (P.wave != nullptr && i == P.i_ext) P.wave[0] = interior_col ? p0 : z;
                            }
                        }
                        if (jf == nth - 2) {   // last pole row from rows nth-2, nth-3
                            const double2 pl = pole_value(P.even, oP, oPp);
                            const double2 ql = pole_value(P.even, oQ, oQp);
                            if (writer) {
                                P.phi_out[static_cast<size_t>(nth - 1) * ld + i] = interior_col ? pl : z;
                                P.pi_out[static_cast<size_t>(nth - 1) * ld + i] = interior_col ? ql : z;
                                if (P.wave != nullptr && i == P.i_ext) P.wave[nth - 1] = interior_col ? pl : z;
                            }
                        }
                        oPp = oP;
                        oQp = oQ;
                    }
                }
            }
        }
    }
}

// Temporal blocking: K consecutive iterations in one launch.  A work item is
// one wave (a workgroup of 64 threads) on 64 columns and a theta segment.
// Level l (1..K) produces rows [jlo - 2(K-l), jhi + 2(K-l)) clipped to the
// grid: each iteration widens the dependence by 2 rows (the full step reads
// u^n at j-2..j+2) and one column on each side, so the 64 lanes end with
// 64 - 2K owner columns.  Levels 1..K-1 stay in this wave's LDS buffer; only
// level K is written to HBM.  Every point goes through stream_level, so a
// block is bitwise identical to K single iterations.
template <int SEG, int K, int L>
__device__ __forceinline__ void block_levels(const StepParams& P, LevelArgs& A, int jlo, int jhi,
                                             const RCol& rn, const RCol& rh,
                                             const ThetaRow* __restrict__ rows) {
    constexpr int NROW = SEG + 2 + 4 * (K - L);
    A.lo = max(0, jlo - 2 * (K - L));
    A.hi = min(P.nth, jhi + 2 * (K - L));
    const size_t wsz = static_cast<size_t>(P.win_r) * P.win_t;
    A.fh = P.fh ? P.fh + (L - 1) * wsz : nullptr;
    A.fn = P.fn ? P.fn + (L - 1) * wsz : nullptr;
    A.org = make_int4(0, 0, 0, 0);
    if (P.org != nullptr) A.org = P.org[L - 1];
    A.wave = P.wave ? P.wave + static_cast<size_t>(L - 1) * P.nth : nullptr;
    stream_level<NROW, (L > 1), (L < K)>(P, A, rn, rh, rows);
    if constexpr (L < K) block_levels<SEG, K, L + 1>(P, A, jlo, jhi, rn, rh, rows);
}

template <int SEG, int K>
__global__ void __launch_bounds__(64) lw_block_kernel(StepParams P, const ThetaRow* __restrict__ rows) {
    constexpr int ROWS = SEG + 2 + 4 * (K - 1);
    __shared__ double2 bufP[ROWS * 64];
    __shared__ double2 bufQ[ROWS * 64];
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    if (item >= P.nstrips * P.nseg) return;
    const int strip = item / P.nseg;
    const int seg = item - strip * P.nseg;
    const int jlo = seg * SEG;
    const int jhi = (seg == P.nseg - 1) ? P.nth : jlo + SEG;
    LevelArgs A;
    A.lane = threadIdx.x;
    A.i = strip * (64 - 2 * K) - K + A.lane;
    A.halo = K;
    A.lp = bufP;
    A.lq = bufQ;
    A.lbase = max(0, jlo - 2 * (K - 1));
    const int ic = min(max(A.i, 0), P.nr - 1);
    const int ih = min(max(A.i, 0), P.nr - 2);
    const RCol rn = load_rcol(P.rnode, P.rpitch, ic);
    const RCol rh = load_rcol(P.rhalf, P.rpitch, ih);
    block_levels<SEG, K, 1>(P, A, jlo, jhi, rn, rh, rows);
}

// Batched persistent stepping: many independent instances (each its own
// grid, coefficients and planes) advance `rounds` iterations in one launch.
// Work item = one tile of one iteration, a tile being a strip of 62 columns
// of one instance over all its theta rows (the wave streams the segments of
// SEG rows one after another, reusing its radial records).  Each workgroup
// is one wave; each pass of its loop takes the next item from a global
// counter, in iteration-major order: every tile of iteration n before any
// tile of n + 1.  The counter value and the abort flag reach all lanes
// through LDS between two barriers, so every lane holds the same item without
// relying on lanes reconverging on their own.
//
// Dependencies: the item (tile, n) reads u^n on its strip plus one column on
// each side, inside the strips s - 1, s, s + 1, and writes the level that
// those strips read at iteration n - 1.  It therefore waits until each of
// them has completed n iterations (done >= n), then publishes done = n + 1.
// Every wait is on an item with a smaller ticket; a ticket is only handed
// out at the top of a pass and is processed right away, so its holder is
// running and the smallest unfinished ticket never waits: every wait ends.
// A wait longer than wait_limit (a broken invariant) sets *abort, and every
// wave leaves at the top of its next pass.  Tile data is made visible across
// the XCDs' L2 caches by an agent-scope release after the tile's stores and
// an agent-scope acquire after the wait.
template <int SEG>
__global__ void __launch_bounds__(64) lw_batch_kernel(BatchParams B) {
    __shared__ unsigned long long s_t;
    __shared__ int s_stop;
    const int lane = threadIdx.x;
    const unsigned long long total = static_cast<unsigned long long>(B.rounds) * B.ntiles;
    while (true) {
        __syncthreads();                     // the previous pass has read s_t / s_stop
        if (lane == 0) {
            s_t = __hip_atomic_fetch_add(B.ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_stop = __hip_atomic_load(B.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const unsigned long long tv = s_t;
        if (s_stop != 0 || tv >= total) break;            // the same decision in every lane
        // equal in every lane: move it to scalar registers
        const unsigned long long t =
            (static_cast<unsigned long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(tv >> 32))) << 32) |
            static_cast<unsigned int>(__builtin_amdgcn_readfirstlane(static_cast<int>(tv & 0xffffffffu)));

        const int n = static_cast<int>(t / static_cast<unsigned long long>(B.ntiles));
        const int k = static_cast<int>(t - static_cast<unsigned long long>(n) * B.ntiles);
        const int4 tile = B.tiles[k];
        const BatchInstance& I = B.inst[tile.x];
        const int strip = tile.y;

        if (n > 0 && lane < 3) {
            const int s2 = strip + lane - 1;
            if (s2 >= 0 && s2 < I.nstrips) {
                const int* f = B.done + I.tile0 + s2;
                const long long t0 = wall_clock64();
                while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < n) {
                    if (__hip_atomic_load(B.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
                    if (wall_clock64() - t0 > B.wait_limit) {
                        __hip_atomic_store(B.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
        }
        // after an abort the item is still computed (on whatever data is
        // there); the host reports the abort and the states are invalid
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

        StepParams P;
        const int lv = (I.cur + n) & 1;
        P.phi = I.plane[lv][0];
        P.pi = I.plane[lv][1];
        P.phi_out = I.plane[lv ^ 1][0];
        P.pi_out = I.plane[lv ^ 1][1];
        P.rnode = I.rnode;
        P.rhalf = I.rhalf;
        P.rows = I.rows;
        P.nr = I.nr;
        P.nth = I.nth;
        P.ld = I.ld;
        P.rpitch = I.rpitch;
        P.nstrips = I.nstrips;
        P.nseg = I.nseg;
        P.dt = I.dt;
        P.inv_hr = I.inv_hr;
        P.ko_c = I.ko_c;
        P.even = I.even;
        P.kerr = I.kerr;
        P.i_ext = I.i_ext;
        P.wave = nullptr;
        P.fh = P.fn = nullptr;
        P.org = nullptr;
        P.win_r = P.win_t = 0;
        LevelArgs A;
        A.lane = lane;
        A.i = strip * 62 - 1 + lane;
        A.halo = 1;
        A.fh = A.fn = nullptr;
        A.org = make_int4(0, 0, 0, 0);
        A.wave = I.wave ? I.wave + static_cast<size_t>(n) * P.nth : nullptr;
        A.lp = A.lq = nullptr;
        A.lbase = 0;
        const int ic = min(max(A.i, 0), P.nr - 1);
        const int ih = min(max(A.i, 0), P.nr - 2);
        const RCol rn = load_rcol(P.rnode, P.rpitch, ic);
        const RCol rh = load_rcol(P.rhalf, P.rpitch, ih);
        for (int q = 0; q < P.nseg; ++q) {
            A.lo = q * SEG;
            A.hi = (q == P.nseg - 1) ? P.nth : A.lo + SEG;
            stream_level<SEG + 2, false, false, kBatchPrefetchRows>(P, A, rn, rh, P.rows);
        }

        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0) __hip_atomic_store(B.done + tile.w, n + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Zero the work counter and the per-tile counters (a kernel, so that it can
// be a node of a captured graph).  The abort flag is left alone: once set, it
// stays set (and later launches exit at once) until the host has read it.
__global__ void __launch_bounds__(256) batch_reset_kernel(BatchParams B) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) *B.ticket = 0ull;
    if (e < B.ntiles) B.done[e] = 0;
}

// Compact source pass: F on the windows near the particle for a batch of
// iterations.  Block y = iteration in the batch; threads cover the window.
// Half-point window (time t_n, sample 2n) and node window (t_n + dt/2,
// sample 2n+1).
__global__ void __launch_bounds__(256) source_pass_kernel(SourceParams S) {
    const int b = blockIdx.y;
    const int n = S.n0 + b;
    // window origins: first index whose coordinate can lie within cut*sigma
    const double* sh = S.orbit + 3 * static_cast<size_t>(2 * n);
    const double* sn_ = S.orbit + 3 * static_cast<size_t>(2 * n + 1);
    const double Rr = S.cut * S.sig_r, Rt = S.cut * S.sig_th;
    int4 org;
    org.x = static_cast<int>(floor((sh[0] - Rr - (S.rs_min + 0.5 * S.h_r)) / S.h_r));
    org.y = static_cast<int>(floor((sh[1] - Rt) / S.h_th));
    org.z = static_cast<int>(floor((sn_[0] - Rr - S.rs_min) / S.h_r));
    org.w = static_cast<int>(floor((sn_[1] - Rt) / S.h_th));
    if (threadIdx.x == 0 && blockIdx.x == 0) S.org[b] = org;
    const int npts = S.win_r * S.win_t;
    for (int e = threadIdx.x + blockIdx.x * blockDim.x; e < 2 * npts; e += blockDim.x * gridDim.x) {
        const bool node = e >= npts;
        const int k = node ? e - npts : e;
        const int dr = k / S.win_r;
        const int dc = k - dr * S.win_r;
        const int col = (node ? org.z : org.x) + dc;
        const int row = (node ? org.w : org.y) + dr;
        const double* smp = S.orbit + 3 * static_cast<size_t>(2 * n + (node ? 1 : 0));
        double2 F = make_double2(0.0, 0.0);
        const int ncol = node ? S.nr : S.nr - 1;
        if (col >= 0 && col < ncol && row >= 0 && row < S.nth) {
            const double rs = (node ? S.rnode_rs : S.rhalf_rs)[col];
            const double th = S.rows[row].theta;
            const double gr = gauss_cut(rs - smp[0], S.sig_r, S.cut);
            const double gt = gauss_cut(th - smp[1], S.sig_th, S.cut);
            const double amp = S.amplitude * gr * gt;
            double sn, cs;
            sincos(S.m * smp[2], &sn, &cs);
            F = make_double2(amp * cs, -amp * sn);
        }
        double2* out = (node ? S.fn : S.fh) + static_cast<size_t>(b) * npts;
        out[k] = F;
    }
}

// Initial data: Gaussian in r* times the angular profile, Pi = b d_r* Phi,
// then the boundary conditions (pole rows recomputed from rows 1, 2).
__global__ void __launch_bounds__(256) init_pulse_kernel(PulseParams Q) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= Q.nr) return;
    const RCol rn = load_rcol(Q.rnode, Q.rpitch, i);
    const double rs = Q.rnode_rs[i];
    const double x = rs - Q.center;
    const double rad = Q.amplitude * exp(-x * x / (2.0 * Q.width * Q.width));
    auto value = [&](int jr, double2& p, double2& q) {
        const ThetaRow R = Q.rows[jr];
        const Coef c = coef_at(rn, R.cos_th, R.sin2, Q.kerr != 0);
        const double phi = rad * R.prof;
        p = make_double2(phi, 0.0);
        q = make_double2(-c.b * x / (Q.width * Q.width) * phi, 0.0);
    };
    double2 p = make_double2(0.0, 0.0), q = p;
    if (i > 0 && i < Q.nr - 1) {
        if (j == 0 || j == Q.nth - 1) {
            if (Q.even) {
                double2 p1, q1, p2, q2;
                const int j1 = (j == 0) ? 1 : Q.nth - 2;
                const int j2 = (j == 0) ? 2 : Q.nth - 3;
                value(j1, p1, q1);
                value(j2, p2, q2);
                p = pole_value(true, p1, p2);
                q = pole_value(true, q1, q2);
            }
        } else {
            value(j, p, q);
        }
    }
    Q.phi[static_cast<size_t>(j) * Q.ld + i] = p;
    Q.pi[static_cast<size_t>(j) * Q.ld + i] = q;
}

// Finiteness check of a plane pair; sets *flag to 1 on any NaN/Inf.
__global__ void __launch_bounds__(256) finite_kernel(const double2* __restrict__ a,
                                                     const double2* __restrict__ b, int nr, int nth,
                                                     int ld, int* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= nr) return;
    const double2 u = a[static_cast<size_t>(j) * ld + i];
    const double2 v = b[static_cast<size_t>(j) * ld + i];
    if (!isfinite(u.x) || !isfinite(u.y) || !isfinite(v.x) || !isfinite(v.y)) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------

bool valid_segment_rows(int seg) {
    for (int v : kSegVariants)
        if (v == seg) return true;
    return false;
}

// P.nseg must have been computed for this segment length: (nth - 3) / seg + 1.
// With events, the launch itself records them at the kernel's start and end.
hipError_t launch_step(const StepParams& P, int seg, hipStream_t stream, hipEvent_t ev_start,
                       hipEvent_t ev_stop) {
    const int items = P.nstrips * P.nseg;
    const dim3 grid((items + 3) / 4), block(256);
    switch (seg) {
        // the angular records are a separate __restrict__ argument: read-only,
        // never aliasing the planes, so their wave-uniform loads are scalar
        case 4: hipExtLaunchKernelGGL(lw_step_kernel<4>, grid, block, 0, stream, ev_start, ev_stop, 0, P, P.rows); break;
        case 8: hipExtLaunchKernelGGL(lw_step_kernel<8>, grid, block, 0, stream, ev_start, ev_stop, 0, P, P.rows); break;
        case 16: hipExtLaunchKernelGGL(lw_step_kernel<16>, grid, block, 0, stream, ev_start, ev_stop, 0, P, P.rows); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool valid_block(int seg, int k) {
    for (const auto& v : kBlockVariants)
        if (v.seg == seg && v.k == k) return true;
    return false;
}

int block_strip_width(int k) { return 64 - 2 * k; }

// P.nstrips = ceil(nr / (64 - 2k)), P.nseg as for launch_step; P.fh, P.fn,
// P.org point at the windows of the block's first iteration (the next k - 1
// follow at strides win_r * win_t and 1), P.wave at k rows of nth.
hipError_t launch_block(const StepParams& P, int seg, int k, hipStream_t stream, hipEvent_t ev_start,
                        hipEvent_t ev_stop) {
    const dim3 grid(P.nstrips * P.nseg), block(64);
    if (seg == 4 && k == 2)
        hipExtLaunchKernelGGL((lw_block_kernel<4, 2>), grid, block, 0, stream, ev_start, ev_stop, 0, P, P.rows);
    else if (seg == 8 && k == 2)
        hipExtLaunchKernelGGL((lw_block_kernel<8, 2>), grid, block, 0, stream, ev_start, ev_stop, 0, P, P.rows);
    else if (seg == 4 && k == 4)
        hipExtLaunchKernelGGL((lw_block_kernel<4, 4>), grid, block, 0, stream, ev_start, ev_stop, 0, P, P.rows);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_batch_reset(const BatchParams& B, hipStream_t stream) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3((B.ntiles + 255) / 256), dim3(256), 0, stream, B);
    return hipGetLastError();
}

// waves = persistent waves to start (one per workgroup); every wave loops
// over the work counter, so any positive number is correct.
hipError_t launch_batch(const BatchParams& B, int seg, int waves, hipStream_t stream) {
    const dim3 grid(waves), block(64);
    switch (seg) {
        case 4: hipLaunchKernelGGL(lw_batch_kernel<4>, grid, block, 0, stream, B); break;
        case 8: hipLaunchKernelGGL(lw_batch_kernel<8>, grid, block, 0, stream, B); break;
        case 16: hipLaunchKernelGGL(lw_batch_kernel<16>, grid, block, 0, stream, B); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_source_pass(const SourceParams& S, int nbatch, hipStream_t stream) {
    const int npts = 2 * S.win_r * S.win_t;
    const int bx = (npts + 255) / 256;
    hipLaunchKernelGGL(source_pass_kernel, dim3(bx, nbatch), dim3(256), 0, stream, S);
    return hipGetLastError();
}

hipError_t launch_init_pulse(const PulseParams& Q, hipStream_t stream) {
    hipLaunchKernelGGL(init_pulse_kernel, dim3((Q.nr + 255) / 256, Q.nth), dim3(256), 0, stream, Q);
    return hipGetLastError();
}

hipError_t launch_finite(const double2* a, const double2* b, int nr, int nth, int ld, int* flag,
                         hipStream_t stream) {
    hipLaunchKernelGGL(finite_kernel, dim3((nr + 255) / 256, nth), dim3(256), 0, stream, a, b, nr, nth,
                       ld, flag);
    return hipGetLastError();
}

}  // namespace teuk
