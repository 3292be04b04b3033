// Device kernels of the engine: the single-step streaming stencil, the
// compact source pass, initial data, and small utilities.  The temporally
// blocked kernel is in block.hip, the batched one in batch_kernel.hip.
//
// Layout in HBM: Phi and Pi are two planes of double2 (complex, interleaved)
// [nth][ld], r* contiguous, ld = nr rounded up to 16 elements (256-byte rows).
// Coefficients are never stored as 2D fields: each wave keeps the radial
// records of its 64 columns in registers and forms b, w, c_t, m_r, C_0 per
// point from them and one angular record per row (see geometry.h).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include <type_traits>

#include "item_order.h"
#include "kernels.h"
#include "lw_point.h"
#include "stream_level.h"

namespace teuk {

// One Lax-Wendroff iteration.  Each wave owns a strip of 64 columns (62
// written, one halo column on each side) and a segment of theta rows, and
// streams down the rows: load row jj of u^n, form the half-step row jj-1,
// then the full-step row jj-2.  Radial neighbours come from the adjacent
// lane; the theta window lives in registers (the loop is fully unrolled).
// This is the sequence of stream_level for one level from and to the planes,
// written out in the kernel itself: the compiler schedules it about 8 %
// faster than the same code reached through the inlined template (same
// instructions on every point, so the results are bitwise identical).
// Rows a segment must keep from the poles to take the interior form:
// jlo >= kStepLoRows, jlo + SEG <= nth - kStepHiRows.
constexpr int kStepLoRows = 4, kStepHiRows = 2;

template <int SEG>
__global__ void __launch_bounds__(256) lw_step_kernel(StepParams P, const ThetaRow* __restrict__ rows) {
    const int lane = threadIdx.x & 63;
    // the wave's work item, in a scalar register: everything derived from it
    // (segment rows, row branches, angular-record addresses) is then known to
    // be wave-uniform, so the row branches are scalar and the records are
    // fetched through the scalar cache.  The frame waves (general form) are
    // dispatched first, round robin over the XCDs; the interior ones follow,
    // each XCD walking a contiguous range.
    int item;
    {
        ItemOrder o = item_order(P.nr, P.nth, P.nstrips, P.nseg, SEG, kStepLoRows, kStepHiRows);
        if (!P.frame_first) {   // plain item order, each XCD a contiguous range
            o.frame = 0;
            o.interior = P.nstrips * P.nseg;
        }
        const int fb = (o.frame + 3) / 4;
        const int blk = blockIdx.x;
        if (blk < fb) {
            const int f = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));
            if (f >= o.frame) return;
            item = frame_item(o, P.nseg, f);
        } else {
            const int wg = xcd_remap(blk - fb, gridDim.x - fb);
            const int k = __builtin_amdgcn_readfirstlane(wg * 4 + (threadIdx.x >> 6));
            if (k >= o.interior) return;
            item = P.frame_first ? interior_item(o, P.nseg, k) : k;
        }
        item = __builtin_amdgcn_readfirstlane(item);
        if (item < 0 || item >= P.nstrips * P.nseg) return;   // uniform per wave
    }
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

    // The wave's rows and columns are either all interior (every row and
    // half row in range, no pole or ghost row, every lane an interior
    // column: most items) or not, and the wave either meets a source window
    // or not (window_meets).  The body is instantiated for interior waves
    // without the source, other waves without it, and waves with it.  In the
    // interior form the range, pole and column tests are constants, so the
    // unrolled window carries no selects or copies for them; without the
    // source there are no lookups (F = 0, as a lookup outside the window
    // gives).  All run the same arithmetic on every point.
    auto body = [&](auto interior_tag, auto src_tag) {
        constexpr bool FAST = decltype(interior_tag)::value;
        constexpr bool SRC = decltype(src_tag)::value;
        // rows of u^n the segment reads: jlo-2 .. jhi+1 (t < NT)
        constexpr int NT = FAST ? SEG + 4 : SEG + 6;
        double2 uP[SEG + 6], uQ[SEG + 6];     // u^n, own column, rows jlo-2+t
        double2 sP[SEG + 6], sQ[SEG + 6], dP[SEG + 6], dQ[SEG + 6];
        double2 hP[SEG + 6], hQ[SEG + 6];     // half-step values at i+1/2, rows jlo-2+t
        double2 gP[SEG + 6], gQ[SEG + 6];     // half-step values at i-1/2 (from lane-1)
        double2 oP1 = z, oQ1 = z;             // full-step row 1 (for the pole row 0)
        double2 oPp = z, oQp = z;             // previous full-step row (for the last pole row)

        // Software prefetch: row t of u^n is fetched PF iterations before it
        // is used, at a clamped (always valid) address and unconditionally, so
        // its latency overlaps the arithmetic of the rows in between;
        // out-of-range rows and columns are masked to zero where they are used.
        constexpr int PF = kPrefetchRows;
        double2 fP[SEG + 6], fQ[SEG + 6];
        const int icl = min(max(i, 0), P.nr - 1);
        // With the source, its values for the half step of row jlo-3+t and
        // the full step of row jlo-4+t are fetched with row t, at clamped
        // window indices, and masked where used (a lookup that waits at
        // once would also wait for every load issued before it).
        double2 fFh[SEG + 6], fFn[SEG + 6];
        const int dch = i - org.x, dcn = i - org.z;
        const bool colh = static_cast<unsigned>(dch) < static_cast<unsigned>(P.win_r);
        const bool coln = static_cast<unsigned>(dcn) < static_cast<unsigned>(P.win_r);
        const int dchc = min(max(dch, 0), P.win_r - 1), dcnc = min(max(dcn, 0), P.win_r - 1);
        auto fetch = [&](int t) {
            const int jc = FAST ? jlo - 2 + t : min(max(jlo - 2 + t, 0), nth - 1);
            fP[t] = P.phi[static_cast<size_t>(jc) * ld + icl];
            fQ[t] = P.pi[static_cast<size_t>(jc) * ld + icl];
            if (SRC) {
                const int rh_ = min(max(jlo - 3 + t - org.y, 0), P.win_t - 1);
                const int rn_ = min(max(jlo - 4 + t - org.w, 0), P.win_t - 1);
                fFh[t] = P.fh[rh_ * P.win_r + dchc];
                fFn[t] = P.fn[rn_ * P.win_r + dcnc];
            }
        };
#pragma unroll
        for (int t = 0; t < PF && t < NT; ++t) fetch(t);

        // Angular records: the half step of iteration t uses row jlo-3+t, the
        // full step of iteration t the row of the half step of t-1.  Each is
        // read once, one iteration before its first use (scalar loads).
        ThetaRow Rh[SEG + 6];
        auto fetch_row = [&](int t) {
            const int jr = FAST ? jlo - 3 + t : min(max(jlo - 3 + t, 0), nth - 1);
            Rh[t] = rows[jr];
        };
        if (2 < NT) fetch_row(2);

#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t + PF < NT) fetch(t + PF);
            if (t >= 1 && t + 1 < NT) fetch_row(t + 1);
            const int jj = jlo - 2 + t;
            if (FAST || jj <= jhi + 1) {
                // ---- row jj of u^n and its column sums/differences ----
                double2 p = z, q = z;
                if (FAST || (jj >= 0 && jj < nth && in_col)) {
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
                        const double2 F =
                            SRC ? masked(colh && static_cast<unsigned>(jh - org.y) < static_cast<unsigned>(P.win_t),
                                         fFh[t])
                                : z;
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
                    if (FAST || (jf >= jlo && jf < jhi)) {
                        double2 oP = z, oQ = z;
                        const bool pole = !FAST && ((jf == 0) || (jf == nth - 1));
                        if (FAST || (!pole && interior_col)) {
                            const ThetaRow& R = Rh[t - 1];
                            const Coef c = coef_at(rn, R.cos_th, R.sin2, P.kerr != 0);
                            const double2 F =
                                SRC ? masked(coln && static_cast<unsigned>(jf - org.w) < static_cast<unsigned>(P.win_t),
                                             fFn[t])
                                    : z;
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
                            if (writer) {
                                P.phi_out[static_cast<size_t>(jf) * ld + i] = oP;
                                P.pi_out[static_cast<size_t>(jf) * ld + i] = oQ;
                                if (P.wave != nullptr && i == P.i_ext) P.wave[jf] = oP;
                            }
                            if (!FAST) {
                                if (jf == 1) { oP1 = oP; oQ1 = oQ; }
                                if (jf == 2) {   // pole row 0 from rows 1, 2
                                    const double2 p0 = masked(interior_col, pole_value(P.even, oP1, oP));
                                    const double2 q0 = masked(interior_col, pole_value(P.even, oQ1, oQ));
                                    if (writer) {
                                        P.phi_out[i] = p0;
                                        P.pi_out[i] = q0;
                                        if (P.wave != nullptr && i == P.i_ext) P.wave[0] = p0;
                                    }
                                }
                                if (jf == nth - 2) {   // last pole row from rows nth-2, nth-3
                                    const double2 pl = masked(interior_col, pole_value(P.even, oP, oPp));
                                    const double2 ql = masked(interior_col, pole_value(P.even, oQ, oQp));
                                    if (writer) {
                                        P.phi_out[static_cast<size_t>(nth - 1) * ld + i] = pl;
                                        P.pi_out[static_cast<size_t>(nth - 1) * ld + i] = ql;
                                        if (P.wave != nullptr && i == P.i_ext) P.wave[nth - 1] = pl;
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
    };

    const bool interior = strip >= 1 && strip * 62 + 64 <= P.nr && seg != P.nseg - 1 &&
                          jlo >= kStepLoRows && jlo + SEG <= nth - kStepHiRows;
    const int i0 = strip * 62 - 1;
    // (the launcher sets both window tables or neither)
    const bool src = P.fh != nullptr && P.fn != nullptr && P.win_r > 0 && P.win_t > 0 &&
                     (window_meets(org, false, P.win_r, P.win_t, i0, jlo - 1, jhi) ||
                      window_meets(org, true, P.win_r, P.win_t, i0, jlo, jhi - 1));
    if (src)   // uniform per wave
        body(std::false_type{}, std::true_type{});
    else if (interior)
        body(std::true_type{}, std::false_type{});
    else
        body(std::false_type{}, std::false_type{});
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

// Clears n16 16-byte words and then tail 4-byte words after them (a kernel,
// not hipMemsetAsync, so that the clear is an ordinary kernel node when a
// caller captures the stream).
__global__ void zero_kernel(uint4* p, size_t n16, unsigned int* tail, int ntail) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t k = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < n16; k += stride)
        p[k] = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0 && static_cast<int>(threadIdx.x) < ntail) tail[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------

hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 4 != 0 || reinterpret_cast<uintptr_t>(p) % 16 != 0) return hipErrorInvalidValue;
    const size_t n16 = bytes / 16;
    const int ntail = static_cast<int>((bytes - 16 * n16) / 4);
    const size_t blocks = std::min<size_t>((n16 + 255) / 256 + 1, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       static_cast<uint4*>(p), n16, reinterpret_cast<unsigned int*>(static_cast<char*>(p) + 16 * n16),
                       ntail);
    return hipGetLastError();
}

bool valid_segment_rows(int seg) {
    for (int v : kSegVariants)
        if (v == seg) return true;
    return false;
}

// P.nseg must have been computed for this segment length: (nth - 3) / seg + 1.
// With events, the launch itself records them at the kernel's start and end.
hipError_t launch_step(const StepParams& P, int seg, hipStream_t stream, hipEvent_t ev_start,
                       hipEvent_t ev_stop) {
    const dim3 grid(P.frame_first ? ordered_blocks(item_order(P.nr, P.nth, P.nstrips, P.nseg, seg, kStepLoRows,
                                                              kStepHiRows))
                                  : (P.nstrips * P.nseg + 3) / 4),
        block(256);
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
