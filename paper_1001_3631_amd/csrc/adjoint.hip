// Adjoint of one Lax-Wendroff iteration: lambda^n = G^H lambda^{n+1}.
//
// The iteration (Sec. 3.2, Eqs. (lw1)-(lw2) with its boundary conditions) is
// C-linear, so its transpose in the real inner product is the conjugate
// transpose.  Taking its sub-steps in reverse order:
//   1. boundary conditions on u^{n+1}: pole rows of lambda fold into rows
//      1, 2 (and nth-2, nth-3) with weights 4/3, -1/3 (even |m|); radial
//      boundary nodes drop out.  Result mu on interior nodes.
//   2. full step: identity part (mu), dissipation transpose, and node-level
//      sources that the full step's averages and differences carry back to
//      the half points i-1/2, i+1/2 (conjugated node coefficients; the
//      angular operator enters through its transpose).
//   3. pole rows of the half-step values fold into rows 1, 2 / nth-2, nth-3.
//   4. half step: half-level sources carried back to nodes i, i+1.
// Every sum is a gather, so a lane owns node i and half point i+1/2 exactly as
// in the forward stencil: half values gather from lane+1, node values from
// lane-1.  Stages run at fixed row lags behind the row being loaded, so the
// fully unrolled loop indexes its register arrays with compile-time offsets.
//
// Source sensitivity: dL/dA = sum Re<lambda-part, dt-weighted unit source>
// over the half points (lw1, time t_n) and the interior nodes (lw2, time
// t_n + dt/2); each wave writes its partial sum, reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "item_order.h"
#include "kernels.h"
#include "lw_point.h"
#include "stream_level.h"   // wave shifts (from_next, from_prev)

namespace teuk {

namespace {

__device__ __forceinline__ double2 cz() { return make_double2(0.0, 0.0); }
// conj(c) * z
__device__ __forceinline__ double2 cmul_conj(double2 c, double2 z) {
    return make_double2(fma(c.x, z.x, c.y * z.y), fma(c.x, z.y, -(c.y * z.x)));
}
__device__ __forceinline__ double2 axpy(double a, double2 x, double2 y) {
    return make_double2(fma(a, x.x, y.x), fma(a, x.y, y.y));
}
__device__ __forceinline__ double re_dot_conj(double2 a, double2 b) {   // Re(conj(a) b)
    return fma(a.x, b.x, a.y * b.y);
}
__device__ __forceinline__ double2 src_at(const double2* __restrict__ tab, int c0, int r0, int win_r,
                                          int win_t, int col, int row) {
    if (tab == nullptr) return cz();
    const unsigned dc = static_cast<unsigned>(col - c0);
    const unsigned dr = static_cast<unsigned>(row - r0);
    if (dc < static_cast<unsigned>(win_r) && dr < static_cast<unsigned>(win_t)) return tab[dr * win_r + dc];
    return cz();
}
__device__ __forceinline__ int a_xcd_remap(int b, int nwg) {
    const int per = nwg / 8;
    const int full = per * 8;
    if (b >= full) return b;
    return (b % 8) * per + (b / 8);
}

// weights of the angular operator at an interior row: Ang[f]_j =
// alpha_j f_{j+1} + beta_j f_j + gamma_j f_{j-1} (the record holds the
// weights halved; doubling is exact)
struct AngW {
    double alpha, beta, gamma;
};
__device__ __forceinline__ AngW ang_weights(const ThetaRow& R) {
    AngW w;
    w.alpha = 2.0 * (R.inv_2h2 + R.cot4h);
    w.beta = 2.0 * fma(-2.0, R.inv_2h2, -R.V2);
    w.gamma = 2.0 * (R.inv_2h2 - R.cot4h);
    return w;
}

}  // namespace

// dL/dA of one reverse iteration from the source windows alone, for the
// launches whose waves skip their source terms (part 3): the node part
// sum_window dt Re(conj(mu_Pi) F_n) over the full step's window and the half
// part sum_window (dt/2) Re(conj(lambda^h_Pi) F_h) over the half step's,
// with mu and the half-level lambda formed by the same expressions as the
// stencil's stages 2-4 (the host uses this only for windows whose rows stay
// in [3, nth - 4], where no pole row folds into them).  Wave b < win_t sums
// node-window row b, wave win_t + b half-window row b, one lane per column,
// in a fixed tree, into partial b of the iteration (part 3's other waves
// write zeros into their partials, and the partials are summed in a fixed
// order).
__device__ __forceinline__ void source_dA_row(const AdjointParams& P, int b, int lane) {
    const int4 org = *P.org;
    const bool half = b >= P.win_t;
    const int dr = half ? b - P.win_t : b;
    const int dc = lane;
    const double dt = P.dt, hdt = 0.5 * P.dt, inv_hr = P.inv_hr;
    double v = 0.0;
    if (dc < P.win_r) {
        const int c = dr * P.win_r + dc;
        if (!half) {
            const int r = org.w + dr, i = org.z + dc;
            if (r >= 1 && r <= P.nth - 2 && i >= 1 && i <= P.nr - 2)
                v = dt * re_dot_conj(P.lam_pi[static_cast<size_t>(r) * P.ld + i], P.fn[c]);
        } else {
            const int r = org.y + dr, i = org.x + dc;
            if (r >= 1 && r <= P.nth - 2 && i >= 0 && i <= P.nr - 2) {
                const ThetaRow R = P.rows[r];
                // stage 2/3 at nodes i and i + 1: Pi~ and dPi sources (zero off
                // the interior columns), then stage 4's half-level lambda_Pi
                double2 aq[2], dqv[2];
                for (int t = 0; t < 2; ++t) {
                    const int ii = i + t;
                    double2 nq = cz(), ndq = cz();
                    if (ii >= 1 && ii <= P.nr - 2) {
                        const double2 p = P.lam_phi[static_cast<size_t>(r) * P.ld + ii];
                        const double2 q = P.lam_pi[static_cast<size_t>(r) * P.ld + ii];
                        const Coef cf = coef_at(load_rcol(P.rnode, P.nr, ii), R.cos_th, R.sin2, P.kerr != 0);
                        const double2 ctq = cmul_conj(cf.ct, q);
                        nq = make_double2(dt * (p.x - ctq.x), dt * (p.y - ctq.y));
                        ndq = make_double2(dt * cf.b * q.x, dt * cf.b * q.y);
                    }
                    aq[t] = make_double2(0.5 * nq.x, 0.5 * nq.y);
                    dqv[t] = make_double2(ndq.x * inv_hr, ndq.y * inv_hr);
                }
                const double2 hq = c_add(c_add(aq[0], dqv[0]), c_sub(aq[1], dqv[1]));
                v = hdt * re_dot_conj(hq, P.fh[c]);
            }
        }
    }
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off);
    if (dc == 0) P.dA_part[b] = v;
}

// Rows a segment must keep from the poles to take the interior form:
// jlo >= kAdjLoRows, jlo + SEG <= nth - kAdjHiRows (the stages read rows
// jlo-4 .. jhi+5 and fold the pole rows into rows 1, 2, nth-3, nth-2).
constexpr int kAdjLoRows = 7, kAdjHiRows = 7;

// Blocks at the front of a part-3 launch that compute dL/dA from the windows
// (four window rows per block).
__host__ __device__ __forceinline__ int dA_blocks(int win_t) { return (2 * win_t + 3) / 4; }

// PART selects the waves a launch runs: 0 all of them; 1 those that meet no
// source window; 2 those that do (its grid covers only the rectangle of
// items near the windows, P.sub_*); 3 all of them without their source
// terms, dL/dA coming from the window rows that the launch's first blocks
// sum (source_dA_row).  A launch of part 1 or 3 carries no source bodies and
// so fits two waves per SIMD without spills at seg 4 (248 VGPRs) and 16;
// at seg 8 a few registers of the general form spill.  The kernel with all
// four bodies runs one wave per SIMD.  Parts 1 and 2 together run every wave once, each through
// the same body as part 0; the source terms only add to dL/dA, so every
// part gives lambda^n the same bits.
template <int SEG, int PART, bool CAPPED>
__device__ __forceinline__ void adjoint_iteration(const AdjointParams& P, const ThetaRow* __restrict__ rows) {
    const int lane = threadIdx.x & 63;
    // wave-uniform work item in a scalar register (row branches become scalar
    // and the angular records, a separate __restrict__ argument, are fetched
    // through the scalar cache)
    int item;
    if constexpr (PART == 2) {   // only the rectangle of items near the source windows
        const int local = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
        if (local >= P.sub_ns * P.sub_ng) return;
        const int a = local / P.sub_ng;
        item = (P.sub_s0 + a) * P.nseg + P.sub_g0 + (local - a * P.sub_ng);
    } else {
        // part 3: the window dL/dA blocks first; then the frame waves (round
        // robin over the XCDs), then the interior ones (each XCD a contiguous
        // range)
        int blk = blockIdx.x, nblk = gridDim.x;
        if constexpr (PART == 3) {
            const int nd = dA_blocks(P.win_t);
            if (blk < nd) {
                const int b = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));
                if (b < 2 * P.win_t) source_dA_row(P, b, lane);
                return;
            }
            blk -= nd;
            nblk -= nd;
        }
        ItemOrder o = item_order(P.nr, P.nth, P.nstrips, P.nseg, SEG, kAdjLoRows, kAdjHiRows);
        if (!P.frame_first) {   // plain item order, each XCD a contiguous range
            o.frame = 0;
            o.interior = P.nstrips * P.nseg;
        }
        const int fb = (o.frame + 3) / 4;
        if (blk < fb) {
            const int f = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));
            if (f >= o.frame) return;
            item = frame_item(o, P.nseg, f);
        } else {
            const int wg = a_xcd_remap(blk - fb, nblk - fb);
            const int k = __builtin_amdgcn_readfirstlane(wg * 4 + (threadIdx.x >> 6));
            if (k >= o.interior) return;
            item = P.frame_first ? interior_item(o, P.nseg, k) : k;
        }
        item = __builtin_amdgcn_readfirstlane(item);
        if (item < 0 || item >= P.nstrips * P.nseg) return;
    }
    const int strip = item / P.nseg;
    const int seg = item - strip * P.nseg;
    const int i = strip * 62 - 1 + lane;
    const bool in_col = (i >= 0) && (i < P.nr);
    const bool writer = in_col && lane >= 1 && lane <= 62;
    const bool interior_col = (i >= 1) && (i <= P.nr - 2);
    const bool has_half = (i >= 0) && (i <= P.nr - 2);
    const int nth = P.nth;
    const int ld = P.ld;
    const int jlo = seg * SEG;
    const int jhi = (seg == P.nseg - 1) ? nth : jlo + SEG;
    const double dt = P.dt, hdt = 0.5 * P.dt, inv_hr = P.inv_hr;
    const double dt2 = 2.0 * P.dt;   // c.c0 is C_0 / 2: dt C_0 = dt2 c.c0, hdt C_0 = dt c.c0
    const double third = 0.33333333333333331483, four_thirds = 1.3333333333333332593;

    int4 org = make_int4(0, 0, 0, 0);
    if (P.org != nullptr) org = *P.org;
    const RCol rn = load_rcol(P.rnode, P.nr, min(max(i, 0), P.nr - 1));
    const RCol rh = load_rcol(P.rhalf, P.nr, min(max(i, 0), P.nr - 2));

    double dA = 0.0;

    // Interior form (the same arithmetic on every point): all 64 columns
    // interior, the segment not the last, and every row the stages touch in
    // [3, nth-4], away from the pole rows and the rows they fold into
    // (jlo >= 7, jhi <= nth - 7).  Its range, fold and column tests are
    // constants, so the unrolled window carries no selects for them.
    // SRC: a source window meets the wave's output rows and columns; without
    // it the wave's source terms are all zero and are skipped.  (A lookup is a
    // load used at once, and its wait also waits for every load before it.)
    // The body over output rows [jlo, jhi) at segment length S (the last
    // segment of a column of segments may hold up to S + 2 rows).
    auto body = [&](auto interior_tag, auto src_tag, const int jlo, const int jhi) {
    constexpr bool FAST = decltype(interior_tag)::value;
    constexpr bool SRC = decltype(src_tag)::value;
    constexpr int S = SEG;
    // rows jlo-4 .. jhi+5 (jhi - jlo <= S + 2).  Output row r needs mu rows
    // r-2..r+2, whose pole folds can reach two rows further (rows 1, 2 <- row 0).
    constexpr int NT = S + 12;
    const int jhi_ = FAST ? jlo + S : jhi;
    // Row lags of the stages behind the row being loaded: node sources 2,
    // half-level lambda 3, half sources L5, output L7.  A half-level pole
    // fold reaches two rows ahead, so the general form runs the half sources
    // at 5 and the output at 6; the interior form has no folds and runs them
    // at 3 and 4, which keeps two fewer rows of mu and of the half-level
    // lambda live.
    constexpr int L5 = FAST ? 3 : 5;
    constexpr int L7 = FAST ? 4 : 6;
    double2 lP[NT], lQ[NT];          // lambda^{n+1}, own column, row jlo-4+t
    double2 mP[NT], mQ[NT];          // mu (after the boundary transpose)
    double2 nQ[NT], nD[NT], nDQ[NT], nC[NT], nW[NT];   // node-level sources
    double2 hP[NT], hQ[NT];          // half-level lambda at i+1/2 (unfolded)
    double2 yW[NT], cC[NT], qb[NT], dp[NT], dq[NT];    // half-level sources

    // Angular records of rows jlo-4+u: every stage at iteration it reads
    // rows at fixed offsets from its k, the newest being u = it - 2 (stage
    // 2/3).  For S <= 4 each is read once, one iteration before that first
    // use, into scalar registers (for longer segments the window's scalar
    // registers spill and each record is read where it is used).
    constexpr bool WINDOW = S <= 4;
    ThetaRow Rw[NT];
    auto fetch_rec = [&](int u) {
        const int row = jlo - 4 + u;
        Rw[u] = rows[FAST ? row : min(max(row, 0), nth - 1)];
    };
    auto rec = [&](int u) -> ThetaRow { return WINDOW ? Rw[u] : rows[jlo - 4 + u]; };

#pragma unroll
    for (int it = 0; it < NT; ++it) {
        const int jj = jlo - 4 + it;
        if (FAST ? it > S + 3 + L7 : jj > jhi + L7 - 1) continue;
        if (WINDOW && it >= 1) fetch_rec(it - 1);
        // ---- 1. load lambda^{n+1}(i, jj) ----
        {
            double2 p = cz(), q = cz();
            if (FAST || (jj >= 0 && jj < nth && in_col)) {
                p = P.lam_phi[static_cast<size_t>(jj) * ld + i];
                q = P.lam_pi[static_cast<size_t>(jj) * ld + i];
            }
            lP[it] = p;
            lQ[it] = q;
        }
        // ---- 2./3. mu and node sources at row r = jj - 2 ----
        if (it >= 2) {
            const int r = jj - 2;
            const int k = it - 2;
            double2 p = cz(), q = cz();
            const bool interior_row = FAST || ((r >= 1) && (r <= nth - 2));
            if (FAST || (interior_row && interior_col)) {
                p = lP[k];
                q = lQ[k];
                if (!FAST && P.even) {
                    if (r == 1 && it >= 3) { p = axpy(four_thirds, lP[k - 1], p); q = axpy(four_thirds, lQ[k - 1], q); }
                    if (r == 2 && it >= 4) { p = axpy(-third, lP[k - 2], p); q = axpy(-third, lQ[k - 2], q); }
                    if (r == nth - 2) { p = axpy(four_thirds, lP[k + 1], p); q = axpy(four_thirds, lQ[k + 1], q); }
                    if (r == nth - 3) { p = axpy(-third, lP[k + 2], p); q = axpy(-third, lQ[k + 2], q); }
                }
            }
            mP[k] = p;
            mQ[k] = q;
            nQ[k] = nD[k] = nDQ[k] = nC[k] = nW[k] = cz();
            if (FAST || (interior_row && interior_col)) {
                const ThetaRow R = rec(k);
                const Coef c = coef_at(rn, R.cos_th, R.sin2, P.kerr != 0);
                // Phi' = Phi + dt (Pi~ - b dPhi);  Pi' = Pi + dt (b dPi + S),
                // S = -c_t Pi~ + m_r dPhi + C_0 Phi~ + w Ang[Phi~] + F
                const double2 ctq = cmul_conj(c.ct, q);
                nQ[k] = make_double2(dt * (p.x - ctq.x), dt * (p.y - ctq.y));          // -> Pi~
                const double2 mrq = cmul_conj(c.mr, q);
                nD[k] = make_double2(dt * fma(-c.b, p.x, mrq.x), dt * fma(-c.b, p.y, mrq.y));   // -> dPhi
                nDQ[k] = make_double2(dt * c.b * q.x, dt * c.b * q.y);                // -> dPi
                const double2 c0q = cmul_conj(c.c0, q);
                nC[k] = make_double2(dt2 * c0q.x, dt2 * c0q.y);                       // -> Phi~ (row r)
                nW[k] = make_double2(dt * c.w * q.x, dt * c.w * q.y);                 // -> Ang^T
                if (SRC && r >= jlo && r < jhi_ && writer) {
                    const double2 F = src_at(P.fn, org.z, org.w, P.win_r, P.win_t, i, r);
                    dA = fma(dt, re_dot_conj(q, F), dA);
                }
            }
        }
        // ---- 4. half-level lambda at (i+1/2, r1), r1 = jj - 3 ----
        if (it >= 4) {
            const int r1 = jj - 3;
            const int k = it - 3;
            double2 ptil = cz();
            if (FAST || (r1 >= 0 && r1 < nth)) {
                ptil = nC[k];
                if (FAST || r1 - 1 >= 1) ptil = axpy(ang_weights(rec(k - 1)).alpha, nW[k - 1], ptil);
                if (FAST || (r1 >= 1 && r1 <= nth - 2)) ptil = axpy(ang_weights(rec(k)).beta, nW[k], ptil);
                if (FAST || r1 + 1 <= nth - 2) ptil = axpy(ang_weights(rec(k + 1)).gamma, nW[k + 1], ptil);
            }
            // contributions of node i to its right half (i+1/2) and left half (i-1/2)
            const double2 a = make_double2(0.5 * ptil.x, 0.5 * ptil.y);
            const double2 d = make_double2(nD[k].x * inv_hr, nD[k].y * inv_hr);
            const double2 aq = make_double2(0.5 * nQ[k].x, 0.5 * nQ[k].y);
            const double2 dqv = make_double2(nDQ[k].x * inv_hr, nDQ[k].y * inv_hr);
            const double2 leftP = c_sub(a, d), leftQ = c_sub(aq, dqv);
            const double2 nbP = from_next(leftP), nbQ = from_next(leftQ);   // node i+1's left part
            if (FAST || has_half) {
                hP[k] = c_add(c_add(a, d), nbP);
                hQ[k] = c_add(c_add(aq, dqv), nbQ);
            } else {
                hP[k] = hQ[k] = cz();
            }
        }
        // ---- 5./6. folded half-level lambda and half sources at r2 = jj - L5 ----
        // (the first half row any output needs is jlo - 1, reached at it = 3 + L5)
        if (it >= 3 + L5) {
            const int r2 = jj - L5;
            const int k = it - L5;
            yW[k] = cC[k] = qb[k] = dp[k] = dq[k] = cz();
            if (FAST || (r2 >= 1 && r2 <= nth - 2 && has_half)) {
                double2 p = hP[k], q = hQ[k];
                if (!FAST && P.even) {
                    if (r2 == 1) { p = axpy(four_thirds, hP[k - 1], p); q = axpy(four_thirds, hQ[k - 1], q); }
                    if (r2 == 2) { p = axpy(-third, hP[k - 2], p); q = axpy(-third, hQ[k - 2], q); }
                    if (r2 == nth - 2) { p = axpy(four_thirds, hP[k + 1], p); q = axpy(four_thirds, hQ[k + 1], q); }
                    if (r2 == nth - 3) { p = axpy(-third, hP[k + 2], p); q = axpy(-third, hQ[k + 2], q); }
                }
                const ThetaRow R = rec(k);
                const Coef c = coef_at(rh, R.cos_th, R.sin2, P.kerr != 0);
                // Phi^h = Phi~ + hdt (Pi~ - b dPhi);  Pi^h = Pi~ + hdt (b dPi + S)
                yW[k] = make_double2(hdt * c.w * q.x, hdt * c.w * q.y);
                const double2 c0q = cmul_conj(c.c0, q);
                cC[k] = make_double2(fma(dt, c0q.x, p.x), fma(dt, c0q.y, p.y));
                const double2 ctq = cmul_conj(c.ct, q);
                qb[k] = make_double2(fma(hdt, p.x - ctq.x, q.x), fma(hdt, p.y - ctq.y, q.y));
                const double2 mrq = cmul_conj(c.mr, q);
                dp[k] = make_double2(hdt * fma(-c.b, p.x, mrq.x), hdt * fma(-c.b, p.y, mrq.y));
                dq[k] = make_double2(hdt * c.b * q.x, hdt * c.b * q.y);
                if (SRC && r2 >= jlo && r2 < jhi_ && writer) {
                    const double2 F = src_at(P.fh, org.x, org.y, P.win_r, P.win_t, i, r2);
                    dA = fma(hdt, re_dot_conj(q, F), dA);
                }
            }
        }
        // ---- 7./8. lambda^n at (i, r3), r3 = jj - L7 ----
        if (it >= 2 + L7) {
            const int r3 = jj - L7;
            const int k = it - L7;
            double2 pb = cz();
            if (FAST || (r3 >= 0 && r3 < nth)) {
                pb = cC[k];
                if (FAST || r3 - 1 >= 1) pb = axpy(ang_weights(rec(k - 1)).alpha, yW[k - 1], pb);
                if (FAST || (r3 >= 1 && r3 <= nth - 2)) pb = axpy(ang_weights(rec(k)).beta, yW[k], pb);
                if (FAST || r3 + 1 <= nth - 2) pb = axpy(ang_weights(rec(k + 1)).gamma, yW[k + 1], pb);
            }
            // half i+1/2 gives its left node (i) 1/2 avg - diff/h, its right node (i+1) 1/2 avg + diff/h
            const double2 hpP = make_double2(0.5 * pb.x, 0.5 * pb.y);
            const double2 hdP = make_double2(dp[k].x * inv_hr, dp[k].y * inv_hr);
            const double2 hpQ = make_double2(0.5 * qb[k].x, 0.5 * qb[k].y);
            const double2 hdQ = make_double2(dq[k].x * inv_hr, dq[k].y * inv_hr);
            const double2 rightP = c_add(hpP, hdP), rightQ = c_add(hpQ, hdQ);
            const double2 fromLeftP = from_prev(rightP), fromLeftQ = from_prev(rightQ);
            if (r3 >= jlo && r3 < jhi_ && writer) {
                double2 oP = c_add(c_sub(hpP, hdP), (FAST || i >= 1) ? fromLeftP : cz());
                double2 oQ = c_add(c_sub(hpQ, hdQ), (FAST || i >= 1) ? fromLeftQ : cz());
                if (FAST || interior_col) {
                    // identity part and the dissipation transpose (mu is zero off the interior)
                    oP = c_add(oP, mP[k]);
                    oQ = c_add(oQ, mQ[k]);
                    if (P.ko_c != 0.0) {
                        const double sg = P.even ? 1.0 : -1.0;
                        double2 kp = ko_apply(cz(), -1.0, mP[k - 2], mP[k - 1], mP[k], mP[k + 1], mP[k + 2]);
                        double2 kq = ko_apply(cz(), -1.0, mQ[k - 2], mQ[k - 1], mQ[k], mQ[k + 1], mQ[k + 2]);
                        if (!FAST && (r3 == 1 || r3 == nth - 2)) {   // ghost row reflected onto this row
                            kp = axpy(sg, mP[k], kp);
                            kq = axpy(sg, mQ[k], kq);
                        }
                        oP = axpy(-P.ko_c, kp, oP);
                        oQ = axpy(-P.ko_c, kq, oQ);
                    }
                }
                if (P.gw != nullptr && i == P.i_ext) oP = c_add(oP, P.gw[r3]);
                P.out_phi[static_cast<size_t>(r3) * ld + i] = oP;
                P.out_pi[static_cast<size_t>(r3) * ld + i] = oQ;
            }
        }
        // held to two waves per SIMD: keep the scheduler from hoisting work
        // across rows, so that the live window fits without spills (where
        // each wave runs alone the barrier only delays the angular-record
        // loads, so the other launches go without it)
        if constexpr (CAPPED) __builtin_amdgcn_sched_barrier(0);
    }
    };

    const bool interior = strip >= 1 && strip * 62 + 64 <= P.nr && seg != P.nseg - 1 &&
                          jlo >= kAdjLoRows && jlo + SEG <= nth - kAdjHiRows;
    // (the launcher sets both window tables or neither)
    const int i0 = strip * 62 - 1;
    // (part 3 treats every wave as one without source terms)
    const bool src = PART != 3 && P.fh != nullptr && P.fn != nullptr && P.win_r > 0 && P.win_t > 0 &&
                     (window_meets(org, false, P.win_r, P.win_t, i0, jlo, jhi - 1) ||
                      window_meets(org, true, P.win_r, P.win_t, i0, jlo, jhi - 1));
    if (src) {   // uniform per wave
        if constexpr (PART == 1 || PART == 3) {
            return;
        } else {
            if (interior)
                body(std::true_type{}, std::true_type{}, jlo, jhi);
            else
                body(std::false_type{}, std::true_type{}, jlo, jhi);
        }
    } else {
        if constexpr (PART == 2) {
            return;
        } else {
            if (interior)
                body(std::true_type{}, std::false_type{}, jlo, jhi);
            else
                body(std::false_type{}, std::false_type{}, jlo, jhi);
        }
    }
    // ---- per-wave partial of dL/dA (fixed-order reduction afterwards) ----
    // (in part 3 the window blocks own partials 0 .. 2 win_t - 1)
    if (P.dA_part != nullptr && (PART != 3 || item >= 2 * P.win_t)) {
        double v = dA;
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off);
        if (lane == 0) P.dA_part[item] = v;
    }
}

template <int SEG, int PART>
__global__ void __launch_bounds__(256) lw_adjoint_kernel(AdjointParams P, const ThetaRow* __restrict__ rows) {
    adjoint_iteration<SEG, PART, false>(P, rows);
}

// The same iteration held to two waves per SIMD, for the launches without
// source bodies at segments of 16 rows, where both forms fit without spills
// (at 8 rows the general form would spill: those launches run uncapped).
template <int SEG, int PART>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
lw_adjoint2_kernel(AdjointParams P, const ThetaRow* __restrict__ rows) {
    static_assert(SEG == 16, "only the 16-row launches fit two waves per SIMD without spills");
    adjoint_iteration<SEG, PART, true>(P, rows);
}

// Sum n per-wave partials into *acc in a fixed order (the result depends only
// on the partials and n): block b sums the chunk [4096 b, 4096 (b + 1)), each
// thread 16 consecutive values and then a fixed tree over the block, into
// blk[b]; finish_partials_kernel adds the block sums in index order.
constexpr int kReduceChunk = 4096;

__global__ void __launch_bounds__(256) reduce_partials_kernel(const double* __restrict__ part, int n,
                                                              double* __restrict__ blk) {
    __shared__ double s[256];
    const int base = blockIdx.x * kReduceChunk + threadIdx.x * 16;
    double v = 0.0;
    for (int k = 0; k < 16; ++k)
        if (base + k < n) v += part[base + k];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if (static_cast<int>(threadIdx.x) < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) blk[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(64) finish_partials_kernel(const double* __restrict__ blk, int nb,
                                                             double* __restrict__ acc) {
    if (threadIdx.x != 0) return;
    double v = 0.0;
    for (int b = 0; b < nb; ++b) v += blk[b];
    acc[0] += v;
}

// Add g (nth complex) into column i_ext of Phi (residual injection).
__global__ void __launch_bounds__(64) inject_column_kernel(double2* __restrict__ phi, int ld, int nth, int col,
                                                           const double2* __restrict__ g) {
    for (int j = threadIdx.x; j < nth; j += 64) phi[static_cast<size_t>(j) * ld + col] = c_add(phi[static_cast<size_t>(j) * ld + col], g[j]);
}

// a += ga, b += gb on [nth][nr] dense inputs into [nth][ld] planes.
__global__ void __launch_bounds__(256) add_planes_kernel(double2* __restrict__ a, double2* __restrict__ b,
                                                         const double2* __restrict__ ga,
                                                         const double2* __restrict__ gb, int nr, int nth, int ld) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= nr || j >= nth) return;
    const size_t o = static_cast<size_t>(j) * ld + i, d = static_cast<size_t>(j) * nr + i;
    if (ga != nullptr) a[o] = c_add(a[o], ga[d]);
    if (gb != nullptr) b[o] = c_add(b[o], gb[d]);
}

hipError_t launch_add_planes(double2* a, double2* b, const double2* ga, const double2* gb, int nr, int nth,
                             int ld, hipStream_t stream) {
    hipLaunchKernelGGL(add_planes_kernel, dim3((nr + 255) / 256, nth), dim3(256), 0, stream, a, b, ga, gb, nr,
                       nth, ld);
    return hipGetLastError();
}

// The rectangle of source items is held in 16-bit fields.
bool adjoint_rect_fits(int nstrips, int nseg) { return nstrips <= INT16_MAX && nseg <= INT16_MAX; }

// At 16 rows the kernel with all four bodies does not fit its registers
// (its arrays go to scratch), so a 16-row reverse iteration with a source is
// always split; at 4 and 8 rows only where the waves outnumber the SIMDs
// (where the source-free launch runs more waves per SIMD).
bool adjoint_splits(int seg, int nstrips, int nseg, int nsimd) {
    return (seg == 16 || nstrips * nseg > nsimd) && adjoint_rect_fits(nstrips, nseg);
}

hipError_t launch_adjoint(const AdjointParams& P, int seg, int nsimd, hipStream_t stream, bool source_by_window) {
    const int items = P.nstrips * P.nseg;
    const dim3 grid(P.frame_first ? ordered_blocks(item_order(P.nr, P.nth, P.nstrips, P.nseg, seg, kAdjLoRows,
                                                              kAdjHiRows))
                                  : (items + 3) / 4),
        block(256);
    const bool src = P.fh != nullptr && P.fn != nullptr;
    // With a source whose windows stay clear of the pole rows, every wave
    // runs without source terms and dL/dA comes from the windows in the
    // launch's first blocks (part 3): one launch on any grid, and no wave
    // waits on window lookups (on 3200 x 64 at seg 4, 12.3 against 12.7 us
    // for all four bodies in one launch).  Otherwise, on a grid of more waves
    // than SIMDs, the waves without the source run in a launch of their own
    // at two waves per SIMD (seg 4), and the few with it in a second launch;
    // smaller grids run every body in one launch, where the second launch
    // would only add its cost.
    const bool by_window = src && source_by_window && P.dA_part != nullptr && P.win_r <= 64 && 2 * P.win_t <= items;
    const bool split = src && adjoint_splits(seg, P.nstrips, P.nseg, nsimd);
    switch (seg) {
        case 4:
            if (by_window) {
                // every wave without its source terms, and dL/dA from the
                // windows in the launch's first blocks
                hipLaunchKernelGGL((lw_adjoint_kernel<4, 3>), dim3(grid.x + dA_blocks(P.win_t)), block, 0, stream, P, P.rows);
            } else if (split) {
                hipLaunchKernelGGL((lw_adjoint_kernel<4, 1>), grid, block, 0, stream, P, P.rows);
                const int sub = P.sub_ns * P.sub_ng;
                if (sub > 0)
                    hipLaunchKernelGGL((lw_adjoint_kernel<4, 2>), dim3((sub + 3) / 4), block, 0, stream, P,
                                       P.rows);
            } else if (src) {
                hipLaunchKernelGGL((lw_adjoint_kernel<4, 0>), grid, block, 0, stream, P, P.rows);
            } else {
                hipLaunchKernelGGL((lw_adjoint_kernel<4, 1>), grid, block, 0, stream, P, P.rows);
            }
            break;
        case 8:
            if (by_window) {
                hipLaunchKernelGGL((lw_adjoint_kernel<8, 3>), dim3(grid.x + dA_blocks(P.win_t)), block, 0, stream, P, P.rows);
            } else if (split) {
                hipLaunchKernelGGL((lw_adjoint_kernel<8, 1>), grid, block, 0, stream, P, P.rows);
                const int sub = P.sub_ns * P.sub_ng;
                if (sub > 0)
                    hipLaunchKernelGGL((lw_adjoint_kernel<8, 2>), dim3((sub + 3) / 4), block, 0, stream, P,
                                       P.rows);
            } else if (src) {
                hipLaunchKernelGGL((lw_adjoint_kernel<8, 0>), grid, block, 0, stream, P, P.rows);
            } else {
                hipLaunchKernelGGL((lw_adjoint_kernel<8, 1>), grid, block, 0, stream, P, P.rows);
            }
            break;
        case 16:
            if (by_window) {
                hipLaunchKernelGGL((lw_adjoint2_kernel<16, 3>), dim3(grid.x + dA_blocks(P.win_t)), block, 0, stream, P, P.rows);
            } else if (split) {
                hipLaunchKernelGGL((lw_adjoint2_kernel<16, 1>), grid, block, 0, stream, P, P.rows);
                const int sub = P.sub_ns * P.sub_ng;
                if (sub > 0)
                    hipLaunchKernelGGL((lw_adjoint_kernel<16, 2>), dim3((sub + 3) / 4), block, 0, stream, P,
                                       P.rows);
            } else if (src) {
                hipLaunchKernelGGL((lw_adjoint_kernel<16, 0>), grid, block, 0, stream, P, P.rows);
            } else {
                hipLaunchKernelGGL((lw_adjoint2_kernel<16, 1>), grid, block, 0, stream, P, P.rows);
            }
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int reduce_partials_blocks(int n) { return (n + kReduceChunk - 1) / kReduceChunk; }

// blk holds reduce_partials_blocks(n) doubles.
hipError_t launch_reduce_partials(const double* part, int n, double* blk, double* acc, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int nb = reduce_partials_blocks(n);
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(nb), dim3(256), 0, stream, part, n, blk);
    hipLaunchKernelGGL(finish_partials_kernel, dim3(1), dim3(64), 0, stream, blk, nb, acc);
    return hipGetLastError();
}

hipError_t launch_inject_column(double2* phi, int ld, int nth, int col, const double2* g, hipStream_t stream) {
    hipLaunchKernelGGL(inject_column_kernel, dim3(1), dim3(64), 0, stream, phi, ld, nth, col, g);
    return hipGetLastError();
}

}  // namespace teuk

namespace teuk {

// ---------------------------------------------------------------------------
// Helpers of the checkpointed gradient: a loss on a rectangle of Phi and the
// injection of its gradient.
// ---------------------------------------------------------------------------

// part[row - j0] = sum_{i0 <= i < i1} |Phi(row, i)|^2 (one block per row, fixed order).
__global__ void __launch_bounds__(256) region_sumsq_kernel(const double2* __restrict__ phi, int ld, int i0,
                                                           int i1, int j0, double* __restrict__ part) {
    __shared__ double red[256];
    const int j = j0 + blockIdx.x;
    double v = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
        const double2 u = phi[static_cast<size_t>(j) * ld + i];
        v = fma(u.x, u.x, fma(u.y, u.y, v));
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// lam(row, i) += scale * src(row, i) over the rectangle; src is either a
// plane with pitch src_ld at the same coordinates, or a dense region buffer
// (src_ld = i1 - i0, origin (j0, i0) subtracted).
__global__ void __launch_bounds__(256) add_region_kernel(double2* __restrict__ lam, int ld,
                                                         const double2* __restrict__ src, int src_ld,
                                                         bool dense, double scale, int i0, int i1, int j0) {
    const int i = i0 + blockIdx.x * blockDim.x + threadIdx.x;
    const int j = j0 + blockIdx.y;
    if (i >= i1) return;
    const double2 s = dense ? src[static_cast<size_t>(blockIdx.y) * src_ld + (i - i0)]
                            : src[static_cast<size_t>(j) * src_ld + i];
    double2& l = lam[static_cast<size_t>(j) * ld + i];
    l = make_double2(fma(scale, s.x, l.x), fma(scale, s.y, l.y));
}

hipError_t launch_region_sumsq(const double2* phi, int ld, int i0, int i1, int j0, int j1, double* part,
                               hipStream_t stream) {
    hipLaunchKernelGGL(region_sumsq_kernel, dim3(j1 - j0), dim3(256), 0, stream, phi, ld, i0, i1, j0, part);
    return hipGetLastError();
}

hipError_t launch_add_region(double2* lam, int ld, const double2* src, int src_ld, bool dense, double scale,
                             int i0, int i1, int j0, int j1, hipStream_t stream) {
    hipLaunchKernelGGL(add_region_kernel, dim3((i1 - i0 + 255) / 256, j1 - j0), dim3(256), 0, stream, lam, ld,
                       src, src_ld, dense, scale, i0, i1, j0);
    return hipGetLastError();
}

}  // namespace teuk
