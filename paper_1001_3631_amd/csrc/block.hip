// Temporally blocked stepping: K Lax-Wendroff iterations per launch.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "lw_point.h"
#include "stream_level.h"

namespace teuk {

// Temporal blocking: K consecutive iterations in one launch.  A work item is
// one wave (a workgroup of 64 threads) on 64 columns and a theta segment.
// Level l (1..K) produces rows [jlo - 2(K-l), jhi + 2(K-l)) clipped to the
// grid: each iteration widens the dependence by 2 rows (the full step reads
// u^n at j-2..j+2) and one column on each side, so the 64 lanes end with
// 64 - 2K owner columns.  Levels 1..K-1 stay in this wave's LDS buffer; only
// level K is written to HBM.  Every point goes through stream_level, so a
// block is bitwise identical to K single iterations.  FAST: every level is
// interior (see stream_level) and has SEG + 4(K - L) rows.  SRC: some level's
// source window meets the wave (else no level does lookups).  The lookups
// are read where used: fetching them ahead, as the single-step kernel does,
// would take this kernel past 256 VGPRs and every wave to one per SIMD, for
// the few waves that have them.
template <int SEG, int K, int L, bool FAST, bool SRC>
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
    stream_level<NROW, (L > 1), (L < K), kPrefetchRows, FAST ? SEG + 4 * (K - L) : 0, SRC>(P, A, rn, rh, rows);
    if constexpr (L < K) block_levels<SEG, K, L + 1, FAST, SRC>(P, A, jlo, jhi, rn, rh, rows);
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
    // level 1 (the widest) away from the poles and every lane an interior
    // column: then every level is, and all take the interior form
    const int i0 = strip * (64 - 2 * K) - K;
    const bool interior = i0 >= 1 && i0 + 63 <= P.nr - 2 && seg != P.nseg - 1 &&
                          jlo - 2 * (K - 1) >= 4 && jhi + 2 * (K - 1) <= P.nth - 2;
    // does any level's source window meet the wave's widest region (columns
    // of all 64 lanes, rows of level 1 and the half rows around them)?
    // (the origins are those the levels' lookups use)
    // The launcher sets both window tables or neither.
    bool src = false;
    if (P.fh != nullptr && P.fn != nullptr && P.win_r > 0 && P.win_t > 0) {
        for (int l = 0; l < K; ++l) {
            const int4 o = (P.org != nullptr) ? P.org[l] : make_int4(0, 0, 0, 0);
            src = src ||
                  window_meets(o, false, P.win_r, P.win_t, i0, jlo - 2 * (K - 1) - 1, jhi + 2 * (K - 1)) ||
                  window_meets(o, true, P.win_r, P.win_t, i0, jlo - 2 * (K - 1), jhi + 2 * (K - 1) - 1);
        }
    }
    // (uniform per wave; each wave runs alone on its SIMD on small grids, so
    // the source waves get the interior form too)
    if (src) {
        if (interior)
            block_levels<SEG, K, 1, true, true>(P, A, jlo, jhi, rn, rh, rows);
        else
            block_levels<SEG, K, 1, false, true>(P, A, jlo, jhi, rn, rh, rows);
    } else if (interior) {
        block_levels<SEG, K, 1, true, false>(P, A, jlo, jhi, rn, rh, rows);
    } else {
        block_levels<SEG, K, 1, false, false>(P, A, jlo, jhi, rn, rh, rows);
    }
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

}  // namespace teuk
