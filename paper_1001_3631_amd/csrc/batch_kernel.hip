// Batched stepping of many independent instances: the persistent kernel and
// the one-launch-per-iteration kernel.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "lw_point.h"
#include "stream_level.h"

namespace teuk {

// Rows of u^n fetched ahead in the batched kernel.  It keeps its instance
// fields in scalar registers, which leaves room for the same prefetch as the
// single-step kernel at two waves per SIMD.
#ifndef TEUK_BATCH_PREFETCH_ROWS
#define TEUK_BATCH_PREFETCH_ROWS 2
#endif
constexpr int kBatchPrefetchRows = TEUK_BATCH_PREFETCH_ROWS;

namespace {

// A value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
template <typename T>
__device__ __forceinline__ T* uni(T* p) {
    const unsigned long long a = reinterpret_cast<unsigned long long>(p);
    const unsigned long long hi = static_cast<unsigned int>(__builtin_amdgcn_readfirstlane(static_cast<int>(a >> 32)));
    const unsigned long long lo = static_cast<unsigned int>(__builtin_amdgcn_readfirstlane(static_cast<int>(a)));
    return reinterpret_cast<T*>((hi << 32) | lo);
}

// Source windows of iteration n of the launch (an instance's fh, fn, org,
// win_r, win_t; see BatchInstance) into P and A, and whether they meet the
// wave's columns [i0, i0 + 63] around the rows [A.lo, A.hi).
__device__ __forceinline__ void batch_source(const double2* fh, const double2* fn, const int4* org, int win_r,
                                             int win_t, int n, StepParams& P, LevelArgs& A) {
    if (fh == nullptr || fn == nullptr || org == nullptr || win_r <= 0 || win_t <= 0) return;
    const size_t wsz = static_cast<size_t>(win_r) * win_t;
    P.win_r = win_r;
    P.win_t = win_t;
    A.fh = global_ptr(fh + static_cast<size_t>(n) * wsz);
    A.fn = global_ptr(fn + static_cast<size_t>(n) * wsz);
    A.org = constant_ptr(org)[n];
}
__device__ __forceinline__ bool source_meets(const StepParams& P, const LevelArgs& A, int i0) {
    return A.fh != nullptr && (window_meets(A.org, false, P.win_r, P.win_t, i0, A.lo - 1, A.hi) ||
                               window_meets(A.org, true, P.win_r, P.win_t, i0, A.lo, A.hi - 1));
}

}  // namespace

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
        // every lane read the same values: move them to scalar registers, so
        // that the exit and everything after it are wave-uniform
        const unsigned long long tv = s_t;
        const unsigned long long t =
            (static_cast<unsigned long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(tv >> 32))) << 32) |
            static_cast<unsigned int>(__builtin_amdgcn_readfirstlane(static_cast<int>(tv & 0xffffffffu)));
        const int stop = __builtin_amdgcn_readfirstlane(s_stop);
        if (stop != 0 || t >= total) break;

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

        // the instance's fields are the same in every lane: keep them in
        // scalar registers (the vector registers go to the stencil); the
        // pointers are rebuilt as global (planes, radial records) and constant
        // (angular records, never written) pointers
        StepParams P;
        const int lv = uni(I.cur + n) & 1;
        P.phi = global_ptr(uni(I.plane[lv][0]));
        P.pi = global_ptr(uni(I.plane[lv][1]));
        P.phi_out = global_ptr(uni(I.plane[lv ^ 1][0]));
        P.pi_out = global_ptr(uni(I.plane[lv ^ 1][1]));
        P.rnode = global_ptr(uni(I.rnode));
        P.rhalf = global_ptr(uni(I.rhalf));
        P.rows = constant_ptr(uni(I.rows));
        P.nr = uni(I.nr);
        P.nth = uni(I.nth);
        P.ld = uni(I.ld);
        P.rpitch = uni(I.rpitch);
        P.nstrips = uni(I.nstrips);
        P.nseg = uni(I.nseg);
        P.dt = uni(I.dt);
        P.inv_hr = uni(I.inv_hr);
        P.ko_c = uni(I.ko_c);
        P.even = uni(I.even);
        P.kerr = uni(I.kerr);
        P.i_ext = uni(I.i_ext);
        P.wave = nullptr;
        P.fh = P.fn = nullptr;
        P.org = nullptr;
        P.win_r = P.win_t = 0;
        double2* const wave = global_ptr(uni(I.wave));
        LevelArgs A;
        A.lane = lane;
        A.i = strip * 62 - 1 + lane;
        A.halo = 1;
        A.fh = A.fn = nullptr;
        A.org = make_int4(0, 0, 0, 0);
        A.wave = wave ? wave + static_cast<size_t>(n) * P.nth : nullptr;
        A.lp = A.lq = nullptr;
        A.lbase = 0;
        batch_source(uni(I.fh), uni(I.fn), uni(I.org), uni(I.win_r), uni(I.win_t), n, P, A);
        const int ic = min(max(A.i, 0), P.nr - 1);
        const int ih = min(max(A.i, 0), P.nr - 2);
        const RCol rn = load_rcol(P.rnode, P.rpitch, ic);
        const RCol rh = load_rcol(P.rhalf, P.rpitch, ih);
        // segments away from the poles on a strip of interior columns take
        // the interior form of the level, segments a source window meets the
        // form with lookups (the same arithmetic)
        const bool cols_interior = strip >= 1 && strip * 62 + 64 <= P.nr;
        for (int q = 0; q < P.nseg; ++q) {
            A.lo = q * SEG;
            A.hi = (q == P.nseg - 1) ? P.nth : A.lo + SEG;
            if (source_meets(P, A, strip * 62 - 1))
                stream_level<SEG + 2, false, false, kBatchPrefetchRows, 0, true>(P, A, rn, rh, P.rows);
            else if (cols_interior && q != P.nseg - 1 && A.lo >= 4 && A.hi <= P.nth - 2)
                stream_level<SEG + 2, false, false, kBatchPrefetchRows, SEG>(P, A, rn, rh, P.rows);
            else
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

hipError_t launch_batch_reset(const BatchParams& B, hipStream_t stream) {
    hipLaunchKernelGGL(batch_reset_kernel, dim3((B.ntiles + 255) / 256), dim3(256), 0, stream, B);
    return hipGetLastError();
}

// One iteration of every instance of a batch in one launch (the batch's
// per-iteration mode): the launch boundary orders the iterations, so there
// are no dependency counters or fences.  Work item = one wave on (instance,
// strip of 62 columns, theta segment), numbered instance-major: the items of
// instance k are [item0[k], item0[k+1]), strip-major as in lw_step_kernel.
// Four waves per workgroup; the instance table and item0 are read-only for
// the launch, so the wave-uniform reads go through the scalar cache.
template <int SEG>
__global__ void __launch_bounds__(256) lw_multi_kernel(const BatchInstance* __restrict__ inst,
                                                       const int* __restrict__ item0, int ninst, int base,
                                                       int n) {
    const int lane = threadIdx.x & 63;
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    const int item = __builtin_amdgcn_readfirstlane(base + wg * 4 + (threadIdx.x >> 6));
    if (item >= item0[ninst]) return;   // uniform per wave
    // instance: the last k with item0[k] <= item (item0 is non-decreasing)
    int k0 = 0, k1 = ninst - 1;
    while (k0 < k1) {
        const int mid = (k0 + k1 + 1) >> 1;
        if (item0[mid] <= item) k0 = mid;
        else k1 = mid - 1;
    }
    const BatchInstance& I = inst[k0];
    const int local = item - item0[k0];
    const int strip = local / I.nseg;
    const int seg = local - strip * I.nseg;

    StepParams P;
    const int lv = (I.cur + n) & 1;
    P.phi = global_ptr(I.plane[lv][0]);
    P.pi = global_ptr(I.plane[lv][1]);
    P.phi_out = global_ptr(I.plane[lv ^ 1][0]);
    P.pi_out = global_ptr(I.plane[lv ^ 1][1]);
    P.rnode = global_ptr(I.rnode);
    P.rhalf = global_ptr(I.rhalf);
    P.rows = constant_ptr(I.rows);
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
    A.wave = I.wave ? global_ptr(I.wave) + static_cast<size_t>(n) * P.nth : nullptr;
    A.lp = A.lq = nullptr;
    A.lbase = 0;
    A.lo = seg * SEG;
    A.hi = (seg == P.nseg - 1) ? P.nth : A.lo + SEG;
    batch_source(I.fh, I.fn, I.org, I.win_r, I.win_t, n, P, A);
    const int ic = min(max(A.i, 0), P.nr - 1);
    const int ih = min(max(A.i, 0), P.nr - 2);
    const RCol rn = load_rcol(P.rnode, P.rpitch, ic);
    const RCol rh = load_rcol(P.rhalf, P.rpitch, ih);
    const bool interior = strip >= 1 && strip * 62 + 64 <= P.nr && seg != P.nseg - 1 && A.lo >= 4 &&
                          A.hi <= P.nth - 2;
    if (source_meets(P, A, strip * 62 - 1))   // uniform per wave
        stream_level<SEG + 2, false, false, kPrefetchRows, 0, true>(P, A, rn, rh, P.rows);
    else if (interior)
        stream_level<SEG + 2, false, false, kPrefetchRows, SEG>(P, A, rn, rh, P.rows);
    else
        stream_level<SEG + 2, false, false, kPrefetchRows>(P, A, rn, rh, P.rows);
}

hipError_t launch_batch_iteration(const BatchInstance* inst, const int* item0, int ninst, int base, int items,
                                  int n, int seg, hipStream_t stream) {
    if (items <= 0) return hipSuccess;
    const dim3 grid((items + 3) / 4), block(256);
    switch (seg) {
        case 4: hipLaunchKernelGGL(lw_multi_kernel<4>, grid, block, 0, stream, inst, item0, ninst, base, n); break;
        case 8: hipLaunchKernelGGL(lw_multi_kernel<8>, grid, block, 0, stream, inst, item0, ninst, base, n); break;
        case 16: hipLaunchKernelGGL(lw_multi_kernel<16>, grid, block, 0, stream, inst, item0, ninst, base, n); break;
        default: return hipErrorInvalidValue;
    }
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

}  // namespace teuk
