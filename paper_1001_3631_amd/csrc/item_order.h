// Dispatch order of the streaming kernels' work items (wave = strip of 62
// columns x segment of rows; item = strip * nseg + segment).  The waves that
// take a kernel's general form (first and last strips, segments near the
// poles, the last segment: the "frame") are dispatched first, so that their
// longer bodies run alongside the interior waves instead of trailing them;
// the interior waves follow in item order.  Host and device code.
#pragma once

namespace teuk {

struct ItemOrder {
    int g_lo, g_hi;   // interior segments [g_lo, g_hi)
    int s_hi;         // interior strips [1, s_hi)
    int nb;           // frame segments of an interior strip
    int frame, interior;
};

// The kernel's interior test: strip >= 1, strip * 62 + 64 <= nr, segment
// not the last, jlo >= lo_rows and jlo + seg <= nth - hi_rows.
__host__ __device__ inline ItemOrder item_order(int nr, int nth, int nstrips, int nseg, int seg, int lo_rows,
                                                int hi_rows) {
    ItemOrder o;
    o.g_lo = (lo_rows + seg - 1) / seg;
    const int gh = (nth - hi_rows - seg >= 0) ? (nth - hi_rows - seg) / seg + 1 : 0;
    o.g_hi = gh < nseg - 1 ? gh : nseg - 1;
    const int sh = (nr >= 64) ? (nr - 64) / 62 + 1 : 0;
    o.s_hi = sh < nstrips ? sh : nstrips;
    const int ng = o.g_hi - o.g_lo, ns = o.s_hi - 1;
    o.interior = (ng > 0 && ns > 0) ? ng * ns : 0;
    o.frame = nstrips * nseg - o.interior;
    o.nb = nseg - (ng > 0 ? ng : 0);
    return o;
}

// Item of frame position f, 0 <= f < o.frame.
__host__ __device__ inline int frame_item(const ItemOrder& o, int nseg, int f) {
    if (o.interior == 0) return f;
    if (f < nseg) return f;   // strip 0
    f -= nseg;
    const int mid = (o.s_hi - 1) * o.nb;
    if (f < mid) {            // the frame segments of the interior strips
        const int s = 1 + f / o.nb;
        const int k = f - (s - 1) * o.nb;
        const int g = (k < o.g_lo) ? k : o.g_hi + (k - o.g_lo);
        return s * nseg + g;
    }
    return o.s_hi * nseg + (f - mid);   // the last strips
}

// Item of interior position k, 0 <= k < o.interior.
__host__ __device__ inline int interior_item(const ItemOrder& o, int nseg, int k) {
    const int ng = o.g_hi - o.g_lo;
    const int s = 1 + k / ng;
    return s * nseg + o.g_lo + (k - (s - 1) * ng);
}

// Workgroups (4 waves each) of a launch in this order.
__host__ __device__ inline int ordered_blocks(const ItemOrder& o) { return (o.frame + 3) / 4 + (o.interior + 3) / 4; }

// The order pays only when a launch has more waves than the device has
// SIMDs: with every wave resident at once, sending a strip's frame and
// interior segments to different XCDs only costs L2 locality.
__host__ __device__ inline bool use_frame_first(int items, int nsimd) { return items > nsimd; }

}  // namespace teuk
