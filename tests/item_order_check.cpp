// Host check of the streaming kernels' dispatch order (item_order.h): for
// many grid shapes, segment lengths and both kernels' interior bounds, the
// frame and interior positions map one to one onto the work items, and each
// item lands in the group that the kernel's own interior test puts it in.
// Built and run by tests/test_item_order.py with a host compiler.
#define __host__
#define __device__
#include "item_order.h"

#include <cstdio>
#include <vector>

using namespace teuk;

int main() {
    long cases = 0, bad = 0;
    const int bounds[2][2] = {{4, 2}, {7, 7}};   // stencil, adjoint
    for (const auto& bd : bounds)
        for (int seg : {4, 8, 16})
            for (int nr : {5, 40, 63, 64, 65, 126, 127, 128, 189, 200, 801, 1600, 3200, 6400, 12800, 25600})
                for (int nth = 5; nth <= 300; ++nth) {
                    const int nstrips = (nr + 61) / 62, nseg = (nth - 3) / seg + 1;
                    const ItemOrder o = item_order(nr, nth, nstrips, nseg, seg, bd[0], bd[1]);
                    auto interior = [&](int it) {
                        const int s = it / nseg, g = it % nseg, jlo = g * seg;
                        return s >= 1 && s * 62 + 64 <= nr && g != nseg - 1 && jlo >= bd[0] &&
                               jlo + seg <= nth - bd[1];
                    };
                    std::vector<int> seen(static_cast<size_t>(nstrips) * nseg, 0);
                    for (int f = 0; f < o.frame; ++f) {
                        const int it = frame_item(o, nseg, f);
                        if (it < 0 || it >= nstrips * nseg || interior(it)) { ++bad; continue; }
                        seen[it]++;
                    }
                    for (int k = 0; k < o.interior; ++k) {
                        const int it = interior_item(o, nseg, k);
                        if (it < 0 || it >= nstrips * nseg || !interior(it)) { ++bad; continue; }
                        seen[it]++;
                    }
                    for (int v : seen)
                        if (v != 1) ++bad;
                    if (ordered_blocks(o) * 4 < nstrips * nseg) ++bad;
                    ++cases;
                }
    std::printf("cases %ld bad %ld\n", cases, bad);
    return bad != 0;
}
