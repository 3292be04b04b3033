// Binomial checkpointing (Griewank's "revolve" schedule; Griewank and
// Walther, ACM TOMS 26 (2000) 19-45), written for the checkpointed gradient
// of the Lax-Wendroff iteration (Sec. 3.2).
//
// With s snapshots (the one holding the segment's start state included) and
// r forward repetitions, at most beta(s, r) = C(s + r, s) iterations can be
// reversed, and reversing l iterations costs r*l - beta(s + 1, r - 1)
// forward iterations with r the smallest repetition number that covers l.
// A segment of l iterations starting at a stored state is reversed by
// advancing m iterations, storing that state in a free slot, reversing the
// right part (l - m iterations, one slot fewer), releasing the slot and then
// reversing the left part (m iterations, as many slots as before).  The
// split m = max(1, beta(s, r - 2), l - beta(s - 1, r)) reaches the minimal
// cost at every (l, s) (checked against an exhaustive search over every
// split in the tests); its right part then needs at most r repetitions with
// s - 1 snapshots and its left part at most r - 1 with s.
//
// The forward sweep runs all nsteps iterations anyway (its waveform defines
// the loss), so it stores the checkpoints of the schedule's first descent
// (the right-most path of the recursion); the backward starts from u^nsteps
// and finds those checkpoints already stored.

#include "revolve.h"

#include <algorithm>
#include <map>

namespace teuk_detail {

namespace {

constexpr int64_t kBetaCap = int64_t(1) << 62;

// Smallest r with beta(s, r) >= l.
int64_t repetitions(int64_t l, int64_t s) {
    int64_t r = 0;
    while (revolve_beta(s, r) < l) ++r;
    return r;
}

// First checkpoint of a segment of l >= 2 iterations with cfree >= 1 free
// slots besides the one holding its start: 1 <= m <= l - 1.
int64_t split(int64_t l, int64_t cfree) {
    const int64_t s = cfree + 1;
    const int64_t r = repetitions(l, s);
    int64_t m = std::max<int64_t>(1, l - revolve_beta(s - 1, r));
    if (r >= 2) m = std::max(m, revolve_beta(s, r - 2));
    return std::min(m, l - 1);
}

}  // namespace

int64_t revolve_beta(int64_t s, int64_t r) {
    if (s < 0 || r < 0) return 0;
    // C(s + r, r) = prod_{i=1..r} (s + i) / i, each partial product an integer
    int64_t v = 1;
    for (int64_t i = 1; i <= r; ++i) {
        if (v > kBetaCap / (s + i)) return kBetaCap;
        v = v * (s + i) / i;
    }
    return v;
}

bool revolve_schedule(int64_t nsteps, int64_t slots, RevolveSchedule* out) {
    if (out == nullptr || nsteps < 1 || slots < 1) return false;
    RevolveSchedule S;
    S.repetitions = repetitions(nsteps, slots);

    // Forward: u^0 into slot 0, then the first descent's checkpoints.
    std::map<int64_t, int64_t> stored;   // iteration -> slot, stored by the forward
    {
        int64_t s0 = 0, l = nsteps, cfree = slots - 1, next_slot = 1;
        S.forward.push_back({kStore, 0, 0});
        stored[0] = 0;
        while (l > 1 && cfree > 0) {
            const int64_t m = split(l, cfree);
            S.forward.push_back({kAdvance, m, s0 + m});
            S.forward.push_back({kStore, next_slot, s0 + m});
            stored[s0 + m] = next_slot++;
            s0 += m;
            l -= m;
            cfree -= 1;
        }
        S.forward.push_back({kAdvance, l, nsteps});
        S.slots_used = next_slot;
    }

    // Backward: the recursion on an explicit stack (the left part is a tail
    // call and reuses its frame).
    std::vector<int64_t> free_slots;
    for (int64_t k = slots - 1; k >= S.slots_used; --k) free_slots.push_back(k);
    int64_t in_use = S.slots_used;
    int64_t cur = nsteps;   // the iteration the current state holds
    auto need_at = [&](int64_t t, int64_t slot) {
        if (cur != t) {
            S.backward.push_back({kRestore, slot, t});
            cur = t;
        }
    };
    auto advance = [&](int64_t k) {
        if (k > 0) {
            cur += k;
            S.backward.push_back({kAdvance, k, cur});
            S.backward_advances += k;
        }
    };
    struct Frame {
        int64_t s0, l, cfree, slot, mid, right_slot;
        bool right_done;
    };
    std::vector<Frame> stack;
    stack.push_back({0, nsteps, slots - 1, 0, 0, -1, false});
    while (!stack.empty()) {
        const size_t fi = stack.size() - 1;
        Frame F = stack[fi];
        if (F.right_done) {
            // the right part is reversed: release its slot, then the left part
            free_slots.push_back(F.right_slot);
            in_use -= 1;
            stack[fi] = {F.s0, F.mid, F.cfree, F.slot, 0, -1, false};
            continue;
        }
        if (F.l == 1) {
            need_at(F.s0, F.slot);
            S.backward.push_back({kReverse, F.s0, 0});
            stack.pop_back();
            continue;
        }
        if (F.cfree == 0) {
            for (int64_t m = F.s0 + F.l - 1; m >= F.s0; --m) {
                need_at(F.s0, F.slot);
                advance(m - F.s0);
                S.backward.push_back({kReverse, m, 0});
            }
            stack.pop_back();
            continue;
        }
        const int64_t mid = split(F.l, F.cfree);
        const int64_t t = F.s0 + mid;
        int64_t rs;
        auto it = stored.find(t);
        if (it != stored.end()) {
            rs = it->second;
            stored.erase(it);
        } else {
            if (free_slots.empty()) return false;   // cannot happen: the recursion holds <= slots
            rs = free_slots.back();
            free_slots.pop_back();
            in_use += 1;
            S.slots_used = std::max(S.slots_used, in_use);
            need_at(F.s0, F.slot);
            advance(mid);
            S.backward.push_back({kStore, rs, t});
        }
        stack[fi].mid = mid;
        stack[fi].right_slot = rs;
        stack[fi].right_done = true;
        stack.push_back({t, F.l - mid, F.cfree - 1, rs, 0, -1, false});
    }
    *out = std::move(S);
    return true;
}

}  // namespace teuk_detail
