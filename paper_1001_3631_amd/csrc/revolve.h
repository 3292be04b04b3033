// Binomial checkpoint schedule for the checkpointed gradient: the order in
// which the forward is advanced, its states stored and restored, and the
// reverse iterations run, given a fixed number of full-state snapshot slots.
// Host code only; not part of the ABI.
#pragma once

#include <cstdint>
#include <vector>

namespace teuk_detail {

enum RevolveOp : int32_t {
    kAdvance = 0,   // a iterations forward from the current state (b: the iteration reached)
    kStore = 1,     // copy the current state u^b into slot a
    kRestore = 2,   // copy slot a (holding u^b) into the current state
    kReverse = 3,   // reverse iteration a (lambda^{a+1} -> lambda^a); the current state is u^a
};

struct RevolveAction {
    int32_t op;
    int64_t a, b;
};

struct RevolveSchedule {
    std::vector<RevolveAction> forward;    // from u^0 to u^nsteps, storing the first checkpoints
    std::vector<RevolveAction> backward;   // from u^nsteps (current) down to reverse iteration 0
    int64_t repetitions = 0;               // r: binomial(slots + r, slots) >= nsteps, r smallest
    int64_t backward_advances = 0;         // forward iterations recomputed in the backward
    int64_t slots_used = 0;                // largest number of slots held at once
};

// Number of iterations a binomial schedule with s snapshots (the start
// state's included) and r forward repetitions can reverse: C(s + r, s),
// saturating at 2^62.
int64_t revolve_beta(int64_t s, int64_t r);

// Builds the schedule for nsteps >= 1 iterations and slots >= 1 snapshot
// slots (slot 0 receives u^0).  Returns false only if the inputs are out of
// range.
bool revolve_schedule(int64_t nsteps, int64_t slots, RevolveSchedule* out);

}  // namespace teuk_detail
