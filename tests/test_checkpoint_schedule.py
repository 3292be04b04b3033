"""The binomial checkpoint schedule of the checkpointed gradient
(teuk_checkpoint_schedule, host only; Griewank's revolve).

* Replay: every schedule is executed on a symbolic state (the iteration it
  holds, the iterations the slots hold): the reverse iterations come in the
  order nsteps-1 .. 0, each with the current state at its iteration; every
  restore names a slot that holds the iteration it claims; no more slots are
  held than allowed; the forward ends at u^nsteps.
* Cost: the forward iterations recomputed in all (the first descent's,
  made by the forward sweep, plus the backward's) equal the minimum over
  every way of splitting, found by exhaustive search on small cases, and the
  closed form r*l - C(s + r, s + 1) on large ones.
* Limits: one slot recomputes l(l-1)/2 iterations; nsteps slots recompute
  none; bad arguments are refused.
"""

import ctypes
from functools import lru_cache
from math import comb

import numpy as np
import pytest

from paper_1001_3631_amd import _lib as L
from paper_1001_3631_amd.engine import checkpoint_schedule

ADVANCE, STORE, RESTORE, REVERSE = 0, 1, 2, 3


def replay(nsteps, snapshots):
    fwd, bwd, stats = checkpoint_schedule(nsteps, snapshots)
    cur, slots, descent = 0, {}, 0
    for op, a, b in fwd:
        if op == STORE:
            assert b == cur and 0 <= a < snapshots and a not in slots
            slots[a] = cur
            descent = cur
        else:
            assert op == ADVANCE and a >= 1 and b == cur + a
            cur = b
    assert cur == nsteps and slots.get(0) == 0
    held = len(slots)
    most = held
    advances = 0
    expect = nsteps - 1
    # a slot is free again once every reverse iteration at or after its
    # iteration has run
    for op, a, b in bwd:
        for k in [k for k, t in slots.items() if t > expect]:
            del slots[k]
        if op == ADVANCE:
            assert a >= 1 and b == cur + a
            cur = b
            advances += a
        elif op == STORE:
            assert b == cur and 0 <= a < snapshots and a not in slots, (a, slots)
            slots[a] = cur
        elif op == RESTORE:
            assert slots.get(a) == b, (a, b, slots)
            cur = b
        else:
            assert op == REVERSE and a == expect and cur == a, (a, expect, cur)
            expect -= 1
        most = max(most, len(slots))
    assert expect == -1
    assert most <= snapshots
    assert stats[1] == advances
    return descent, advances, stats


@lru_cache(None)
def optimum(l, c):
    """Fewest forward iterations to reverse l iterations from a held start
    state with c further slots: every split tried."""
    if l == 1:
        return 0
    if c == 0:
        return l * (l - 1) // 2
    return min(m + optimum(l - m, c - 1) + optimum(m, c) for m in range(1, l))


def closed_form(l, s):
    r = 0
    while comb(s + r, s) < l:
        r += 1
    return r, r * l - comb(s + r, s + 1)


@pytest.mark.parametrize("snapshots", [1, 2, 3, 4, 6])
def test_schedule_is_valid_and_optimal_on_small_cases(snapshots):
    for n in range(1, 70):
        descent, advances, stats = replay(n, snapshots)
        assert descent + advances == optimum(n, snapshots - 1), (n, snapshots)
        if n > 1:
            assert stats[0] == closed_form(n, snapshots)[0]


@pytest.mark.parametrize("n,snapshots", [(500, 10), (2000, 7), (50000, 171), (50000, 145), (4096, 64),
                                         (997, 31)])
def test_schedule_cost_matches_closed_form(n, snapshots):
    descent, advances, stats = replay(n, snapshots)
    r, cost = closed_form(n, snapshots)
    assert stats[0] == r
    assert descent + advances == cost
    assert stats[2] <= snapshots


def test_limits():
    _, advances, _ = replay(40, 1)
    assert advances == 40 * 39 // 2           # one slot: restart from u^0 for every reverse iteration
    descent, advances, stats = replay(40, 40)
    assert advances == 0 and descent == 39     # a slot per iteration: the forward stores everything
    _, advances, stats = replay(1, 1)
    assert advances == 0


def test_bad_arguments_are_refused():
    lib = L.load()
    count = ctypes.c_int64()
    for n, s, phase in ((0, 3, 0), (10, 0, 0), (10, 3, 2), (-5, 3, 1)):
        assert lib.teuk_checkpoint_schedule(n, s, phase, None, 0, ctypes.byref(count), None) == L.TEUK_EINVAL
    buf = np.zeros((2, 3), dtype=np.int64)
    # a short buffer receives the first actions; the count is the full one
    assert lib.teuk_checkpoint_schedule(100, 3, 1, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 2,
                                        ctypes.byref(count), None) == L.TEUK_OK
    assert count.value > 2
    full = checkpoint_schedule(100, 3)[1]
    assert np.array_equal(buf, full[:2])
