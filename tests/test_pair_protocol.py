"""Liveness of the hand-off order used by the two-sweep kernel (CPU model).

The two-sweep launch runs one work-group per block k = 1..n (the last one
also takes block n+1).  After its first sweep a work-group publishes a flag
and waits for the flags of blocks k-1 and k+1 before its second sweep.  The
device holds only so many work-groups at once and may start them in any
order, so the kernel does not use its launch index as the block: each
work-group draws the next value of a counter when it starts.

This model plays that protocol against a dispatcher that starts pending
work-groups in random order whenever a slot is free, and checks that every
schedule drains whenever at least two work-groups fit.  The same model with
the launch index as the block shows schedules that never drain, which is the
case the ticket order exists for.  (On the device every wait is also bounded
in time, so even the bad order would end, with an error.)
"""
import random

import pytest


def run(n, slots, policy, rng):
    """True if all n work-groups finish; False on a deadlock."""
    pending = list(range(n))                   # launch indices not yet started
    rng.shuffle(pending)                       # any start order
    next_ticket = 0
    running = {}                               # wg -> [block, phase]
    flags = [False] * n
    done = 0
    while done < n:
        # start work-groups while slots are free
        while pending and len(running) < slots:
            wg = pending.pop()
            block = next_ticket if policy == "ticket" else wg
            next_ticket += 1
            running[wg] = [block, 0]
        progressed = False
        for wg in rng.sample(list(running), len(running)):
            block, phase = running[wg]
            if phase == 0:                     # first sweep never waits
                flags[block] = True
                running[wg][1] = 1
                progressed = True
            elif phase == 1:
                lo_ok = block == 0 or flags[block - 1]
                hi_ok = block == n - 1 or flags[block + 1]
                if lo_ok and hi_ok:            # second sweep, then exit
                    del running[wg]
                    done += 1
                    progressed = True
            if progressed:
                break
        if not progressed and (not pending or len(running) >= slots):
            return False
    return True


@pytest.mark.parametrize("n", [1, 2, 5, 17, 64])
@pytest.mark.parametrize("slots", [2, 3, 8])
def test_ticket_order_always_drains(n, slots):
    rng = random.Random(1000 * n + slots)
    assert all(run(n, slots, "ticket", rng) for _ in range(200))


def test_launch_index_order_can_deadlock():
    rng = random.Random(7)
    outcomes = [run(17, 3, "index", rng) for _ in range(200)]
    assert not all(outcomes)


def test_one_slot_is_not_enough():
    # the first work-group waits for block 2, which cannot start
    assert not run(4, 1, "ticket", random.Random(0))
