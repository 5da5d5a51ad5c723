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
in time, so even the bad order would end, with an error.)  The chained
launch, which runs the two-sweep blocks of several levels with one ticket
counter and adds waits for the previous level's blocks, is played the same
way.
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


def run_chain(sizes, down, slots, rng):
    """The chained launch: tickets run through the levels in order (sizes in
    ticket order).  A block of level c > 0 first waits until the blocks of
    level c-1 it reads have finished (down: restriction, blocks 2kb-2 ..
    2kb+4 of the finer level; up: interpolation, blocks kb/2-2 .. kb/2+2 of
    the coarser level), then sweeps, publishes, waits for its neighbours and
    finishes.  True if every work-group finishes."""
    starts = [0]
    for s in sizes:
        starts.append(starts[-1] + s)
    total = starts[-1]

    def level_of(t):
        c = 0
        while c + 1 < len(sizes) and t >= starts[c + 1]:
            c += 1
        return c, t - starts[c]

    pending = list(range(total))
    rng.shuffle(pending)
    next_ticket = 0
    running = {}
    first = [False] * total
    finished = [False] * total
    done = 0
    while done < total:
        while pending and len(running) < slots:
            wg = pending.pop()
            running[wg] = [next_ticket, 0]
            next_ticket += 1
        progressed = False
        for wg in rng.sample(list(running), len(running)):
            t, phase = running[wg]
            c, kb = level_of(t)
            n = sizes[c]
            if phase == 0:
                ok = True
                if c > 0:
                    nd = sizes[c - 1]
                    lo, hi = (2 * kb - 2, 2 * kb + 4) if down else (kb // 2 - 2, kb // 2 + 2)
                    lo, hi = max(lo, 0), min(hi, nd - 1)
                    ok = all(finished[starts[c - 1] + j] for j in range(lo, hi + 1))
                if ok:
                    first[t] = True
                    running[wg][1] = 1
                    progressed = True
            else:
                lo_ok = kb == 0 or first[t - 1]
                hi_ok = kb == n - 1 or first[t + 1]
                if lo_ok and hi_ok:
                    finished[t] = True
                    del running[wg]
                    done += 1
                    progressed = True
            if progressed:
                break
        if not progressed and (not pending or len(running) >= slots):
            return False
    return True


@pytest.mark.parametrize("n0,levels", [(16, 3), (64, 4), (96, 5)])
@pytest.mark.parametrize("slots", [2, 3, 8, 40])
@pytest.mark.parametrize("down", [True, False])
def test_chained_levels_always_drain(n0, levels, slots, down):
    sizes = [n0 >> l for l in range(levels)]
    if not down:
        sizes = sizes[::-1]
    rng = random.Random(7 * n0 + slots + (0 if down else 1))
    assert all(run_chain(sizes, down, slots, rng) for _ in range(40))
