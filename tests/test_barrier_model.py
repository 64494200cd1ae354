"""Host-thread model of the device-wide round protocol of AC-3 (and of the
AC-6 forest rounds): the sense-free grid barrier (arrival counter reset by the
last arrival, generation bumped after the reset, generation read before
arriving, a poll budget as watchdog) and the three-slot rotation of the
per-round list counters (round r reads slot r % 3, appends to slot
(r + 1) % 3, block 0 clears slot (r + 2) % 3, every block ends when a round
removed nothing).

Each block is a thread; random pauses perturb the interleaving.  With every
block resident the rounds always complete with the same round count the
sequential rule gives.  With fewer resident slots than blocks (a launch that
does not fit at once) the first barrier can never be released: the resident
blocks wait until the watchdog budget ends them, which is the failure mode of
a grid barrier whose workgroups are not all co-resident.
"""
import random
import threading
import time


class Device:
    def __init__(self, blocks, budget):
        self.lock = threading.Lock()
        self.count = 0
        self.gen = 0
        self.stall = 0
        self.slots = [0, 0, 0]
        self.blocks = blocks
        self.budget = budget

    def add(self, name, v, idx=None):
        with self.lock:
            if idx is None:
                old = getattr(self, name)
                setattr(self, name, old + v)
            else:
                old = self.slots[idx]
                self.slots[idx] = old + v
            return old

    def barrier(self, rng):
        g0 = self.gen                       # read before arriving
        if self.add("count", 1) == self.blocks - 1:
            self.count = 0                  # reset, then release
            self.add("gen", 1)
        else:
            polls = 0
            while self.gen == g0:
                polls += 1
                if polls > self.budget or self.stall:
                    self.stall = 1
                    return False
                time.sleep(rng.random() * 1e-4)
        return self.stall == 0


def block(dev, b, work, rounds_out, rng):
    """Round r: read the input count, append this block's survivors of the
    round to the next slot, clear the slot after it, barrier, stop when the
    round removed nothing."""
    r = 1
    while True:
        cnt_in = dev.slots[r % 3]
        if b == 0:
            dev.slots[(r + 2) % 3] = 0
        time.sleep(rng.random() * 2e-4)
        dev.add(None, work(b, r, cnt_in), (r + 1) % 3)
        if not dev.barrier(rng):
            rounds_out[b] = -1
            return
        if dev.slots[(r + 1) % 3] == cnt_in:
            rounds_out[b] = r
            return
        r += 1


def run(blocks, resident, seed, budget=20000):
    """Blocks start only when one of `resident` slots is free (a slot frees
    when its block exits).  Returns each block's round count (-1: abandoned
    by the watchdog)."""
    rng = random.Random(seed)
    n0 = 1000
    dev = Device(blocks, budget)
    dev.slots[1] = n0
    # survivors of round r, split over the blocks: 1000, 500, 250, ... 7, 7
    def total(r):
        return max(7, n0 >> r)

    def work(b, r, cnt_in):
        t = min(total(r), cnt_in)
        return t // blocks + (1 if b < t % blocks else 0)
    out = [None] * blocks
    sem = threading.Semaphore(resident)

    def start(b):
        with sem:
            block(dev, b, work, out, random.Random(seed * 1000 + b))
    th = [threading.Thread(target=start, args=(b,)) for b in range(blocks)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=60)
    assert not any(t.is_alive() for t in th), "a block never finished"
    return out


def test_all_resident_completes_with_the_sequential_round_count():
    # sequential rule: rounds until a round removes nothing (1000, 500, ...,
    # 7, 7): 8 halvings to reach 7, then the round that keeps all 7
    want = next(r for r in range(1, 64) if max(7, 1000 >> r) == max(7, 1000 >> (r - 1)))
    for seed in range(6):
        out = run(blocks=12, resident=12, seed=seed)
        assert out == [want] * 12, (seed, out)


def test_not_all_resident_is_ended_only_by_the_watchdog():
    out = run(blocks=12, resident=8, seed=3, budget=200)
    # the resident blocks can never see the first release; the watchdog ends
    # them, and the blocks that start later find the stall word raised
    assert all(r == -1 for r in out), out
