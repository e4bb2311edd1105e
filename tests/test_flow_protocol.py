"""CPU model of the batched scheduler's hand-off protocol (flow_kernel,
flow_advance, flow_arm_kernel), run under random interleavings.

Every workgroup is a generator that yields at each access to shared state,
so a random scheduler explores orders of claims, completions and phase
openings among workgroups (sequentially consistent memory).  The model
restates the protocol: per run a word (phase epoch << 32 | items claimed)
for the wheel and breed phases and eight XCD slices for the fitness phase;
a claim is an atomic add whose returned epoch names the phase; the
workgroup that finishes a phase's last item restarts the completion count,
updates the run and opens the next phase (word first, then the fitness
slices) or parks the run; the launch ends when no run is active.  Checked:
the active count never goes below zero, no workgroup waits forever, and
every run evaluates exactly its generations across launches of a few
generations each, with stops by generation count."""
import random

import pytest

PARK = 0xFFFFFFFF
XCDS = 8


class Run:
    def __init__(self, n_pt, n_ranges, n_breed, wheel, max_gen):
        self.n_pt, self.n_ranges, self.n_breed, self.wheel = n_pt, n_ranges, n_breed, wheel
        self.max_gen = max_gen
        self.n_fit = n_pt * n_ranges
        self.generation, self.stopped = 0, 0
        self.word, self.xw, self.done, self.gen, self.left = 0, [0] * XCDS, 0, 0, 0
        self.tile_arrivals, self.tiles_done = [0] * n_pt, 0
        self.evaluated = []


def count(r, e):
    if e == PARK:
        return 0
    return (r.n_fit, 1, r.n_breed)[e % 3]


def word_count(r, e):
    return 0 if e == PARK or e % 3 == 0 else count(r, e)


def slice_lo(r, x):
    return x * r.n_ranges // XCDS


def slice_count(r, e, x):
    if e == PARK or e % 3 != 0:
        return 0
    return (slice_lo(r, x + 1) - slice_lo(r, x)) * r.n_pt


class Shared:
    def __init__(self, runs):
        self.runs, self.active, self.error, self.underflow = runs, 0, 0, False


def workgroup(m, xcd, eval_only, rng, idle_limit=20000):
    idle = 0
    while True:
        choice = None
        for i, r in enumerate(m.runs):           # this XCD's slice or the word
            w = r.word
            yield
            e = w >> 32
            if (w & 0xFFFFFFFF) < word_count(r, e):
                choice = choice or (i, -1)
            elif e != PARK and e % 3 == 0:
                xw = r.xw[xcd]
                yield
                if (xw & 0xFFFFFFFF) < slice_count(r, xw >> 32, xcd):
                    choice = choice or (i, xcd)
        if choice is None:                        # any open slice
            for i, r in enumerate(m.runs):
                for x in range(XCDS):
                    xw = r.xw[x]
                    yield
                    if (xw & 0xFFFFFFFF) < slice_count(r, xw >> 32, x):
                        choice = choice or (i, x)
        claim = None
        if choice is not None:
            i, sl = choice
            r = m.runs[i]
            if sl < 0:
                old = r.word
                r.word = old + 1
                yield
                e, k = old >> 32, old & 0xFFFFFFFF
                if k < word_count(r, e):
                    claim = (i, e, k)
            else:
                old = r.xw[sl]
                r.xw[sl] = old + 1
                yield
                e, k = old >> 32, old & 0xFFFFFFFF
                if k < slice_count(r, e, sl):
                    claim = (i, e, slice_lo(r, sl) * r.n_pt + k)
        if claim is None:
            active = m.active
            yield
            if active == 0 or m.error or m.underflow:
                return
            idle += 1
            if idle > idle_limit:
                m.error = 1
                return
            continue
        idle = 0
        i, e, item = claim
        r = m.runs[i]
        if e % 3 == 0:                            # fitness item and its tail
            pt = item % r.n_pt
            for _ in range(rng.randint(0, 3)):
                yield
            r.tile_arrivals[pt] += 1
            yield
            if r.tile_arrivals[pt] == r.n_ranges:
                r.tile_arrivals[pt] = 0
                r.tiles_done += 1
                yield
                if r.tiles_done == r.n_pt:        # ranking, tracking, stop rule
                    r.tiles_done = 0
                    r.evaluated.append(r.generation)
                    if r.generation + 1 >= r.max_gen:
                        r.stopped = 1
                    yield
        else:
            for _ in range(rng.randint(0, 3)):
                yield
        r.done += 1
        d = r.done
        yield
        if d != count(r, e):
            continue
        r.done = 0                                # advance: restart the count first
        yield
        if e % 3 == 0:
            nxt = PARK if (eval_only or r.stopped) else e + (1 if r.wheel else 2)
        elif e % 3 == 1:
            nxt = e + 1
        else:
            r.generation += 1
            r.gen = r.generation
            r.left -= 1
            yield
            nxt = e + 1 if r.left > 0 else PARK
        r.word = nxt << 32                        # the word names the phase
        yield
        if nxt == PARK:
            m.active -= 1
            if m.active < 0:
                m.underflow = True
            yield
        elif nxt % 3 == 0:                        # then the fitness slices open
            for x in range(XCDS):
                r.xw[x] = nxt << 32
                yield


def launch(m, n_wg, chunk, eval_only, rng):
    active = 0
    for r in m.runs:                              # the arm kernel
        halted = r.stopped
        opened = (PARK << 32) if halted else 0
        r.word, r.xw, r.done, r.gen, r.left = opened, [opened] * XCDS, 0, r.generation, chunk
        active += 0 if halted else 1
    m.active, m.error = active, 0
    live = [workgroup(m, b % XCDS, eval_only, rng) for b in range(n_wg)]
    while live:
        g = rng.choice(live)
        try:
            next(g)
        except StopIteration:
            live.remove(g)
    return not m.error and not m.underflow


@pytest.mark.parametrize("seed", range(300))
def test_protocol_under_random_interleavings(seed):
    rng = random.Random(seed)
    runs = [Run(rng.choice([1, 2]), rng.choice([1, 2, 3, 9]), rng.choice([1, 3, 6]), rng.random() < 0.5,
                rng.choice([5, 9, 13])) for _ in range(rng.randint(1, 3))]
    m = Shared(runs)
    chunk = rng.choice([4, 128])
    n_wg = rng.choice([1, 3, 8, 16])
    if rng.random() < 0.3:                        # an evaluation-only launch first
        assert launch(m, n_wg, 0, True, rng)
        for r in runs:
            r.evaluated.clear()
    for _ in range(20):
        assert launch(m, n_wg, chunk, False, rng), "lost hand-off or double park"
        if all(r.stopped for r in runs):
            break
    for r in runs:
        assert r.evaluated == list(range(r.max_gen))


def test_model_catches_reopened_slices_of_a_stopped_run():
    """The arm step opening a stopped run's slices (the fault this model
    found) makes the active count go below zero."""
    rng = random.Random(0)
    bad = 0
    for seed in range(30):
        rng = random.Random(seed)
        runs = [Run(1, 1, 3, False, 5), Run(2, 3, 3, True, 9)]
        m = Shared(runs)
        for _ in range(10):
            # the faulty arm: slices reset to epoch 0 for every run
            act = 0
            for r in runs:
                halted = r.stopped
                r.word = (PARK << 32) if halted else 0
                r.xw, r.done, r.gen, r.left = [0] * XCDS, 0, r.generation, 4
                act += 0 if halted else 1
            m.active, m.error = act, 0
            live = [workgroup(m, b % XCDS, False, rng) for b in range(8)]
            while live:
                g = rng.choice(live)
                try:
                    next(g)
                except StopIteration:
                    live.remove(g)
            if m.error or m.underflow:
                bad += 1
                break
            if all(r.stopped for r in runs):
                break
    assert bad > 0
