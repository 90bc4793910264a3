"""A host model of the LDS link between the waves of a chain workgroup (the banded
global passes: start pass, reconstruction halves), run over random band
geometries: every stripe must finish, and every column a stripe reads from its
producer's ring must be there (written, not yet overwritten).

The model follows the kernel's rules step by step -- which ticks a stripe runs
(only those whose cells can meet the kept diagonal band), what the producer
publishes at its start (the reader's first column as already read, its own
columns left of its first tick as settled) and after each tick (its column
count), when it waits for ring space (a 256-column ring: the reader must be done
with every column 256 or more behind), and what the reader waits for (the count
covering the columns it reads, none outside the producer's written range) -- and
reports a circular wait as a failure.  It models the protocol, not the kernel's
arithmetic; the GPU tests check the results against the oracle.
"""
import random

import pytest

TICK = 64
RING = 4 * TICK


def band_ticks(d_lo, d_hi, R0, c0, R, n_ticks):
    """Ticks [lo, hi] of a stripe (rows from R0) whose cells can meet the band."""
    a = d_lo - (TICK - 1) + R0 - c0
    b = d_hi + R0 + 64 * R + (TICK - 2) - c0
    lo = 0 if a <= 0 else min((a + TICK - 1) // TICK, n_ticks)
    hi = -1 if b < 0 else min(b // TICK, n_ticks - 1)
    return lo, hi


def task_in_band(d_lo, d_hi, q, R, c0, W, M):
    R0 = q * 64 * R
    R1 = min(R0 + 64 * R, M)
    return not (c0 + W - R0 - 1 < d_lo or c0 + 1 - R1 > d_hi)


def run_chain(S, R, W, c0, d_lo, d_hi, trim_last=True, startup_count=True):
    """True when every stripe of the chain finishes, False on a circular wait;
    asserts on a bad read.  trim_last / startup_count off: the first version of
    the link (the last stripe ran all its ticks; the producer published nothing
    before its first tick)."""
    n_ticks = (W + 2 * TICK - 2) // TICK
    M = S * 64 * R
    act = [task_in_band(d_lo, d_hi, q, R, c0, W, M) for q in range(S)]

    def ticks(q):
        if not trim_last and q == S - 1:
            return 0, n_ticks - 1
        lo, hi = band_ticks(d_lo, d_hi, q * 64 * R, c0, R, n_ticks)
        return (0, n_ticks - 1) if lo > hi else (lo, hi)

    cnt, used = [0] * S, [0] * S
    ring = [dict() for _ in range(S)]  # slot -> column held
    steps = [0]

    def wave(q):
        if not act[q]:
            return
        lo, hi = ticks(q)
        has_prod = q > 0 and act[q - 1]
        has_cons = q + 1 < S and act[q + 1]
        if has_cons:
            clo, chi = ticks(q + 1)
            used[q] = 0 if clo > chi else max(0, TICK * clo - 1)
            if startup_count:
                cnt[q] = max(1, TICK * lo - (TICK - 1))
        pf, pl = 0, 1 << 40
        if has_prod:
            plo, phi = ticks(q - 1)
            pf, pl = max(0, TICK * plo - (TICK - 1)), TICK * phi

        def read(col, need):
            while cnt[q - 1] < need:
                yield
            assert ring[q - 1].get(col % RING) == col, (q, col)

        def fetch(base, need):
            need = min(need, pl + 1)
            cols = [base + l for l in range(TICK) if base + l < W]
            if has_prod:
                for col in cols:
                    if pf <= col <= pl:
                        yield from read(col, need)
                if cols:
                    used[q - 1] = max(used[q - 1], min(base + TICK, W))

        if has_prod:
            rd = TICK * lo - 1
            if lo > 0 and rd < W and pf <= rd <= pl:
                yield from read(rd, rd + 1)
            elif lo == 0:
                while cnt[q - 1] < 1:
                    yield
        yield from fetch(TICK * lo, min(TICK * (lo + 1), W))
        for tau in range(lo, hi + 1):
            if has_cons:
                while used[q] < TICK * tau - RING + 1:
                    yield
                for col in range(TICK * tau - (TICK - 1), TICK * tau + 1):
                    if col >= 0:
                        ring[q][col % RING] = col
                cnt[q] = max(cnt[q], min(TICK * tau + 1, W))
            steps[0] += 1
            if tau + 1 <= hi:
                yield from fetch(TICK * (tau + 1), min(TICK * (tau + 2), W))

    gens = {q: wave(q) for q in range(S)}
    while gens:
        before = (tuple(cnt), tuple(used), steps[0], len(gens))
        for q in list(gens):
            try:
                next(gens[q])
            except StopIteration:
                del gens[q]
        if gens and before == (tuple(cnt), tuple(used), steps[0], len(gens)):
            return False  # a whole round of polls changed nothing: a circular wait
    return True


@pytest.mark.parametrize("seed", range(4))
def test_chain_link_model_random_bands(seed):
    rnd = random.Random(seed)
    for _ in range(150):
        S = rnd.randint(2, 9)
        W = rnd.choice([rnd.randint(1, 3000), 64 * rnd.randint(1, 40)])
        c0 = rnd.choice([0, 0, 640, 1280])
        G = rnd.randint(0, 1500)
        off = rnd.randint(-800, 800)
        assert run_chain(S, 4, W, c0, off - G, off + G), (S, W, c0, off - G, off + G)


def test_chain_link_model_finds_the_old_circular_wait():
    """The model tells a circular wait from progress: the first version of the link
    (last stripe running all its ticks, no start-up count) deadlocks on geometries
    where that stripe starts left of its producer, as it did on the GPU (where the
    bounded waits ended it), and the current rules finish on the same ones."""
    rnd = random.Random(7)
    stuck = 0
    for _ in range(300):
        S = rnd.randint(2, 9)
        W = rnd.choice([rnd.randint(1, 3000), 64 * rnd.randint(1, 40)])
        c0 = rnd.choice([0, 0, 640, 1280])
        G = rnd.randint(0, 1500)
        off = rnd.randint(-800, 800)
        if not run_chain(S, 4, W, c0, off - G, off + G, trim_last=False, startup_count=False):
            stuck += 1
            assert run_chain(S, 4, W, c0, off - G, off + G)
    assert stuck > 0
