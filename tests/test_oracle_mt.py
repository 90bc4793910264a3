"""Pins of the oracle's multi-threaded linear-space mode (oracle/gotoh.c, orc_sw_*_mt).

The threaded mode visits cells in stripe-and-chunk order instead of row-major
order and picks the answer cell by an explicit (row, column) comparison.  It is
pinned by equality with the full-matrix and row-by-row oracles (themselves
pinned by brute-force enumeration) on random shapes whose stripe and chunk
edges fall everywhere, including one-row stripes, one-column chunks, more
threads than stripes and tie-heavy two-letter inputs.  The C10 upper bound of
the pruning rule is checked on the full matrix.
"""
import numpy as np
import pytest

import oracle

SCORINGS = [(1, 3, 5, 2), (2, 1, 3, 1), (1, 1, 1, 1), (3, 2, 7, 3)]


def _rand(rng, n, letters=b"ACGT"):
    return rng.choice(np.frombuffer(letters, dtype=np.uint8), n).tobytes()


@pytest.mark.parametrize("sc", SCORINGS)
def test_mt_equals_single_threaded(sc):
    rng = np.random.default_rng(sum(sc))
    for _ in range(60):
        m, n = int(rng.integers(0, 70)), int(rng.integers(0, 70))
        letters = b"AC" if rng.random() < 0.4 else b"ACGT"
        a, b = _rand(rng, m, letters), _rand(rng, n, letters)
        ref = oracle.sw_score(a, b, sc, full=True)
        assert oracle.sw_score(a, b, sc) == ref
        for th, h, c in [(1, 1, 1), (3, 2, 3), (4, 5, 7), (2, 7, 64), (8, 1, 2), (5, 64, 5)]:
            assert oracle.sw_score_mt(a, b, sc, threads=th, stripe_rows=h, chunk_cols=c) == ref, (m, n, th, h, c)
            if ref[0] > 0:
                assert oracle.sw_start_mt(a, b, *ref, scoring=sc, threads=th, stripe_rows=h,
                                          chunk_cols=c) == oracle.sw_start(a, b, *ref, scoring=sc)


def test_mt_homologous_default_shape():
    """A pair with one long optimum: the default stripe (512 rows) and chunk (16 384 columns)."""
    from paper_1304_5966_amd import synth
    p = synth.homologous_pair(77, 3000, 2600, 0.08)
    a, b = p.a.tobytes(), p.b.tobytes()
    ref = oracle.sw_score(a, b)
    for th in (1, 2, 7):
        got = oracle.sw_score_mt(a, b, threads=th)
        assert got == ref
        assert oracle.sw_start_mt(a, b, *got, threads=th) == oracle.sw_start(a, b, *ref)


def test_mt_ties_pick_first_cell():
    """All-A against all-A: S = min length, reached first on the last row/column of the shorter side."""
    for m, n in ((40, 25), (25, 40), (33, 33)):
        a, b = b"A" * m, b"A" * n
        s, ea, eb = oracle.sw_score_mt(a, b, threads=3, stripe_rows=4, chunk_cols=6)
        assert s == min(m, n)
        if m >= n:
            assert (ea, eb) == (n - 1, n - 1)
        else:
            assert (ea, eb) == (m - 1, m - 1)
        assert oracle.sw_start_mt(a, b, s, ea, eb, threads=3, stripe_rows=4, chunk_cols=6) == (0, 0)


def test_mt_errors():
    with pytest.raises(ValueError):
        oracle.sw_start_mt(b"ACGT", b"TTTT", 3, 3, 3, threads=2)   # no alignment of score 3 ends there
    assert oracle.sw_score_mt(b"", b"ACGT", threads=2) == (0, -1, -1)


@pytest.mark.parametrize("tile", [(4, 4), (8, 3), (5, 11)])
def test_pruning_upper_bound_holds_on_every_tile(tile):
    """C10: the largest H inside a tile is at most max(0, H on its input borders) plus match
    times the shorter of the rows and columns left from the tile's corner."""
    rng = np.random.default_rng(tile[0] * 31 + tile[1])
    tr, tc = tile
    for k in range(8):
        sc = SCORINGS[k % len(SCORINGS)]
        m, n = int(rng.integers(20, 60)), int(rng.integers(20, 60))
        if k % 2:
            from paper_1304_5966_amd import synth
            p = synth.homologous_pair(1000 + k, m, n, 0.1)
            a, b = p.a.tobytes(), p.b.tobytes()
        else:
            a, b = _rand(rng, m), _rand(rng, n)
        H = oracle.sw_matrix(a, b, sc)
        for r0 in range(1, m + 1, tr):
            for c0 in range(1, n + 1, tc):
                r1, c1 = min(r0 + tr, m + 1), min(c0 + tc, n + 1)
                border = max(H[r0 - 1, c0 - 1:c1].max(), H[r0:r1, c0 - 1].max(), 0)
                ub = border + sc[0] * min(m - r0 + 1, n - c0 + 1)
                assert H[r0:r1, c0:c1].max() <= ub
