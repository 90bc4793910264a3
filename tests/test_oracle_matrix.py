"""Pins of the oracle's substitution-matrix scoring (protein alignment, paper Section 3).

Local alignments are enumerated path by path with the matrix score of each
aligned pair (``oracle/brute.py``) and compared with every oracle mode: full
matrix, linear space, row stripes on threads, the anchored start pass and the
canonical Myers-Miller CIGAR.  A matrix that reproduces match/mismatch over
ACGT must give the tuple scoring's results; relabelling the letters (with the
matrix permuted alike) must change nothing.  The matrices are seeded random
ones over the 20 amino-acid letters; the paper gives no matrix.
"""
import random

import numpy as np
import pytest

import oracle
from oracle import brute

AMINO = b"ARNDCQEGHILKMFPSTWYV"


def random_matrix(seed: int, k: int = 20, symmetric: bool = True) -> np.ndarray:
    rng = np.random.default_rng(seed)
    m = rng.integers(-4, 3, size=(k, k))
    if symmetric:
        m = np.triu(m) + np.triu(m, 1).T
    np.fill_diagonal(m, rng.integers(4, 12, size=k))
    return m.astype(np.int8)


def _check(orc, a, b, sc):
    s, sa, sb, ea, eb = brute.local_best(a, b, sc)
    assert orc.sw_score(a, b, sc) == (s, ea, eb)
    assert orc.sw_score(a, b, sc, full=True) == (s, ea, eb)
    assert orc.sw_score_mt(a, b, sc, threads=3, stripe_rows=2, chunk_cols=3) == (s, ea, eb)
    al = orc.sw_align(a, b, sc)
    assert (al.score, al.start_a, al.start_b, al.end_a, al.end_b) == (s, sa, sb, ea, eb)
    if s > 0:
        g = sc.gap_open - sc.gap_extend
        exp = brute.ops_to_cigar(a[sa:ea + 1], b[sb:eb + 1],
                                 brute.canonical_global(a[sa:ea + 1], b[sb:eb + 1], sc, g, g))
        assert al.cigar == exp
        assert orc.rescore(a, b, sa, sb, al.cigar, sc) == (s, ea, eb)
        assert orc.sw_start_mt(a, b, s, ea, eb, sc, threads=2, stripe_rows=1, chunk_cols=2) == (sa, sb)


@pytest.mark.parametrize("seed,symmetric,gaps", [(1, True, (10, 1)), (2, True, (6, 2)), (3, False, (8, 3)),
                                                 (4, True, (3, 3))])
def test_matrix_scoring_against_enumeration(orc, seed, symmetric, gaps):
    sc = orc.MatrixScoring(AMINO, random_matrix(seed, symmetric=symmetric), *gaps)
    rng = random.Random(seed)
    for _ in range(60):
        letters = AMINO[:rng.choice((3, 6, 20))]
        a = bytes(rng.choice(letters) for _ in range(rng.randint(0, 6)))
        b = bytes(rng.choice(letters) for _ in range(rng.randint(0, 6)))
        _check(orc, a, b, sc)


def test_matrix_case_insensitive_and_bad_letters(orc):
    sc = orc.MatrixScoring(AMINO, random_matrix(5), 10, 1)
    assert orc.sw_score(b"wyvarn", b"WYVARN", sc) == orc.sw_score(b"WYVARN", b"WYVARN", sc)
    with pytest.raises(ValueError):
        orc.sw_score(b"ARNDB", b"ARND", sc)  # B is not one of the 20 letters


def test_dna_matrix_equals_match_mismatch(orc):
    """match/mismatch over ACGT written as a matrix: identical scores, ends, starts and CIGARs."""
    for tup in ((1, 3, 5, 2), (2, 1, 3, 1)):
        m = np.full((4, 4), -tup[1], dtype=np.int8)
        np.fill_diagonal(m, tup[0])
        sc = orc.MatrixScoring(b"ACGT", m, tup[2], tup[3])
        rng = np.random.default_rng(sum(tup))
        for _ in range(40):
            a = rng.choice(np.frombuffer(b"ACGT", np.uint8), int(rng.integers(0, 60))).tobytes()
            b = rng.choice(np.frombuffer(b"ACGT", np.uint8), int(rng.integers(0, 60))).tobytes()
            assert orc.sw_score(a, b, sc) == orc.sw_score(a, b, tup)
            x, y = orc.sw_align(a, b, sc), orc.sw_align(a, b, tup)
            assert (x.score, x.start_a, x.start_b, x.end_a, x.end_b, x.cigar) == \
                (y.score, y.start_a, y.start_b, y.end_a, y.end_b, y.cigar)


def test_relabelling_letters_changes_nothing(orc):
    m = random_matrix(9)
    sc = orc.MatrixScoring(AMINO, m, 8, 2)
    perm = np.random.default_rng(9).permutation(20)
    new_letters = bytes(AMINO[p] for p in perm)  # letter i is renamed new_letters[i]
    trans = bytes.maketrans(AMINO, new_letters)
    sc2 = orc.MatrixScoring(new_letters, m, 8, 2)  # same matrix, indexed by the new names
    rng = np.random.default_rng(10)
    for _ in range(20):
        a = rng.choice(np.frombuffer(AMINO, np.uint8), int(rng.integers(1, 300))).tobytes()
        b = rng.choice(np.frombuffer(AMINO, np.uint8), int(rng.integers(1, 300))).tobytes()
        x, y = orc.sw_align(a, b, sc), orc.sw_align(a.translate(trans), b.translate(trans), sc2)
        assert (x.score, x.start_a, x.start_b, x.end_a, x.end_b, x.cigar) == \
            (y.score, y.start_a, y.start_b, y.end_a, y.end_b, y.cigar)
