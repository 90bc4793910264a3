"""Pins the CPU oracle to explicit enumeration of alignments on tiny inputs.

Local alignments (score, endpoint, start point) are enumerated path by path
(``oracle/brute.py``); the canonical Myers-Miller alignment is pinned by
enumerating every optimal global path and applying the midline rule to the
enumeration, recursively.  No dynamic program is involved on the brute-force
side.
"""
import itertools
import random

import pytest

from oracle import brute

SCORINGS = [
    (1, 3, 5, 2),   # the benchmark scoring: match +1, mismatch -3, open 5, extend 2
    (2, 1, 3, 1),
    (1, 1, 2, 2),   # open == extend (linear gaps)
    (3, 2, 7, 1),
]


def _words(alphabet, max_len):
    for L in range(0, max_len + 1):
        for w in itertools.product(alphabet, repeat=L):
            yield bytes(w)


def _check_local(orc, a, b, sc):
    s, sa, sb, ea, eb = brute.local_best(a, b, sc)
    assert orc.sw_score(a, b, sc) == (s, ea, eb)
    assert orc.sw_score(a, b, sc, full=True) == (s, ea, eb)
    al = orc.sw_align(a, b, sc)
    assert (al.score, al.start_a, al.start_b, al.end_a, al.end_b) == (s, sa, sb, ea, eb)
    if s > 0:
        exp = brute.ops_to_cigar(a[sa:ea + 1], b[sb:eb + 1],
                                 brute.canonical_global(a[sa:ea + 1], b[sb:eb + 1], sc,
                                                        sc[2] - sc[3], sc[2] - sc[3]))
        assert al.cigar == exp
        assert orc.rescore(a, b, sa, sb, al.cigar, sc) == (s, ea, eb)
        assert al.cigar[-1] == "=" and al.cigar.split("=")[0].isdigit()
    else:
        assert al.cigar == ""


def test_exhaustive_binary_alphabet(orc):
    words = list(_words(b"AC", 4))
    for a in words:
        for b in words:
            _check_local(orc, a, b, SCORINGS[0])


@pytest.mark.parametrize("sc", SCORINGS)
def test_random_tiny_acgt(orc, sc):
    rng = random.Random(1304 + sum(sc))
    for _ in range(150):
        a = bytes(rng.choice(b"ACGT") for _ in range(rng.randint(0, 6)))
        b = bytes(rng.choice(b"ACGT") for _ in range(rng.randint(0, 6)))
        _check_local(orc, a, b, sc)


def test_lowercase_equals_uppercase(orc):
    rng = random.Random(7)
    for _ in range(50):
        a = bytes(rng.choice(b"ACGT") for _ in range(rng.randint(1, 6)))
        b = bytes(rng.choice(b"ACGT") for _ in range(rng.randint(1, 6)))
        assert orc.sw_score(a.lower(), b, SCORINGS[0]) == orc.sw_score(a, b.lower(), SCORINGS[0])
        assert brute.local_best(a.lower(), b, SCORINGS[0]) == brute.local_best(a, b, SCORINGS[0])


@pytest.mark.parametrize("sc", SCORINGS)
def test_myers_miller_midline_rule(orc, sc):
    """Canonical global alignments with every gap-open convention at the ends."""
    g = sc[2] - sc[3]
    rng = random.Random(99 + sum(sc))
    for _ in range(120):
        A = bytes(rng.choice(b"ACGT") for _ in range(rng.randint(0, 5)))
        B = bytes(rng.choice(b"ACGT") for _ in range(rng.randint(0, 5)))
        tb, te = rng.choice([0, g]), rng.choice([0, g])
        exp = brute.ops_to_cigar(A, B, brute.canonical_global(A, B, sc, tb, te)) if (A or B) else ""
        assert orc.mm_align(A, B, sc, tb, te) == exp if (A or B) else True
        assert orc.global_score(A, B, sc, tb, te) == brute.best_global(A, B, sc, tb, te)


def test_myers_miller_is_optimal_on_larger_inputs(orc):
    """Beyond enumeration sizes the canonical path must still score the global optimum."""
    rng = random.Random(5)
    sc = SCORINGS[0]
    for _ in range(40):
        A = bytes(rng.choice(b"ACGT") for _ in range(rng.randint(1, 60)))
        B = bytes(rng.choice(b"ACGT") for _ in range(rng.randint(1, 60)))
        cig = orc.mm_align(A, B, sc)
        ops = orc.parse_cigar(cig)
        assert sum(n for n, o in ops if o in "=XD") == len(A)
        assert sum(n for n, o in ops if o in "=XI") == len(B)
        # rescoring a global path: leading/trailing gaps open at g + h*k like all others
        s, ea, eb = orc.rescore(A, B, 0, 0, cig, sc)
        assert (ea, eb) == (len(A) - 1, len(B) - 1)
        assert s == orc.global_score(A, B, sc)
