"""The reconstruction's host Myers-Miller (libswmi, no GPU) against the oracle.

Runs on the CPU: the library's host code only.  Banded (optimal score given)
and unbanded runs must both give the oracle's canonical CIGAR.
"""
import os

import numpy as np
import pytest

from paper_1304_5966_amd import synth

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1304_5966_amd", "libswmi.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libswmi.so not built")

SCORINGS = [(1, 3, 5, 2), (2, 1, 3, 1), (1, 1, 2, 2)]


@pytest.mark.parametrize("sc", SCORINGS)
def test_host_mm_random(orc, sc):
    from paper_1304_5966_amd import swmi
    rng = np.random.default_rng(sum(sc))
    g = sc[2] - sc[3]
    for t in range(150):
        M, N = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        if M == 0 and N == 0:
            continue
        p = synth.homologous_pair(int(rng.integers(1 << 30)), max(M, 1), max(N, 1), 0.2)
        A, B = p.a.tobytes()[:M], p.b.tobytes()[:N]
        tb, te = int(rng.choice([0, g])), int(rng.choice([0, g]))
        exp = orc.mm_align(A, B, sc, tb, te)
        assert swmi.mm_host(A, B, sc, tb, te) == exp
        s = orc.global_score(A, B, sc, tb, te)
        assert swmi.mm_host(A, B, sc, tb, te, score=s) == exp


def test_host_mm_local_rectangles(orc):
    """The entry call of the reconstruction: the start..end rectangle of a local optimum."""
    from paper_1304_5966_amd import swmi
    rng = np.random.default_rng(5)
    for t in range(30):
        la, lb = int(rng.integers(50, 1500)), int(rng.integers(50, 1500))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, float(rng.uniform(0.02, 0.3)))
        a, b = p.a.tobytes(), p.b.tobytes()
        al = orc.sw_align(a, b)
        if al.score == 0:
            continue
        A, B = a[al.start_a:al.end_a + 1], b[al.start_b:al.end_b + 1]
        assert swmi.mm_host(A, B) == al.cigar
        assert swmi.mm_host(A, B, score=al.score) == al.cigar


@pytest.mark.parametrize("seed,symmetric,gaps", [(1, True, (11, 1)), (2, False, (6, 2)), (3, True, (4, 4))])
def test_host_mm_matrix(orc, seed, symmetric, gaps):
    """Substitution-matrix scoring (protein): the host recursion scores aligned pairs from
    the matrix, in the oracle's canonical form, banded and unbanded."""
    from paper_1304_5966_amd import swmi
    m = synth.substitution_matrix(seed, 20, symmetric)
    o_sc = orc.MatrixScoring(synth.AMINO, m, *gaps)
    g_sc = swmi.MatrixScoring(synth.AMINO, m, *gaps)
    g = gaps[0] - gaps[1]
    rng = np.random.default_rng(seed)
    for t in range(120):
        M, N = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        if M == 0 and N == 0:
            continue
        p = synth.protein_pair(int(rng.integers(1 << 30)), max(M, 1), max(N, 1), 0.4)
        A, B = p.a.tobytes()[:M], p.b.tobytes()[:N]
        if t % 3 == 0:
            A, B = A.lower(), B  # letters are case-insensitive
        tb, te = int(rng.choice([0, g])), int(rng.choice([0, g]))
        exp = orc.mm_align(A, B, o_sc, tb, te)
        assert swmi.mm_host(A, B, g_sc, tb, te) == exp
        s = orc.global_score(A, B, o_sc, tb, te)
        assert swmi.mm_host(A, B, g_sc, tb, te, score=s) == exp
    with pytest.raises(swmi.SwError) as e:
        swmi.mm_host(b"ARNDB", b"ARND", g_sc)  # B is not one of the 20 letters
    assert e.value.status == swmi.SW_EINVAL and "offset 4" in str(e.value)
    with pytest.raises(swmi.SwError) as e:
        swmi.mm_host(b"AR", b"AR", swmi.MatrixScoring(b"ARA", m[:3, :3], 11, 1))  # a letter twice
    assert e.value.status == swmi.SW_EINVAL
