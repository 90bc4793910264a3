"""Both strands (paper Section 3; SW_FLAG_BOTH_STRANDS) against the oracle.

The library aligns A against B and against the reverse complement of B in one
launch and keeps the better strand (the forward one on a tie).  The oracle side
is the plain definition: the oracle run on (A, B) and on (A, rc(B)), with the
reverse complement written out here letter by letter.  Score, strand, endpoint,
start and CIGAR must agree bit for bit; on a genome-scale-shaped pair whose
best copy may lie on either strand, every planted copy bounds its strand's
score from below and the alignment rescores on the reported strand.
"""
import numpy as np
import pytest

from paper_1304_5966_amd import synth

pytestmark = pytest.mark.gpu

_COMP = {ord("A"): ord("T"), ord("C"): ord("G"), ord("G"): ord("C"), ord("T"): ord("A")}


def revcomp(s: bytes) -> bytes:
    return bytes(_COMP[c] for c in reversed(s))


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1304_5966_amd import swmi
    c = swmi.Context(0)
    yield c
    c.close()


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _expected(orc, a, b):
    f = orc.sw_score(a, b)
    r = orc.sw_score(a, revcomp(b))
    return (f, 0) if f[0] >= r[0] else (r, 1)


def test_revcomp_helper():
    assert revcomp(b"AACGT") == b"ACGTT"
    assert revcomp(revcomp(b"GATTACA")) == b"GATTACA"


def test_strands_small_pairs(ctx, orc):
    rng = np.random.default_rng(31)
    for t in range(30):
        la, lb = int(rng.integers(1, 1500)), int(rng.integers(1, 1500))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.1) if t % 3 else \
            synth.random_pair(int(rng.integers(1 << 30)), la, lb)
        a, b = p.a.tobytes(), p.b.tobytes()
        if t % 2:  # the homolog on the reverse strand
            b = revcomp(b)
        (exp, strand) = _expected(orc, a, b)
        for opts in ({}, dict(prune=1), dict(prune=1, slab_rows=300)):
            _case(f"strands {la}x{lb} t={t} {opts}")
            got = ctx.score(a, b, both_strands=True, **opts)
            assert (got.key(), got.strand) == (exp, strand), opts


def test_strands_tie_keeps_forward(ctx, orc):
    # a reverse-complement palindrome aligns equally on both strands
    x = b"ACGTTGCAAGCTTGCA"
    x = x + revcomp(x)
    got = ctx.score(x, x, both_strands=True)
    assert got.strand == 0 and got.key() == orc.sw_score(x, x)


def test_strands_config1_reverse_complemented(ctx, orc):
    p = synth.config1()
    a, b = p.a.tobytes(), revcomp(p.b.tobytes())
    exp = orc.sw_align(a, revcomp(b))
    _case("config1 with B reverse-complemented: score pass and alignment")
    sc = ctx.score(a, b, both_strands=True)
    assert sc.strand == 1 and sc.key() == (exp.score, exp.end_a, exp.end_b)
    al = ctx.align(a, b, both_strands=True)
    assert al.strand == 1
    assert (al.score, al.start_a, al.start_b, al.end_a, al.end_b, al.cigar) == \
        (exp.score, exp.start_a, exp.start_b, exp.end_a, exp.end_b, exp.cigar)
    # forward only: the weak forward-strand optimum
    assert ctx.score(a, b).key() == orc.sw_score(a, b)


def test_strands_genome_shaped_pair(ctx, orc):
    """A 2 Mbp x 1.75 Mbp pair from the genome-scale generator (ten pieces, one reverse-
    complemented): each strand's score is at least every planted copy on it."""
    from paper_1304_5966_amd import swmi
    p = synth.config5(len_a=2_000_000, len_b=1_750_000, n_seg=10)
    a, b = p.a.tobytes(), p.b.tobytes()
    rcb = revcomp(b)
    _case("genome-shaped pair, both strands")
    al = ctx.align(a, b, both_strands=True, prune=swmi.PRUNE_BEST)
    fwd = ctx.score(a, b, prune=swmi.PRUNE_BEST)
    rev = ctx.score(a, rcb, prune=swmi.PRUNE_BEST)
    assert al.score == max(fwd.score, rev.score)
    assert al.strand == (1 if rev.score > fwd.score else 0)
    on = b if al.strand == 0 else rcb
    assert (al.end_a, al.end_b) == ((fwd if al.strand == 0 else rev).end_a, (fwd if al.strand == 0 else rev).end_b)
    assert orc.rescore(a, on, al.start_a, al.start_b, al.cigar) == (al.score, al.end_a, al.end_b)
    assert {pl.strand for pl in p.planted} == {0, 1}
    for pl in p.planted:
        bound = orc.rescore(a, b if pl.strand == 0 else rcb, pl.a_off, pl.b_off, pl.transcript.cigar())[0]
        assert (fwd if pl.strand == 0 else rev).score >= bound


def test_strands_errors(ctx):
    from paper_1304_5966_amd import swmi
    for bad in (dict(prune=swmi.PRUNE_LEARNED, threshold=3), dict(halves=True)):
        with pytest.raises(swmi.SwError) as ei:
            ctx.score(b"ACGT", b"ACGT", both_strands=True, **bad)
        assert ei.value.status == swmi.SW_EUNSUPPORTED
    with pytest.raises(swmi.SwError) as ei:
        ctx.batch([(b"ACGT", b"ACGT")], both_strands=True)
    assert ei.value.status == swmi.SW_EUNSUPPORTED
    with pytest.raises(swmi.SwError) as ei:
        ctx.score(b"ACGT", b"ACNT", both_strands=True)
    assert ei.value.status == swmi.SW_EINVAL
