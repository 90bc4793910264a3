"""Substitution-matrix scoring (protein alignment) on the GPU against the CPU oracle, bit-exact.

The engine scores aligned pairs from a per-stripe query profile in LDS instead
of the DNA row tables; every pass that runs on it is compared with the oracle's
matrix scoring: score and endpoint over every tile shape, several stripes and
column bands, pruning on and off, external thresholds, row slabs and the two
halves; start point and canonical CIGAR (host tail and GPU levels); batches,
on the device entry point and through captured graphs.  The matrices are
seeded random ones (symmetric and not) over the 20 amino-acid letters and over
larger alphabets; the paper gives none.  A DNA matrix equal to match/mismatch
must reproduce the DNA path's results exactly.
"""
import numpy as np
import pytest

from paper_1304_5966_amd import synth

pytestmark = pytest.mark.gpu

BIG = b"ARNDCQEGHILKMFPSTWYVBZX*UOJ"  # 27 letters, '*' included
WIDEST = bytes(range(ord("0"), ord("0") + 31))  # 31 letters, the most a matrix may have


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


def _scorings(orc, alphabet, seed, symmetric, gap_open, gap_extend):
    """The same matrix scoring for the oracle and for the library."""
    from paper_1304_5966_amd import swmi
    m = synth.substitution_matrix(seed, len(alphabet), symmetric)
    return orc.MatrixScoring(alphabet, m, gap_open, gap_extend), swmi.MatrixScoring(alphabet, m, gap_open, gap_extend)


SIZES = [1, 2, 63, 64, 65, 257, 511, 512, 513, 1031]


@pytest.mark.parametrize("rows_per_lane,waves_per_cu", [(4, 0), (8, 0), (8, 12), (6, 8), (6, 12), (4, 16)])
def test_protein_random_shapes(ctx, orc, rows_per_lane, waves_per_cu):
    o_sc, g_sc = _scorings(orc, synth.AMINO, 11 + rows_per_lane, True, 11, 1)
    rng = np.random.default_rng(17 + rows_per_lane + waves_per_cu)
    for t in range(16):
        la, lb = int(rng.choice(SIZES)), int(rng.choice(SIZES))
        p = synth.protein_pair(int(rng.integers(1 << 30)), la, lb, 0.3 if t % 2 else 0.95)
        a, b = p.a.tobytes(), p.b.tobytes()
        _case(f"protein shapes R={rows_per_lane} waves/CU={waves_per_cu} {la}x{lb} t={t}")
        exp = orc.sw_score(a, b, o_sc)
        for prune in (0, 1):
            got = ctx.score(a, b, g_sc, prune=prune, rows_per_lane=rows_per_lane, waves_per_cu=waves_per_cu)
            assert got.key() == exp, (la, lb, t, prune)


@pytest.mark.parametrize("alphabet,symmetric,gaps", [(synth.AMINO, False, (10, 1)), (BIG, True, (8, 2)),
                                                     (WIDEST, False, (5, 5)), (b"W", True, (3, 1)),
                                                     (synth.AMINO, True, (127, 120))])
def test_protein_alphabets_and_gaps(ctx, orc, alphabet, symmetric, gaps):
    """Asymmetric matrices, the largest alphabet, one letter, gap costs that leave the
    column-shifted domain (score + extend above 127 runs the plain domain)."""
    o_sc, g_sc = _scorings(orc, alphabet, len(alphabet) + gaps[0], symmetric, *gaps)
    rng = np.random.default_rng(len(alphabet) * 7 + gaps[1])
    for la, lb in [(700, 650), (1500, 40), (64, 2100), (2600, 2500)]:
        p = synth.protein_pair(int(rng.integers(1 << 30)), la, lb, 0.25, alphabet)
        a, b = p.a.tobytes(), p.b.tobytes()
        _case(f"protein alphabet {len(alphabet)} gaps {gaps} {la}x{lb}")
        exp = orc.sw_score(a, b, o_sc)
        assert ctx.score(a, b, g_sc).key() == exp
        assert ctx.score(a, b, g_sc, prune=1, band_width=128).key() == exp
        if la * lb < 2e6:  # the whole alignment, letters outside A-Z included ('*', digits)
            e, g = orc.sw_align(a, b, o_sc), ctx.align(a, b, g_sc)
            assert (g.score, g.start_a, g.start_b, g.end_a, g.end_b, g.cigar) == \
                (e.score, e.start_a, e.start_b, e.end_a, e.end_b, e.cigar)


@pytest.mark.parametrize("rows_per_lane", [4, 8])
def test_protein_bands_thresholds_slabs_halves(ctx, orc, rows_per_lane):
    """Several column bands, external thresholds reached and missed, row slabs, two halves."""
    from paper_1304_5966_amd import swmi
    o_sc, g_sc = _scorings(orc, synth.AMINO, 5, True, 11, 1)
    for seed, la, lb in [(1, 3000, 2800), (2, 2100, 3900), (3, 4500, 900)]:
        p = synth.protein_pair(seed, la, lb, 0.4)
        a, b = p.a.tobytes(), p.b.tobytes()
        exp = orc.sw_score(a, b, o_sc)
        kw = dict(rows_per_lane=rows_per_lane)
        _case(f"protein bands/thresholds R={rows_per_lane} {la}x{lb} score {exp[0]}")
        assert ctx.score(a, b, g_sc, prune=1, band_width=192, **kw).key() == exp
        for T in (exp[0] // 2, exp[0], exp[0] + 1):
            r = ctx.score(a, b, g_sc, prune=swmi.PRUNE_LEARNED, threshold=T, **kw)
            assert r.key() == exp, T
        for h in (1, 333, 1000):
            assert ctx.score(a, b, g_sc, slab_rows=h, **kw).key() == exp, h
        assert ctx.score(a, b, g_sc, halves=True, **kw).key() == exp
        assert ctx.score(a, b, g_sc, halves=True, prune=1, **kw).key() == exp


@pytest.mark.parametrize("seed,la,lb,div", [(1, 300, 280, 0.2), (2, 3000, 2900, 0.3), (3, 2500, 5000, 0.5),
                                            (4, 6000, 5800, 0.15)])
def test_protein_align(ctx, orc, seed, la, lb, div):
    """Start point and canonical CIGAR (GPU Myers-Miller levels from 2048 rows, host tail)."""
    o_sc, g_sc = _scorings(orc, synth.AMINO, 40 + seed, seed % 2 == 0, 10, 1)
    p = synth.protein_pair(seed, la, lb, div)
    a, b = p.a.tobytes(), p.b.tobytes()
    _case(f"protein align {la}x{lb} div {div}")
    exp = orc.sw_align(a, b, o_sc)
    got = ctx.align(a, b, g_sc)
    assert (got.score, got.start_a, got.start_b, got.end_a, got.end_b, got.cigar) == \
        (exp.score, exp.start_a, exp.start_b, exp.end_a, exp.end_b, exp.cigar)
    assert ctx.start(a, b, exp.score, exp.end_a, exp.end_b, g_sc) == (exp.start_a, exp.start_b)
    for R in (4, 6):
        again = ctx.align(a, b, g_sc, rows_per_lane=R)
        assert (again.score, again.start_a, again.cigar) == (exp.score, exp.start_a, exp.cigar), R


def test_protein_batch(ctx, orc):
    """Mixed batch (empty and one-letter sequences included) on both entry points and
    through captured-graph replays, every pair against the oracle."""
    import torch
    from paper_1304_5966_amd import swmi
    o_sc, g_sc = _scorings(orc, synth.AMINO, 77, True, 11, 1)
    rng = np.random.default_rng(78)
    pairs = []
    for t in range(160):
        la = int(rng.choice([0, 1, 20, 64, 65, 150, 400, 1200, 2500]))
        lb = int(rng.choice([0, 1, 33, 64, 129, 300, 900, 2000]))
        p = synth.protein_pair(int(rng.integers(1 << 30)), la, lb, float(rng.choice([0.2, 0.5, 0.95])))
        pairs.append((p.a.tobytes(), p.b.tobytes()))
    _case("protein batch: 160 pairs")
    exp = [orc.sw_score(a, b, o_sc) if a and b else (0, -1, -1) for a, b in pairs]
    res = ctx.batch(pairs, g_sc)
    assert [r.key() for r in res] == exp
    assert [r.key() for r in ctx.batch(pairs, g_sc, prune=1)] == exp
    a_all = np.frombuffer(b"".join(x for x, _ in pairs), np.uint8).copy()
    b_all = np.frombuffer(b"".join(y for _, y in pairs), np.uint8).copy()
    offs_a = np.concatenate(([0], np.cumsum([len(x) for x, _ in pairs]))).astype(np.int64)
    offs_b = np.concatenate(([0], np.cumsum([len(y) for _, y in pairs]))).astype(np.int64)
    d_a, d_b = torch.from_numpy(a_all).cuda(), torch.from_numpy(b_all).cuda()
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        gctx = swmi.Context(0, stream=stream)
        try:
            for rep in range(3):
                _case(f"protein batch graph replay {rep}")
                r = gctx.batch_dev(d_a, offs_a, d_b, offs_b, g_sc, graph=True, prune=1)
                assert [x.key() for x in r] == exp, rep
                torch.cuda.synchronize()
                # other work between replays: the plain device entry point on the same pairs
                r2 = gctx.batch_dev(d_a, offs_a, d_b, offs_b, g_sc)
                assert [x.key() for x in r2] == exp
        finally:
            gctx.close()


def test_protein_matches_dna_path(ctx, orc):
    """match/mismatch over ACGT written as a matrix runs the profile path; its results
    must equal the DNA row-table path's bit for bit (score, ends, start, CIGAR)."""
    from paper_1304_5966_amd import swmi
    m = np.full((4, 4), -3, dtype=np.int8)
    np.fill_diagonal(m, 1)
    g_sc = swmi.MatrixScoring(b"ACGT", m, 5, 2)
    for seed, la, lb in [(5, 4000, 3700), (6, 700, 2500)]:
        p = synth.homologous_pair(seed, la, lb, 0.1)
        a, b = p.a.tobytes(), p.b.tobytes()
        _case(f"DNA as a matrix {la}x{lb}")
        x, y = ctx.align(a, b, g_sc), ctx.align(a, b)
        assert (x.score, x.start_a, x.start_b, x.end_a, x.end_b, x.cigar) == \
            (y.score, y.start_a, y.start_b, y.end_a, y.end_b, y.cigar)
        assert ctx.score(a, b, g_sc, prune=1).key() == ctx.score(a, b, prune=1).key() == orc.sw_score(a, b)


def test_protein_letters_and_errors(ctx, orc):
    from paper_1304_5966_amd import swmi
    o_sc, g_sc = _scorings(orc, synth.AMINO, 3, True, 11, 1)
    p = synth.protein_pair(9, 500, 480, 0.3)
    a, b = p.a.tobytes(), p.b.tobytes()
    _case("protein letters and errors")
    assert ctx.score(a.lower(), b, g_sc).key() == ctx.score(a, b.lower(), g_sc).key() == orc.sw_score(a, b, o_sc)
    bad = bytearray(b)
    bad[123] = ord("B")  # not one of the 20 letters
    with pytest.raises(swmi.SwError) as e:
        ctx.score(a, bytes(bad), g_sc)
    assert e.value.status == swmi.SW_EINVAL and "offset 123" in str(e.value)
    with pytest.raises(swmi.SwError) as e:
        ctx.score(a, b, g_sc, prune=swmi.PRUNE_LEARNED, threshold=0)  # the model path
    assert e.value.status == swmi.SW_EUNSUPPORTED
    with pytest.raises(swmi.SwError) as e:
        ctx.score(a, b, g_sc, both_strands=True)
    assert e.value.status == swmi.SW_EUNSUPPORTED
    m = synth.substitution_matrix(1)
    for alphabet, mat in [(b"ARNA", m[:4, :4]), (b"", m[:0, :0]), (WIDEST + b"~", np.zeros((32, 32), np.int8)),
                          (b"AR", np.array([[1, -128], [0, 1]], np.int8)), (b"A\x01", m[:2, :2])]:
        with pytest.raises(swmi.SwError) as e:
            ctx.score(b"AR", b"AR", swmi.MatrixScoring(alphabet, mat, 11, 1))
        assert e.value.status == swmi.SW_EINVAL, alphabet
    assert ctx.score(b"", b, g_sc).key() == (0, -1, -1)
