"""Score pass in row slabs (paper Section 2, linear memory) against one launch and the oracle.

A slab is a launch over consecutive rows of A whose row 0 is the previous
slab's last row of H and F.  Results must be bit-identical to the oracle for
every slab height: heights that cut stripes raggedly, slabs thinner than one
stripe, every tile shape, pruning on and off (the bound counts the rows of later
slabs), an external threshold that is reached and one that misses, and ties
between slabs (the earlier slab's cell comes first).
"""
import numpy as np
import pytest

from paper_1304_5966_amd import synth

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("R", [4, 6, 8])
def test_slabs_random_and_homologous(ctx, orc, R):
    from paper_1304_5966_amd import swmi
    rng = np.random.default_rng(500 + R)
    for t in range(6):
        la, lb = int(rng.integers(300, 2600)), int(rng.integers(100, 2300))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.1) if t % 3 else \
            synth.random_pair(int(rng.integers(1 << 30)), la, lb)
        a, b = p.a.tobytes(), p.b.tobytes()
        exp = orc.sw_score(a, b)
        for h in (37, 64 * R, 64 * R + 5, 1000, la // 2 + 1, la - 1):
            for prune in (swmi.PRUNE_NONE, swmi.PRUNE_BEST):
                _case(f"slabs R={R} {la}x{lb} t={t} rows/slab={h} prune={prune}")
                got = ctx.score(a, b, rows_per_lane=R, slab_rows=h, prune=prune)
                assert got.key() == exp, (la, lb, t, h, prune)
                if prune == swmi.PRUNE_NONE:
                    assert got.cells_computed == la * lb


def test_slabs_ties_between_slabs(ctx, orc):
    """A piece repeated in A: both copies align with the same score; the first copy's
    endpoint wins whichever slab boundary separates them."""
    rng = np.random.default_rng(77)
    x = synth.random_dna(rng, 700)
    filler = synth.random_dna(rng, 333)
    a = np.concatenate([x, filler, x, filler]).tobytes()
    b = np.concatenate([synth.random_dna(rng, 150), x, synth.random_dna(rng, 90)]).tobytes()
    exp = orc.sw_score(a, b)
    assert exp[0] == 700 and exp[1] == 699
    for h in (512, 700, 701, 1033, 1100, 1700):
        for prune in (0, 1):
            _case(f"slab ties rows/slab={h} prune={prune}")
            assert ctx.score(a, b, slab_rows=h, prune=prune).key() == exp
    # all-A against all-A: ties on every row from the shorter length on
    for m, n in ((1500, 600), (600, 1500)):
        a, b = b"A" * m, b"A" * n
        exp = orc.sw_score(a, b)
        for h in (100, 599, 600, 601):
            assert ctx.score(a, b, slab_rows=h, prune=1).key() == exp


def test_slabs_external_threshold(ctx, orc):
    """LEARNED mode with a given threshold: reached (exact in one pass) and missed (rerun)."""
    from paper_1304_5966_amd import swmi
    p = synth.homologous_pair(31337, 3000, 2500, 0.08)
    a, b = p.a.tobytes(), p.b.tobytes()
    exp = orc.sw_score(a, b)
    for T, miss in ((exp[0], 0), (exp[0] // 2, 0), (exp[0] + 1, 1), (10 * exp[0], 1)):
        for h in (300, 1111):
            _case(f"slab threshold T={T} rows/slab={h}")
            got = ctx.score(a, b, prune=swmi.PRUNE_LEARNED, threshold=T, slab_rows=h)
            assert got.key() == exp
            assert got.fallback == miss


def test_slabs_progress_and_device_entry(ctx, orc):
    import torch
    p = synth.homologous_pair(4242, 5000, 3000, 0.1)
    exp = orc.sw_score(p.a.tobytes(), p.b.tobytes())
    calls = []
    d_a, d_b = torch.from_numpy(p.a).cuda(), torch.from_numpy(p.b).cuda()
    got = ctx.score_dev(d_a, d_b, slab_rows=1200, progress=lambda done, total: calls.append((done, total)))
    assert got.key() == exp
    assert calls == [(1200, 5000), (2400, 5000), (3600, 5000), (4800, 5000), (5000, 5000)]
    calls.clear()
    assert ctx.score_dev(d_a, d_b, progress=lambda d, t: calls.append((d, t))).key() == exp
    assert calls == [(5000, 5000)]


def test_slabs_config1_and_alignment(ctx, orc):
    p = synth.config1()
    a, b = p.a.tobytes(), p.b.tobytes()
    exp = orc.sw_align(a, b)
    for h in (512, 2500, 4097):
        _case(f"config1 slabs rows/slab={h}")
        assert ctx.score(a, b, slab_rows=h, prune=1).key() == (exp.score, exp.end_a, exp.end_b)
    al = ctx.align(a, b, slab_rows=3000, prune=1)
    assert (al.score, al.start_a, al.start_b, al.end_a, al.end_b, al.cigar) == \
        (exp.score, exp.start_a, exp.start_b, exp.end_a, exp.end_b, exp.cigar)
