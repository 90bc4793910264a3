"""GPU score pass (paper Section 2, first phase) against the CPU oracle, bit-exact.

Score and endpoint (lexicographically smallest cell holding the best score)
must equal the oracle's on every case: random and homologous pairs spanning
several stripes and bands with ragged tails, degenerate alphabets and ties,
every tile shape, pruning on and off, band splitting forced small, and few
resident waves (slot reuse).
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


SIZES = [1, 2, 3, 63, 64, 65, 255, 256, 257, 511, 512, 513, 700, 1031]


@pytest.mark.parametrize("rows_per_lane,waves_per_cu", [(4, 0), (8, 0), (8, 12), (4, 16), (6, 12)])
def test_random_shapes(ctx, orc, rows_per_lane, waves_per_cu):
    rng = np.random.default_rng(7 + rows_per_lane + waves_per_cu)
    for t in range(24):
        la, lb = int(rng.choice(SIZES)), int(rng.choice(SIZES))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.15) if t % 2 else \
            synth.random_pair(int(rng.integers(1 << 30)), la, lb)
        a, b = p.a.tobytes(), p.b.tobytes()
        _case(f"random_shapes R={rows_per_lane} waves/CU={waves_per_cu} {la}x{lb} t={t}")
        exp = orc.sw_score(a, b)
        got = ctx.score(a, b, rows_per_lane=rows_per_lane, waves_per_cu=waves_per_cu)
        assert got.key() == exp, (la, lb, t)


@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("rows_per_lane,waves_per_cu", [(4, 0), (8, 0), (8, 10), (6, 8)])
def test_homologous_multi_stripe(ctx, orc, prune, rows_per_lane, waves_per_cu):
    rng = np.random.default_rng(100 + prune + rows_per_lane)
    for la, lb in [(3000, 2900), (2100, 3300), (4100, 700), (900, 5000)]:
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.08)
        a, b = p.a.tobytes(), p.b.tobytes()
        _case(f"homologous R={rows_per_lane} waves/CU={waves_per_cu} prune={prune} {la}x{lb}")
        exp = orc.sw_score(a, b)
        got = ctx.score(a, b, prune=prune, rows_per_lane=rows_per_lane, waves_per_cu=waves_per_cu)
        assert got.key() == exp


@pytest.mark.parametrize("band_width", [64, 128, 320, 1024])
def test_bands_and_slot_reuse(ctx, orc, band_width):
    rng = np.random.default_rng(200 + band_width)
    for la, lb, wpc in [(2000, 1900, 1), (1300, 2500, 2), (700, 3001, 8)]:
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.1)
        a, b = p.a.tobytes(), p.b.tobytes()
        _case(f"bands W={band_width} {la}x{lb} wpc={wpc}")
        exp = orc.sw_score(a, b)
        for prune in (0, 1):
            got = ctx.score(a, b, band_width=band_width, waves_per_cu=wpc, prune=prune, rows_per_lane=4)
            assert got.key() == exp, (la, lb, wpc, prune)


def test_degenerate_and_ties(ctx, orc):
    for m, n in [(1, 1), (5, 300), (300, 5), (700, 700), (1025, 513)]:
        a, b = b"A" * m, b"A" * n
        _case(f"all-A {m}x{n}")
        assert ctx.score(a, b).key() == orc.sw_score(a, b) == (min(m, n), min(m, n) - 1, min(m, n) - 1)
    _case("A-only vs C-only")
    assert ctx.score(b"A" * 900, b"C" * 700).key() == (0, -1, -1)
    rng = np.random.default_rng(3)
    for t in range(6):
        a = synth.random_pair(50 + t, 600, 10, b"AC").a.tobytes()
        b = synth.random_pair(60 + t, 10, 800, b"AC").b.tobytes()
        _case(f"two-letter ties t={t}")
        assert ctx.score(a, b, rows_per_lane=4).key() == orc.sw_score(a, b)
        assert ctx.score(a, b, rows_per_lane=8, prune=1).key() == orc.sw_score(a, b)
    _case("lowercase")
    p = synth.homologous_pair(9, 800, 900, 0.1)
    a, b = p.a.tobytes(), p.b.tobytes()
    assert ctx.score(a.lower(), b).key() == orc.sw_score(a, b)
    _case("repeats")
    a = (b"ACGTTGCA" * 150)[:1111]
    b = (b"ACGTTGCA" * 140)[:1000]
    assert ctx.score(a, b).key() == orc.sw_score(a, b)


def test_empty_and_errors(ctx):
    from paper_1304_5966_amd import swmi
    _case("empty inputs")
    assert ctx.score(b"", b"ACGT").key() == (0, -1, -1)
    assert ctx.score(b"ACGT", b"").key() == (0, -1, -1)
    _case("bad letter")
    with pytest.raises(swmi.SwError) as e:
        ctx.score(b"ACGTN", b"ACGT")
    assert e.value.status == swmi.SW_EINVAL and "offset 4" in str(e.value)
    with pytest.raises(swmi.SwError) as e:
        ctx.score(b"ACGT", b"AC-GT")
    assert e.value.status == swmi.SW_EINVAL and "offset 2" in str(e.value)
    with pytest.raises(swmi.SwError):
        ctx.score(b"ACGT", b"ACGT", scoring=(0, 3, 5, 2))
    with pytest.raises(swmi.SwError):
        ctx.score(b"ACGT", b"ACGT", scoring=(1, 3, 1, 2))
    with pytest.raises(swmi.SwError):
        ctx.score(b"ACGT", b"ACGT", band_width=100)


def test_workspace_limit(orc):
    """A context's device-memory cap: a call beyond it fails with SW_ENOMEM before any device
    work, a raised cap lets it run, and results are unchanged."""
    from paper_1304_5966_amd import swmi
    p = synth.homologous_pair(77, 3000, 2800, 0.1)
    a, b = p.a.tobytes(), p.b.tobytes()
    exp = orc.sw_score(a, b)
    c = swmi.Context(0)
    try:
        _case("workspace limit 64 KiB")
        c.set_max_workspace(64 << 10)
        for call in (lambda: c.score(a, b), lambda: c.align(a, b), lambda: c.batch([(a, b)])):
            with pytest.raises(swmi.SwError) as e:
                call()
            assert e.value.status == swmi.SW_ENOMEM and "limit" in str(e.value)
        _case("workspace limit raised")
        c.set_max_workspace(1 << 30)
        assert c.score(a, b).key() == exp
        assert c.align(a, b).score == exp[0]
        _case("workspace limit lowered below what is held")
        c.set_max_workspace(64 << 10)
        with pytest.raises(swmi.SwError) as e:
            c.score(a, b)
        assert e.value.status == swmi.SW_ENOMEM
        c.set_max_workspace(0)
        assert c.score(a, b).key() == exp
    finally:
        c.close()


def test_other_scorings(ctx, orc):
    """Includes scorings at and beyond the limits of the shifted ticks: match + 2 gap_extend = 127
    for 4 and 8 rows per lane (their score bytes hold s + 2 ext), match + gap_extend = 127 for 6;
    beyond them the pass runs the plain domain."""
    rng = np.random.default_rng(11)
    for sc in [(2, 1, 3, 1), (1, 1, 2, 2), (3, 2, 7, 1), (5, 4, 12, 3), (100, 120, 30, 27), (100, 3, 30, 28),
               (1, 3, 150, 130), (1, 127, 2, 1), (61, 3, 40, 33), (63, 2, 40, 33)]:
        p = synth.homologous_pair(int(rng.integers(1 << 30)), 1200, 1100, 0.2)
        a, b = p.a.tobytes(), p.b.tobytes()
        _case(f"scoring {sc}")
        exp = orc.sw_score(a, b, sc)
        assert ctx.score(a, b, scoring=sc).key() == exp
        assert ctx.score(a, b, scoring=sc, prune=1, rows_per_lane=4).key() == exp
        assert ctx.score(a, b, scoring=sc, rows_per_lane=6).key() == exp
        assert ctx.score(a, b, scoring=sc, rows_per_lane=8).key() == exp


def test_external_threshold_is_exact_when_reached(ctx, orc):
    p = synth.homologous_pair(77, 3000, 2800, 0.1)
    a, b = p.a.tobytes(), p.b.tobytes()
    exp = orc.sw_score(a, b)
    for T in (1, exp[0] // 2, exp[0]):
        _case(f"threshold T={T}")
        got = ctx.score(a, b, prune=2, threshold=T)
        assert got.key() == exp


def test_device_entry_point(ctx, orc):
    import torch
    p = synth.homologous_pair(5, 2500, 2000, 0.1)
    a, b = p.a.tobytes(), p.b.tobytes()
    d_a = torch.frombuffer(bytearray(a), dtype=torch.uint8).cuda()
    d_b = torch.frombuffer(bytearray(b), dtype=torch.uint8).cuda()
    _case("score_dev")
    assert ctx.score_dev(d_a, d_b).key() == orc.sw_score(a, b)


def test_config1_full(ctx, orc):
    p = synth.config1()
    a, b = p.a.tobytes(), p.b.tobytes()
    exp = orc.sw_score(a, b)
    for R in (4, 6, 8):
        for prune in (0, 1):
            _case(f"config1 R={R} prune={prune}")
            assert ctx.score(a, b, rows_per_lane=R, prune=prune).key() == exp
