"""GPU start point and reconstruction (paper Section 2, second phase and
Myers-Miller) against the CPU oracle: start coordinates and the canonical
CIGAR must match bit for bit; every CIGAR rescored must give the score."""
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


def _key(al):
    return (al.score, al.start_a, al.start_b, al.end_a, al.end_b, al.cigar)


def test_start_point(ctx, orc):
    rng = np.random.default_rng(21)
    for t in range(16):
        la, lb = int(rng.integers(1, 1500)), int(rng.integers(1, 1500))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.12) if t % 3 else \
            synth.random_pair(int(rng.integers(1 << 30)), la, lb)
        a, b = p.a.tobytes(), p.b.tobytes()
        s, ea, eb = orc.sw_score(a, b)
        _case(f"start {la}x{lb} S={s}")
        if s == 0:
            assert ctx.start(a, b, s, ea, eb) == (-1, -1)
            continue
        assert ctx.start(a, b, s, ea, eb) == orc.sw_start(a, b, s, ea, eb)


def test_start_rejects_wrong_endpoint(ctx, orc):
    from paper_1304_5966_amd import swmi
    p = synth.homologous_pair(3, 600, 600, 0.1)
    a, b = p.a.tobytes(), p.b.tobytes()
    s, ea, eb = orc.sw_score(a, b)
    _case("start with an impossible score")
    with pytest.raises(swmi.SwError):
        ctx.start(a, b, s + 1, ea, eb)


@pytest.mark.parametrize("div", [0.02, 0.1, 0.25])
def test_align_small(ctx, orc, div):
    rng = np.random.default_rng(int(div * 1000))
    for t in range(10):
        la, lb = int(rng.integers(1, 900)), int(rng.integers(1, 900))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, div)
        a, b = p.a.tobytes(), p.b.tobytes()
        _case(f"align {la}x{lb} div={div}")
        got = ctx.align(a, b)
        exp = orc.sw_align(a, b)
        assert _key(got) == (exp.score, exp.start_a, exp.start_b, exp.end_a, exp.end_b, exp.cigar)


@pytest.mark.parametrize("R", [0, 6, 8])
@pytest.mark.parametrize("la,lb,div", [(3000, 2900, 0.05), (5200, 4100, 0.1), (2500, 6000, 0.15)])
def test_align_gpu_levels(ctx, orc, la, lb, div, R):
    """Large enough that the top Myers-Miller levels run on the GPU; R = 0 lets the
    library pick rows per lane from the band width (4 on these narrow bands)."""
    p = synth.homologous_pair(la * 7 + lb, la, lb, div)
    a, b = p.a.tobytes(), p.b.tobytes()
    _case(f"align gpu levels {la}x{lb} R={R}")
    got = ctx.align(a, b, rows_per_lane=R)
    exp = orc.sw_align(a, b)
    assert _key(got) == (exp.score, exp.start_a, exp.start_b, exp.end_a, exp.end_b, exp.cigar)
    assert orc.rescore(a, b, got.start_a, got.start_b, got.cigar) == (got.score, got.end_a, got.end_b)


def test_align_degenerate(ctx, orc):
    _case("align self")
    a = synth.random_pair(5, 4000, 1).a.tobytes()
    al = ctx.align(a, a)
    assert (al.score, al.start_a, al.start_b, al.cigar) == (4000, 0, 0, "4000=")
    _case("align empty / zero")
    assert ctx.align(b"", b"ACGT").cigar == ""
    z = ctx.align(b"AAAA", b"CCCC")
    assert (z.score, z.start_a, z.end_a, z.cigar) == (0, -1, -1, "")
    _case("align other scoring")
    p = synth.homologous_pair(8, 2600, 2400, 0.1)
    a, b = p.a.tobytes(), p.b.tobytes()
    # (100, 120, 140, 30): match + extend > 127, outside the column-shifted domain
    for sc in [(2, 1, 3, 1), (1, 1, 2, 2), (100, 120, 140, 30)]:
        got = ctx.align(a, b, scoring=sc)
        exp = orc.sw_align(a, b, sc)
        assert _key(got) == (exp.score, exp.start_a, exp.start_b, exp.end_a, exp.end_b, exp.cigar)


def test_align_config1(ctx, orc):
    p = synth.config1()
    a, b = p.a.tobytes(), p.b.tobytes()
    _case("align config1")
    got = ctx.align(a, b)
    exp = orc.sw_align(a, b)
    assert _key(got) == (exp.score, exp.start_a, exp.start_b, exp.end_a, exp.end_b, exp.cigar)


_CHAIN_CASES = [(12000, 11000, 0.08, {}), (9000, 15000, 0.12, {}), (14000, 13000, 0.05, dict(band_width=640)),
                (6000, 5800, 0.2, dict(band_width=1280)), (7000, 6500, 0.1, dict(waves_per_cu=1))]
_chain_expected = {}


@pytest.mark.parametrize("chain", ["1", "4", "8"])
def test_align_chain_workgroups(ctx, orc, monkeypatch, chain):
    """The banded global passes (start pass, reconstruction levels) with K waves per
    workgroup on consecutive stripes, linked through LDS (K = 4, 8), and with one wave
    per workgroup (K = 1), against the oracle: long pairs (long chains of stripes),
    narrow column bands (chains cut at band edges, left-boundary hand-offs inside a
    group) and a small grid (slot reuse, few resident groups)."""
    monkeypatch.setenv("SWMI_CHAIN_WAVES", chain)
    for i, (la, lb, div, opts) in enumerate(_CHAIN_CASES):
        p = synth.homologous_pair(900 + i, la, lb, div)
        a, b = p.a.tobytes(), p.b.tobytes()
        if i not in _chain_expected:
            e = orc.sw_align(a, b)
            _chain_expected[i] = (e.score, e.start_a, e.start_b, e.end_a, e.end_b, e.cigar)
        _case(f"chain {chain}: align {la}x{lb} div={div} {opts}")
        got = ctx.align(a, b, rows_per_lane=4, **opts)
        assert _key(got) == _chain_expected[i], (chain, opts)
