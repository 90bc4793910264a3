"""Two-halves score pass (paper Section 2, last paragraphs; SW_FLAG_HALVES) against the oracle.

The upper half of A's rows runs forward and the lower half reversed in one
launch; their last rows are joined at the midline.  Score and endpoint must
equal the oracle's single pass bit for bit, and the reported case must be the
one the oracle's own half scores imply: (b) upper when the upper half alone
reaches S, (c) middle when S exceeds both halves alone (only a crossing path
reaches it), (a) lower or (c) when the lower half alone reaches S.  One pinned
input per case, including a deletion run through the midline, where only the
gap-spanning term of the join reaches S.
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


def _expected_cases(orc, a, b):
    """Cases consistent with the oracle's scores of the whole pair and of each half alone."""
    from paper_1304_5966_amd import swmi
    s = orc.sw_score(a, b)[0]
    mid = len(a) // 2
    s_up = orc.sw_score(a[:mid], b)[0]
    s_low = orc.sw_score(a[mid:], b)[0]
    if s == 0:
        return {swmi.SPLIT_NONE}
    if s_up == s:
        return {swmi.SPLIT_UPPER}
    if s > s_low:
        return {swmi.SPLIT_MIDDLE}
    return {swmi.SPLIT_LOWER, swmi.SPLIT_MIDDLE}


def _check(ctx, orc, a, b, **opts):
    exp = orc.sw_score(a, b)
    got = ctx.score(a, b, halves=True, **opts)
    assert got.key() == exp, (len(a), len(b), opts)
    assert got.split_case in _expected_cases(orc, a, b), got.split_case
    return got


@pytest.mark.parametrize("prune", [0, 1])
@pytest.mark.parametrize("R", [4, 8])
def test_halves_random_and_homologous(ctx, orc, prune, R):
    rng = np.random.default_rng(900 + 2 * R + prune)
    for t in range(10):
        la, lb = int(rng.integers(2, 2600)), int(rng.integers(1, 2300))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.1) if t % 2 else \
            synth.random_pair(int(rng.integers(1 << 30)), la, lb)
        _case(f"halves R={R} prune={prune} {la}x{lb} t={t}")
        _check(ctx, orc, p.a.tobytes(), p.b.tobytes(), prune=prune, rows_per_lane=R)


def _with_piece(seed, la, lb, a_off, core, div=0.05):
    """A random of length la with B holding a mutated copy of A[a_off : a_off + core]."""
    rng = np.random.default_rng(seed)
    a = synth.random_dna(rng, la)
    mut, _ = synth.mutate(rng, a[a_off:a_off + core], div, div / 10)
    left = (lb - mut.size) // 3
    b = np.concatenate([synth.random_dna(rng, left), mut, synth.random_dna(rng, lb - left - mut.size)])
    return a.tobytes(), b.tobytes()


def test_case_upper(ctx, orc):
    from paper_1304_5966_amd import swmi
    a, b = _with_piece(1, 4000, 3000, 300, 1200)
    for prune in (0, 1):
        assert _check(ctx, orc, a, b, prune=prune).split_case == swmi.SPLIT_UPPER


def test_case_lower(ctx, orc):
    from paper_1304_5966_amd import swmi
    a, b = _with_piece(2, 4000, 3000, 2500, 1200)
    for prune in (0, 1):
        assert _check(ctx, orc, a, b, prune=prune).split_case == swmi.SPLIT_LOWER


def test_case_middle(ctx, orc):
    from paper_1304_5966_amd import swmi
    a, b = _with_piece(3, 4000, 3000, 1300, 1500)
    for prune in (0, 1):
        assert _check(ctx, orc, a, b, prune=prune).split_case == swmi.SPLIT_MIDDLE


def test_case_middle_deletion_run_through_the_midline(ctx, orc):
    """A = P D Q, B = P Q with the midline row inside D: the optimum deletes D as one run,
    and only the join's deletion-run term (F up + F down + open - extend) reaches it."""
    from paper_1304_5966_amd import swmi
    rng = np.random.default_rng(4)
    P, D, Q = synth.random_dna(rng, 300), synth.random_dna(rng, 6), synth.random_dna(rng, 300)
    a = np.concatenate([P, D, Q]).tobytes()
    b = np.concatenate([P, Q]).tobytes()
    assert 300 < len(a) // 2 < 306
    s = orc.sw_score(a, b)[0]
    assert s == 600 - (5 + 2 * 5)
    for prune in (0, 1):
        got = _check(ctx, orc, a, b, prune=prune)
        assert got.split_case == swmi.SPLIT_MIDDLE


def test_halves_config1_device_entry_and_errors(ctx, orc):
    import torch
    from paper_1304_5966_amd import swmi
    p = synth.config1()
    a, b = p.a.tobytes(), p.b.tobytes()
    _check(ctx, orc, a, b)
    d_a, d_b = torch.from_numpy(p.a).cuda(), torch.from_numpy(p.b).cuda()
    assert ctx.score_dev(d_a, d_b, halves=True).key() == orc.sw_score(a, b)
    assert ctx.score(b"ACGT", b"", halves=True).key() == (0, -1, -1)
    for bad in (dict(prune=swmi.PRUNE_LEARNED, threshold=5), dict(slab_rows=1000)):
        with pytest.raises(swmi.SwError) as ei:
            ctx.score(a, b, halves=True, **bad)
        assert ei.value.status == swmi.SW_EUNSUPPORTED
    with pytest.raises(swmi.SwError) as ei:
        ctx.score(b"A", b"ACGT", halves=True)
    assert ei.value.status == swmi.SW_EUNSUPPORTED
    with pytest.raises(swmi.SwError) as ei:
        ctx.batch([(a, b)], halves=True)
    assert ei.value.status == swmi.SW_EUNSUPPORTED
