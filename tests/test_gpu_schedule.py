"""The stripe hand-off protocol under perturbed schedules (SWMI_SCHEDULE_JITTER).

With a nonzero seed every wave pauses at pseudo-random points: when it takes a
ticket and before it publishes a tick's column count.  Producers then run late
or early against their consumers, slots are reused at other moments and the
running best grows in another order.  Results depend on none of that (pruning
and the hand-off are exact), so every case must still equal the oracle bit for
bit.  Cases: single pairs over many stripes and bands with few resident waves
(slot reuse), pruning on, row slabs, a mixed batch, and a whole alignment
(reverse pass and reconstruction levels).  Stops at the first mismatch.
"""
import os

import numpy as np
import pytest

from paper_1304_5966_amd import synth

pytestmark = pytest.mark.gpu

SEEDS = [1, 7, 12345]


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1304_5966_amd import swmi
    c = swmi.Context(0)
    yield c
    c.close()


@pytest.fixture
def jitter(request):
    os.environ["SWMI_SCHEDULE_JITTER"] = str(request.param)
    yield request.param
    os.environ.pop("SWMI_SCHEDULE_JITTER", None)


def _case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.mark.parametrize("jitter", SEEDS, indirect=True)
def test_pairs_under_jitter(ctx, orc, jitter):
    rng = np.random.default_rng(jitter)
    for t in range(6):
        la, lb = int(rng.integers(500, 4000)), int(rng.integers(300, 3000))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.1) if t % 2 else \
            synth.random_pair(int(rng.integers(1 << 30)), la, lb)
        a, b = p.a.tobytes(), p.b.tobytes()
        exp = orc.sw_score(a, b)
        for opts in (dict(rows_per_lane=4, waves_per_cu=1, band_width=256), dict(prune=1, band_width=640),
                     dict(rows_per_lane=6, slab_rows=700, prune=1)):
            _case(f"jitter={jitter} {la}x{lb} t={t} {opts}")
            assert ctx.score(a, b, **opts).key() == exp, opts


@pytest.mark.parametrize("jitter", SEEDS[:2], indirect=True)
def test_batch_under_jitter(ctx, orc, jitter):
    rng = np.random.default_rng(100 + jitter)
    pairs = []
    for k in range(40):
        la, lb = int(rng.integers(1, 2500)), int(rng.integers(1, 2500))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.15) if k % 2 else \
            synth.random_pair(int(rng.integers(1 << 30)), la, lb)
        pairs.append((p.a.tobytes(), p.b.tobytes()))
    _case(f"jitter={jitter} batch of {len(pairs)}")
    got = ctx.batch(pairs, rows_per_lane=4, waves_per_cu=2).keys()
    assert got == [orc.sw_score(a, b) for a, b in pairs]


@pytest.mark.parametrize("jitter", SEEDS[:1], indirect=True)
def test_alignment_under_jitter(ctx, orc, jitter):
    p = synth.homologous_pair(2718, 6000, 5200, 0.06)
    a, b = p.a.tobytes(), p.b.tobytes()
    exp = orc.sw_align(a, b)
    _case(f"jitter={jitter} alignment 6000x5200")
    al = ctx.align(a, b, rows_per_lane=4)
    assert (al.score, al.start_a, al.start_b, al.end_a, al.end_b, al.cigar) == \
        (exp.score, exp.start_a, exp.start_b, exp.end_a, exp.end_b, exp.cigar)


def test_wait_limit_abort_path(ctx, orc, monkeypatch):
    """The bounded-wait failure path, forced from the host: with a wait limit of one
    microsecond (and perturbed schedules, so that consumers wait), a wave gives up, raises the
    launch's abort flag, every wait ends, the kernel completes and the call reports an internal
    error instead of hanging.  Without the limit the same context gives exact results again."""
    from paper_1304_5966_amd import swmi
    p = synth.homologous_pair(31, 5000, 4800, 0.1)
    a, b = p.a.tobytes(), p.b.tobytes()
    exp = orc.sw_score(a, b)
    aborted = 0
    for seed in (5, 6, 7):
        monkeypatch.setenv("SWMI_WAIT_LIMIT_US", "1")
        monkeypatch.setenv("SWMI_SCHEDULE_JITTER", str(seed))
        _case(f"wait limit 1 us, jitter seed {seed}")
        try:
            r = ctx.score(a, b)
            assert r.key() == exp  # no wait reached the limit: the result is exact
        except swmi.SwError as e:
            assert e.status == swmi.SW_EINTERNAL and "timed out" in str(e), e
            aborted += 1
        monkeypatch.delenv("SWMI_WAIT_LIMIT_US")
        monkeypatch.delenv("SWMI_SCHEDULE_JITTER")
        _case("default wait limit after the abort")
        assert ctx.score(a, b).key() == exp
        assert ctx.align(a, b).score == exp[0]
    assert aborted > 0


def test_wait_limit_abort_path_chain_workgroups(ctx, orc, monkeypatch):
    """The same failure path in the banded start pass, which runs in chain workgroups
    (waves of a workgroup linked through LDS, with their own bounded waits): under a
    one-microsecond limit and perturbed schedules a launch either gives the exact start
    point or ends with an internal error; the default limit gives the exact result."""
    from paper_1304_5966_amd import swmi
    p = synth.homologous_pair(37, 9000, 8600, 0.08)
    a, b = p.a.tobytes(), p.b.tobytes()
    exp = orc.sw_align(a, b)
    aborted = 0
    for seed in (3, 4, 5):
        monkeypatch.setenv("SWMI_WAIT_LIMIT_US", "1")
        monkeypatch.setenv("SWMI_SCHEDULE_JITTER", str(seed))
        _case(f"start pass, wait limit 1 us, jitter seed {seed}")
        try:
            st = ctx.start(a, b, exp.score, exp.end_a, exp.end_b)
            assert st == (exp.start_a, exp.start_b)
        except swmi.SwError as e:
            assert e.status == swmi.SW_EINTERNAL and "timed out" in str(e), e
            aborted += 1
        monkeypatch.delenv("SWMI_WAIT_LIMIT_US")
        monkeypatch.delenv("SWMI_SCHEDULE_JITTER")
        _case("start pass and alignment at the default limit")
        assert ctx.start(a, b, exp.score, exp.end_a, exp.end_b) == (exp.start_a, exp.start_b)
        al = ctx.align(a, b)
        assert (al.start_a, al.start_b, al.cigar) == (exp.start_a, exp.start_b, exp.cigar)
    assert aborted > 0
