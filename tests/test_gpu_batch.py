"""GPU batch (many pairs in one persistent launch) against the CPU oracle."""
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


def test_batch_mixed(ctx, orc):
    rng = np.random.default_rng(31)
    pairs = []
    for t in range(300):
        la = int(rng.choice([0, 1, 5, 63, 64, 65, 200, 513, 1500, 3000]))
        lb = int(rng.choice([0, 1, 7, 64, 100, 511, 700, 2100]))
        p = synth.homologous_pair(t, la, lb, 0.1) if (t % 2 and la and lb) else synth.random_pair(t, la, lb)
        pairs.append((p.a.tobytes(), p.b.tobytes()))
    for prune in (0, 1):
        for R in (4, 6, 8):
            _case(f"batch mixed prune={prune} R={R}")
            got = ctx.batch(pairs, prune=prune, rows_per_lane=R)
            for (a, b), g in zip(pairs, got):
                assert g.key() == orc.sw_score(a, b), (len(a), len(b))


def test_batch_config3_sample(ctx, orc):
    idx = list(range(0, 400, 1)) + list(range(19_600, 20_000, 7))
    pairs = [synth.config3_pair(i) for i in idx]
    _case(f"batch config3 sample of {len(pairs)}")
    got = ctx.batch([(p.a, p.b) for p in pairs])
    for p, g in zip(pairs, got):
        assert g.key() == orc.sw_score(p.a.tobytes(), p.b.tobytes()), p.tag


def test_batch_device_entry(ctx, orc):
    import torch
    pairs = [synth.config3_pair(i) for i in range(60)]
    a = np.concatenate([p.a for p in pairs])
    b = np.concatenate([p.b for p in pairs])
    oa = np.concatenate(([0], np.cumsum([p.a.size for p in pairs])))
    ob = np.concatenate(([0], np.cumsum([p.b.size for p in pairs])))
    d_a = torch.from_numpy(a).cuda()
    d_b = torch.from_numpy(b).cuda()
    _case("batch_dev")
    got = ctx.batch_dev(d_a, oa, d_b, ob)
    for p, g in zip(pairs, got):
        assert g.key() == orc.sw_score(p.a.tobytes(), p.b.tobytes())


def test_batch_errors(ctx):
    from paper_1304_5966_amd import swmi
    _case("batch bad letter")
    with pytest.raises(swmi.SwError):
        ctx.batch([(b"ACGT", b"ACGT"), (b"ACXT", b"AC")])
    assert ctx.batch([]) == []


def _packed(pairs):
    import torch
    a = np.concatenate([p.a for p in pairs])
    b = np.concatenate([p.b for p in pairs])
    oa = np.concatenate(([0], np.cumsum([p.a.size for p in pairs]))).astype(np.int64)
    ob = np.concatenate(([0], np.cumsum([p.b.size for p in pairs]))).astype(np.int64)
    return torch.from_numpy(a).cuda(), oa, torch.from_numpy(b).cuda(), ob


def test_batch_graph_replay(orc):
    """SW_FLAG_GRAPH: capture once, replay with eager calls in between, new letters in the same buffers."""
    import torch
    from paper_1304_5966_amd import swmi
    stream = torch.cuda.Stream()
    c = swmi.Context(0, stream=stream)
    try:
        first = [synth.config3_pair(i) for i in range(120)]
        d_a, oa, d_b, ob = _packed(first)
        exp = [orc.sw_score(p.a.tobytes(), p.b.tobytes()) for p in first]
        ws = torch.empty(c.batch_workspace_size(oa, ob, graph=True), dtype=torch.uint8, device="cuda")
        other = [synth.config3_pair(1000 + i) for i in range(40)]
        d_ao, oao, d_bo, obo = _packed(other)
        exp_o = [orc.sw_score(p.a.tobytes(), p.b.tobytes()) for p in other]
        torch.cuda.synchronize()
        for rep in range(3):
            _case(f"graph replay {rep}")
            got = c.batch_dev(d_a, oa, d_b, ob, workspace=ws, graph=True)
            assert [g.key() for g in got] == exp
            _case(f"eager between replays {rep}")
            got = c.batch_dev(d_a, oa, d_b, ob, workspace=ws)
            assert [g.key() for g in got] == exp
            # another batch's tables overwrite the workspace: the replay copies its own again
            assert c.batch_dev(d_ao, oao, d_bo, obo, workspace=ws).keys() == exp_o
            torch.cuda.synchronize()
        # Same lengths, different letters, same buffers: the replay must read the new letters.
        second = [synth.homologous_pair(900 + k, p.a.size, p.b.size, 0.15) for k, p in enumerate(first)]
        with torch.cuda.stream(stream):
            d_a.copy_(torch.from_numpy(np.concatenate([p.a for p in second])))
            d_b.copy_(torch.from_numpy(np.concatenate([p.b for p in second])))
        exp2 = [orc.sw_score(p.a.tobytes(), p.b.tobytes()) for p in second]
        for rep in range(2):
            _case(f"graph replay on new letters {rep}")
            got = c.batch_dev(d_a, oa, d_b, ob, workspace=ws, graph=True)
            assert [g.key() for g in got] == exp2
        # A different batch shape re-captures.
        third = first[:50]
        d_a3, oa3, d_b3, ob3 = _packed(third)
        ws3 = torch.empty(c.batch_workspace_size(oa3, ob3, graph=True), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        _case("graph re-capture on a new shape")
        got = c.batch_dev(d_a3, oa3, d_b3, ob3, workspace=ws3, graph=True)
        assert [g.key() for g in got] == exp[:50]
    finally:
        c.close()


def test_batch_graph_needs_stream():
    import torch
    from paper_1304_5966_amd import swmi
    c = swmi.Context(0, stream=torch.cuda.default_stream(0))
    try:
        pairs = [synth.config3_pair(i) for i in range(4)]
        d_a, oa, d_b, ob = _packed(pairs)
        _case("graph on the null stream is refused")
        with pytest.raises(swmi.SwError):
            c.batch_dev(d_a, oa, d_b, ob, graph=True)
    finally:
        c.close()


def test_tuning_is_used(ctx, orc):
    """A tuned shape per class is taken when options leave the shape at 0; results stay exact."""
    from paper_1304_5966_amd import swmi
    pairs = [(p.a.tobytes(), p.b.tobytes()) for p in (synth.config3_pair(i) for i in range(40))]
    exp = [orc.sw_score(a, b) for a, b in pairs]
    assert ctx.get_tuning(swmi.TUNE_BATCH) == (0, 0)
    for R, w in ((4, 12), (8, 2), (0, 0)):
        ctx.set_tuning(swmi.TUNE_BATCH, R, w)
        assert ctx.get_tuning(swmi.TUNE_BATCH) == (R, w)
        _case(f"tuned batch R={R} waves/CU={w}")
        assert [g.key() for g in ctx.batch(pairs)] == exp
    with pytest.raises(swmi.SwError):
        ctx.set_tuning(swmi.TUNE_BATCH, 16, 4)
    with pytest.raises(swmi.SwError):
        ctx.set_tuning(7, 8, 4)
    # a tuned column band width (local passes), narrow enough to cut the pairs into many bands
    for bw in (128, 1024, 0):
        ctx.set_band_width(swmi.TUNE_BATCH, bw)
        assert ctx.get_band_width(swmi.TUNE_BATCH) == bw
        _case(f"tuned batch band width {bw}")
        assert [g.key() for g in ctx.batch(pairs)] == exp
    p = synth.homologous_pair(5, 3000, 2900, 0.1)
    ctx.set_band_width(swmi.TUNE_PAIR_SMALL, 192)
    assert ctx.score(p.a.tobytes(), p.b.tobytes()).key() == orc.sw_score(p.a.tobytes(), p.b.tobytes())
    assert ctx.align(p.a.tobytes(), p.b.tobytes()).cigar == orc.sw_align(p.a.tobytes(), p.b.tobytes()).cigar
    ctx.set_band_width(swmi.TUNE_PAIR_SMALL, 0)
    for bad in (100, -64):
        with pytest.raises(swmi.SwError):
            ctx.set_band_width(swmi.TUNE_BATCH, bad)


def test_batch_slot_reuse_across_problems(ctx, orc, monkeypatch):
    """Regression: a slot is reused only after its previous owner finished writing it.  The last
    stripe of a problem has no reader, so the task after it can finish first; with few slots
    (one wave per CU, no slot room beyond the minimal ring) and many multi-stripe pairs the reuse
    happens constantly."""
    monkeypatch.setenv("SWMI_SLOT_ROOM_BYTES", "0")
    rng = np.random.default_rng(77)
    pairs = []
    for t in range(700):
        la, lb = int(rng.integers(520, 2600)), int(rng.integers(40, 260))
        p = synth.homologous_pair(5000 + t, la, lb, 0.1) if t % 3 == 0 else synth.random_pair(5000 + t, la, lb)
        pairs.append((p.a.tobytes(), p.b.tobytes()))
    exp = [orc.sw_score(a, b) for a, b in pairs]
    for R in (4, 6, 8):
        for rep in range(2):
            _case(f"slot reuse R={R} rep={rep}")
            got = ctx.batch(pairs, rows_per_lane=R, waves_per_cu=1)
            bad = [i for i, (g, e) in enumerate(zip(got, exp)) if g.key() != e]
            assert not bad, (R, rep, bad[:5])


def test_batch_per_pair_thresholds(ctx, orc):
    """PRUNE_LEARNED with one threshold per pair: thresholds at or below the true score are
    reached in one pass; thresholds above it miss and rerun; results are exact either way."""
    from paper_1304_5966_amd import swmi
    rng = np.random.default_rng(8080)
    pairs = []
    for k in range(24):
        la, lb = int(rng.integers(200, 3000)), int(rng.integers(200, 3000))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.1) if k % 2 else \
            synth.random_pair(int(rng.integers(1 << 30)), la, lb)
        pairs.append((p.a.tobytes(), p.b.tobytes()))
    exp = [orc.sw_score(a, b) for a, b in pairs]
    T = [s if k % 3 == 0 else (s // 2 if k % 3 == 1 else s + 5) for k, (s, _, _) in enumerate(exp)]
    res = ctx.batch(pairs, prune=swmi.PRUNE_LEARNED, pair_thresholds=T)
    assert res.keys() == exp
    for k, r in enumerate(res):
        assert r.threshold == T[k]
        assert r.fallback == (1 if T[k] > exp[k][0] else 0), k


def test_autotuner_installs_shape_and_band_width(orc, tmp_path, monkeypatch):
    """The tuner on a pair of 1e10 cells (the LARGE class): it times shapes, then column band
    widths at the chosen shape, installs both in the context, and later calls that leave the
    shape at 0 run with them; results equal the oracle's."""
    import torch
    from paper_1304_5966_amd import autotune, swmi
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    p = synth.homologous_pair(123, 100_000, 100_000, 0.1)
    a, b = p.a.tobytes(), p.b.tobytes()
    exp = orc.sw_score_mt(a, b, threads=orc.host_cores())
    c = swmi.Context(0)
    try:
        d_a, d_b = torch.from_numpy(p.a).cuda(), torch.from_numpy(p.b).cuda()
        table = []
        _case("autotune a 1e10-cell pair: shapes, then band widths")
        best = autotune.tune_score(c, d_a, d_b, use_cache=False, table=table, candidates=[(8, 8), (4, 12)])
        assert "band_width" in best
        assert best["band_width"] in autotune.band_candidates(100_000, 256 * best["waves_per_cu"])
        assert c.get_tuning(swmi.TUNE_PAIR_LARGE) == (best["rows_per_lane"], best["waves_per_cu"])
        assert c.get_band_width(swmi.TUNE_PAIR_LARGE) == best["band_width"]
        assert len(table) == 2 + len(autotune.band_candidates(100_000, 256 * best["waves_per_cu"]))
        assert c.score_dev(d_a, d_b).key() == exp
        assert autotune.cached(c, swmi.TUNE_PAIR_LARGE) == best
    finally:
        c.close()
