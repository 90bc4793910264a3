"""Learned threshold on the GPU against the CPU references (oracle/mlp.py).

Features must match the float64 definition; forward and backward of the BF16 /
FP32 network must match the float64 network on the same BF16 inputs and
weights (per-tensor relative Frobenius error <= 1e-2, cosine >= 0.999); the
learned pruning mode must return exactly the plain result, with a counted
fallback whenever the threshold exceeds the best score.
"""
import os

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


def _dev_pairs(pairs):
    import torch
    a = np.concatenate([p.a for p in pairs])
    b = np.concatenate([p.b for p in pairs])
    oa = np.concatenate(([0], np.cumsum([p.a.size for p in pairs]))).astype(np.int64)
    ob = np.concatenate(([0], np.cumsum([p.b.size for p in pairs]))).astype(np.int64)
    return torch.from_numpy(a).cuda(), oa, torch.from_numpy(b).cuda(), ob


def test_features_match_definition(ctx):
    from oracle import mlp
    from paper_1304_5966_amd import swmi
    pairs = [synth.homologous_pair(1, 3000, 2500, 0.05), synth.random_pair(2, 5000, 4000),
             synth.homologous_pair(3, 20_000, 18_000, 0.1), synth.random_pair(4, 3, 100),
             synth.config3_pair(6)]
    d_a, oa, d_b, ob = _dev_pairs(pairs)
    _case("features")
    got = swmi.features_dev(ctx, d_a, oa, d_b, ob).cpu().numpy().astype(np.float64)
    for p, g in zip(pairs, got):
        exp = mlp.features(p.a.tobytes(), p.b.tobytes())
        np.testing.assert_allclose(g, exp, rtol=1e-6, atol=1e-6)


def _rand_model(seed):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    p = np.zeros(mlp.N_PARAMS, dtype=np.float32)
    p[mlp.OFF_W1:mlp.OFF_B1] = rng.normal(scale=0.09, size=mlp.OFF_B1)
    p[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(scale=0.1, size=128)
    p[mlp.OFF_W2:mlp.OFF_B2] = rng.normal(scale=0.12, size=128 * 128)
    p[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(scale=0.1, size=128)
    p[mlp.OFF_W3:mlp.OFF_B3] = rng.normal(scale=0.12, size=128)
    p[mlp.OFF_B3] = 0.3
    return p


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("quantile", [0.0, 0.1])
def test_forward_backward_against_float64(ctx, quantile):
    import torch
    from oracle import mlp
    from paper_1304_5966_amd import swmi, train
    rng = np.random.default_rng(7)
    n = 96
    feats = rng.normal(size=(n, 256)).astype(np.float32)
    params = _rand_model(3)
    tgt = rng.normal(loc=2.0, size=n).astype(np.float32)
    d_feat = torch.from_numpy(feats).cuda()
    mean = np.zeros(256, np.float32)
    inv = np.ones(256, np.float32)
    d_x = swmi.mlp_standardize(ctx, d_feat, torch.from_numpy(mean).cuda(), torch.from_numpy(inv).cuda())
    d_p = torch.from_numpy(params).cuda()
    d_w = torch.from_numpy(train._bf16_bits(params)).cuda()
    _case("mlp forward/backward")
    y, h1, h2 = swmi.mlp_forward(ctx, d_x, d_w, d_p)
    g = swmi.mlp_backward(ctx, d_x, d_w, h1, h2, y, torch.from_numpy(tgt).cuda(), quantile)
    xb = d_x.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    x64 = xb.view(np.float32).astype(np.float64)
    np.testing.assert_array_equal(x64, mlp.bf16(feats))
    ye, h1e, h2e = mlp.forward(x64, params.astype(np.float64))
    assert _rel(y.cpu().numpy(), ye) < 1e-2
    # the pinball loss's sign decisions are taken on the GPU's own outputs (both sides decide alike)
    ysign = y.cpu().numpy().astype(np.float64) if quantile > 0 else ye
    ge = mlp.backward(x64, params.astype(np.float64), h1e, h2e, ysign, tgt.astype(np.float64), quantile)
    gg = g.cpu().numpy().astype(np.float64)
    for lo, hi in ((mlp.OFF_W1, mlp.OFF_B1), (mlp.OFF_B1, mlp.OFF_W2), (mlp.OFF_W2, mlp.OFF_B2),
                   (mlp.OFF_B2, mlp.OFF_W3), (mlp.OFF_W3, mlp.OFF_B3), (mlp.OFF_B3, mlp.N_PARAMS)):
        assert _rel(gg[lo:hi], ge[lo:hi]) < 1e-2, (lo, hi)
    assert gg @ ge / (np.linalg.norm(gg) * np.linalg.norm(ge)) > 0.999


def test_adam_step(ctx):
    import torch
    from paper_1304_5966_amd import swmi, train
    rng = np.random.default_rng(9)
    n = swmi.param_count()
    p = rng.normal(size=n).astype(np.float32)
    m = rng.normal(scale=0.1, size=n).astype(np.float32)
    v = np.abs(rng.normal(scale=0.1, size=n)).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    d_p, d_m, d_v, d_g = (torch.from_numpy(t.copy()).cuda() for t in (p, m, v, g))
    d_w = torch.zeros(n, dtype=torch.int16).cuda()
    _case("adam")
    swmi.mlp_adam(ctx, d_p, d_m, d_v, d_g, 3, 1e-3, d_w)
    b1, b2, eps = 0.9, 0.999, 1e-8
    m2 = b1 * m.astype(np.float64) + (1 - b1) * g
    v2 = b2 * v.astype(np.float64) + (1 - b2) * g.astype(np.float64) ** 2
    p2 = p - 1e-3 * (m2 / (1 - b1 ** 3)) / (np.sqrt(v2 / (1 - b2 ** 3)) + eps)
    np.testing.assert_allclose(d_p.cpu().numpy(), p2, rtol=1e-5, atol=1e-6)
    np.testing.assert_array_equal(d_w.cpu().numpy(), train._bf16_bits(d_p.cpu().numpy()))


def test_learned_mode_is_exact(ctx, orc, tmp_path):
    from paper_1304_5966_amd import swmi, train
    path = str(tmp_path / "m.bin")
    train.save_model(path, np.zeros(256, np.float32), np.full(256, 0.05, np.float32), _rand_model(5))
    model = swmi.Model(ctx, path)
    rng = np.random.default_rng(12)
    fallbacks = 0
    for t in range(10):
        la, lb = int(rng.integers(500, 4000)), int(rng.integers(500, 4000))
        p = synth.homologous_pair(int(rng.integers(1 << 30)), la, lb, 0.1) if t % 2 else \
            synth.random_pair(int(rng.integers(1 << 30)), la, lb)
        a, b = p.a.tobytes(), p.b.tobytes()
        exp = orc.sw_score(a, b)
        _case(f"learned {la}x{lb}")
        got = ctx.score(a, b, prune=swmi.PRUNE_LEARNED, model=model.handle)
        assert got.key() == exp
        fallbacks += got.fallback
        assert got.fallback == (exp[0] < got.threshold)
        for T, fb in ((exp[0], 0), (exp[0] + 1, 1)):
            r = ctx.score(a, b, prune=swmi.PRUNE_LEARNED, threshold=max(T, 1))
            assert r.key() == exp and r.fallback == (1 if exp[0] < max(T, 1) else 0)
    model.close()


def test_learned_batch_graph_replay(orc, tmp_path):
    """SW_FLAG_GRAPH in LEARNED mode: the captured batch is keyed on the predicted thresholds too;
    every replay returns the oracle's results and the eager call's thresholds and fallbacks."""
    import torch
    from paper_1304_5966_amd import swmi, train
    stream = torch.cuda.Stream()
    c = swmi.Context(0, stream=stream)
    try:
        path = str(tmp_path / "m.bin")
        train.save_model(path, np.zeros(256, np.float32), np.full(256, 0.05, np.float32), _rand_model(7))
        model = swmi.Model(c, path)
        pairs = [synth.config3_pair(i) for i in range(60)]
        d_a, oa, d_b, ob = _dev_pairs(pairs)
        exp = [orc.sw_score(p.a.tobytes(), p.b.tobytes()) for p in pairs]
        kw = dict(prune=swmi.PRUNE_LEARNED, model=model.handle)
        ws = torch.empty(c.batch_workspace_size(oa, ob, graph=True, **kw), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        _case("learned batch, eager")
        eager = c.batch_dev(d_a, oa, d_b, ob, workspace=ws, **kw)
        assert eager.keys() == exp
        marks = [(r.threshold, r.fallback) for r in eager]
        for rep in range(3):
            _case(f"learned batch, graph replay {rep}")
            got = c.batch_dev(d_a, oa, d_b, ob, workspace=ws, graph=True, **kw)
            assert got.keys() == exp
            assert [(r.threshold, r.fallback) for r in got] == marks
        model.close()
    finally:
        c.close()


def test_trained_model_on_evaluation_pairs(ctx):
    """The committed network on evaluation-seed pairs (shortened to 0.2-0.4 Mbp): learned pruning
    returns exactly the unpruned results; the cells each mode computes show what it gains."""
    import torch
    from paper_1304_5966_amd import swmi, train
    path = train.DEFAULT_OUT
    if not os.path.exists(path):
        pytest.skip("no trained model in the tree")
    model = swmi.Model(ctx, path)
    pairs = [synth.config4_pair(i, synth.SEED_CONFIG4_EVAL, 200_000, 400_000) for i in range(8)]
    d_a, oa, d_b, ob = _dev_pairs(pairs)
    cells = sum(p.cells for p in pairs)
    got = {}
    for name, kw in (("none", dict(prune=swmi.PRUNE_NONE)), ("best", dict(prune=swmi.PRUNE_BEST)),
                     ("learned", dict(prune=swmi.PRUNE_LEARNED, model=model.handle))):
        _case(f"trained model, mode {name}")
        got[name] = ctx.batch_dev(d_a, oa, d_b, ob, **kw)
    ref = [r.key() for r in got["none"]]
    for name in ("best", "learned"):
        assert [r.key() for r in got[name]] == ref, name
    for r in got["learned"]:
        assert r.fallback == (r.key()[0] < r.threshold)
    frac = {k: sum(r.cells_computed for r in v) / cells for k, v in got.items()}
    print(f"cells computed: {frac}; thresholds {[r.threshold for r in got['learned']]}; "
          f"scores {[k[0] for k in ref]}", flush=True)
    assert frac["none"] == 1.0
    model.close()


def test_trained_model_gain_on_stratified_full_size_pairs(ctx):
    """What the network gains, at full size: ten pairs of the 2 000-pair evaluation set
    (1-4 Mbp per side) drawn with the set's mix (four homologous, six unrelated), every mode
    batched: no pruning, running-best pruning, the learned threshold and the true score as
    threshold (the ceiling).  All modes return the same results; pruning never computes more
    cells than the unpruned pass, the ceiling never more than running-best pruning; the learned
    mode's cells and time against running-best pruning are reported either way (on the
    200-pair stratified evaluation it loses to running-best pruning)."""
    from paper_1304_5966_amd import eval_learned, swmi, train
    if not os.path.exists(train.DEFAULT_OUT):
        pytest.skip("no trained model in the tree")
    model = swmi.Model(ctx, train.DEFAULT_OUT)
    idx = eval_learned.stratified_subset(10, seed=eval_learned.SUBSET_SEED + 2)
    _case(f"trained model on evaluation pairs {idx}")
    part = eval_learned.evaluate(ctx, model, idx, chunk=10, log=lambda m: print(m, flush=True))
    model.close()
    res = eval_learned.summarize([part])
    print({k: res[k] for k in ("none", "best", "learned", "ceiling", "misses", "thresholds_set",
                               "speedup_learned_vs_best", "learned_beats_best")}, flush=True)
    assert part["homologous"] == 4
    assert res["none"]["cells_computed_frac"] == 1.0
    assert res["best"]["cells_computed_frac"] <= 1.0
    assert res["ceiling"]["cells_computed_frac"] <= res["best"]["cells_computed_frac"]
    assert res["learned"]["cells_computed_frac"] <= 2.0  # a miss reruns its pair once
