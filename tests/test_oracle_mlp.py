"""Pins of the CPU references for the learned threshold (oracle/mlp.py).

The feature extractor is pinned by hand-derivable cases (identical sequences,
a single planted diagonal, bin boundaries) and invariants; the float64
backward pass is pinned by central finite differences.
"""
import numpy as np
import pytest

from oracle import mlp
from paper_1304_5966_amd import synth


def test_log_bins():
    # floor(log2((1+c)^4)): c=0 -> 0, c=1 -> 4, c=2 -> floor(log2 81)=6, c=3 -> 8, c=15 -> 16
    assert [mlp.log_bin(c) for c in (0, 1, 2, 3, 15)] == [0, 4, 6, 8, 16]
    assert mlp.log_bin(10 ** 12) == 125


def test_identical_sequences():
    a = synth.random_pair(1, 2000, 1).a.tobytes()
    x = mlp.features(a, a)
    cnt = mlp.kmer4_classes(mlp.codes(a))
    assert cnt.sum() == len(a) - 3
    np.testing.assert_allclose(x[:128], 128 * cnt / (len(a) - 3))
    # every 12-mer of a hits itself on diagonal 0 (band 2000 // 64 = 31); a random
    # 2 kbp sequence has essentially no other exact 12-mer repeats
    hist = np.round(np.expm1(x[128:254])).astype(int)
    n_bands = (2 * len(a)) // 64 + 2
    assert hist.sum() == n_bands
    assert hist[mlp.log_bin(len(a) - 11)] >= 1
    assert abs(x[254] - np.log(2000) / np.log(4e6)) < 1e-12


def test_unrelated_sequences_have_few_hits():
    p = synth.random_pair(2, 3000, 2500)
    x = mlp.features(p.a.tobytes(), p.b.tobytes())
    hist = np.round(np.expm1(x[128:254])).astype(int)
    assert hist[0] >= hist.sum() - 5   # nearly every band has zero hits


def test_complement_invariance():
    p = synth.homologous_pair(3, 1500, 1400, 0.1)
    a, b = p.a.tobytes(), p.b.tobytes()
    tr = bytes.maketrans(b"ACGT", b"TGCA")
    np.testing.assert_allclose(mlp.features(a, b), mlp.features(a.translate(tr), b.translate(tr)))


@pytest.mark.parametrize("quantile", [0.0, 0.05, 0.7])
def test_finite_differences_validate_backward(quantile):
    rng = np.random.default_rng(0)
    n = 6
    x = rng.normal(size=(n, 256))
    p = rng.normal(scale=0.08, size=mlp.N_PARAMS)
    y, _, _ = mlp.forward_exact(x, p)
    # targets at least 0.5 away from the outputs keep the pinball loss smooth under the probe
    t = y + rng.choice([-1.0, 1.0], size=n) * rng.uniform(0.5, 1.5, size=n)
    g = mlp.backward_exact(x, p, t, quantile)
    idx = np.concatenate([rng.choice(np.arange(mlp.OFF_B1), 12, replace=False),
                          np.arange(mlp.OFF_B1, mlp.OFF_B1 + 3),
                          rng.choice(np.arange(mlp.OFF_W2, mlp.OFF_B2), 12, replace=False),
                          np.arange(mlp.OFF_W3, mlp.OFF_W3 + 4), [mlp.OFF_B3]])
    eps = 1e-3
    for q in idx:
        pp, pm = p.copy(), p.copy()
        pp[q] += eps
        pm[q] -= eps
        fd = (mlp.loss_exact(x, pp, t, quantile) - mlp.loss_exact(x, pm, t, quantile)) / (2 * eps)
        assert abs(fd - g[q]) <= 1e-5 + 1e-3 * abs(g[q]), q


def test_rounded_backward_matches_exact_on_representable_values():
    """With inputs, weights and activations already representable in BF16 the two agree."""
    rng = np.random.default_rng(1)
    n = 5
    x = mlp.bf16(rng.normal(size=(n, 256)))
    p = rng.normal(scale=0.08, size=mlp.N_PARAMS)
    for lo, hi in ((mlp.OFF_W1, mlp.OFF_B1), (mlp.OFF_W2, mlp.OFF_B2), (mlp.OFF_W3, mlp.OFF_B3)):
        p[lo:hi] = mlp.bf16(p[lo:hi])
    t = rng.normal(size=n)
    y, h1, h2 = mlp.forward(x, p)
    g = mlp.backward(x, p, h1, h2, y, t)
    ye, h1e, h2e = mlp.forward_exact(x, p)
    assert np.max(np.abs(y - ye)) < 0.05 * (1 + np.max(np.abs(ye)))
    ge = mlp.backward_exact(x, p, t)
    cos = g @ ge / (np.linalg.norm(g) * np.linalg.norm(ge))
    assert cos > 0.99


def test_pinball_loss_pins():
    """The pinball loss: q * r above the target's side, (1 - q) * |r| below; its minimiser over a
    constant prediction is the q-quantile of the targets."""
    t = np.array([0.0, 1.0, 2.0, 3.0, 10.0])
    assert mlp.loss_value(np.full(5, 2.0), t, 0.25) == pytest.approx(
        np.mean([0.75 * 2, 0.75 * 1, 0.0, 0.25 * 1, 0.25 * 8]))
    grid = np.linspace(-1, 11, 1201)
    best = grid[np.argmin([mlp.loss_value(np.full(5, c), t, 0.2) for c in grid])]
    assert 0.0 <= best <= 1.0  # any point of [t(1), t(2)] minimises at q = 0.2 with five targets
    np.testing.assert_array_equal(mlp.loss_grad(np.array([0.0, 1.0, 2.0]), np.array([1.0, 1.0, 1.0]), 0.3),
                                  np.array([-0.3, 0.0, 0.7]) / 3)
