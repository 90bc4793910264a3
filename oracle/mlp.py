"""CPU references for the learned pruning threshold -- TEST INFRASTRUCTURE ONLY.

Not part of the paper: the threshold model of the benchmark's learned-pruning
configuration.  Written from the feature and network definitions (see
include/swmi.h), independently of the GPU kernels:

* ``features(a, b)``: the 256 pair features, counted the plain way in numpy
  (4-mer classes by sliding windows, 12-mer hits by a dictionary of A's
  positions, diagonal bands, integer log bins).
* ``forward`` / ``backward``: the 256-128-128-1 ReLU network in float64 on
  BF16-rounded inputs, weights and hidden activations (rounding by torch's CPU
  bfloat16 conversion); mean-squared error on y, or with ``quantile`` q in
  (0, 1) the mean pinball loss max(q r, (q - 1) r), r = t - y.
* ``forward_exact`` / ``loss_exact``: the same network without activation
  rounding, for central finite differences that check ``backward`` itself.
"""
from __future__ import annotations

import math

import numpy as np

F, H = 256, 128
OFF_W1 = 0
OFF_B1 = OFF_W1 + F * H
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
N_PARAMS = OFF_B3 + 1
BINS = 126
CAP = 64

_LUT = np.full(256, 255, dtype=np.uint8)
for _i, _c in enumerate(b"ACGT"):
    _LUT[_c] = _i
    _LUT[_c + 32] = _i


def codes(seq) -> np.ndarray:
    s = np.frombuffer(seq if isinstance(seq, bytes) else np.asarray(seq, np.uint8).tobytes(), dtype=np.uint8)
    c = _LUT[s]
    assert (c < 4).all()
    return c.astype(np.int64)


def kmer4_classes(c: np.ndarray) -> np.ndarray:
    if c.size < 4:
        return np.zeros(128, dtype=np.int64)
    k = (c[:-3] << 6) | (c[1:-2] << 4) | (c[2:-1] << 2) | c[3:]
    q = np.where(k < 128, k, k ^ 0xFF)
    return np.bincount(q, minlength=128)


def kmer12(c: np.ndarray) -> np.ndarray:
    if c.size < 12:
        return np.zeros(0, dtype=np.int64)
    v = np.zeros(c.size - 11, dtype=np.int64)
    for k in range(12):
        v = (v << 2) | c[k:c.size - 11 + k]
    return v


def log_bin(count: int) -> int:
    """floor(log2((1 + count)^4)) capped at 125, in exact integer arithmetic."""
    x4 = (1 + int(count)) ** 4
    return min(BINS - 1, x4.bit_length() - 1)


def features(a, b) -> np.ndarray:
    ca, cb = codes(a), codes(b)
    na, nb = ca.size, cb.size
    x = np.zeros(F, dtype=np.float64)
    fa = kmer4_classes(ca) / (na - 3) if na >= 4 else np.zeros(128)
    fb = kmer4_classes(cb) / (nb - 3) if nb >= 4 else np.zeros(128)
    x[:128] = 128.0 * np.minimum(fa, fb)
    ka, kb = kmer12(ca), kmer12(cb)
    pos = {}
    for i, k in enumerate(ka.tolist()):
        pos.setdefault(k, []).append(i)
    nbands = (na + nb) // 64 + 2
    band = np.zeros(nbands, dtype=np.int64)
    for j, k in enumerate(kb.tolist()):
        ps = pos.get(k)
        if ps is None or len(ps) > CAP:
            continue
        for i in ps:
            band[(j - i + na) // 64] += 1
    hist = np.zeros(BINS, dtype=np.int64)
    for cnt in band.tolist():
        hist[log_bin(cnt)] += 1
    x[128:128 + BINS] = np.log1p(hist)
    x[254] = math.log(max(na, 1)) / math.log(4.0e6)
    x[255] = math.log(max(nb, 1)) / math.log(4.0e6)
    return x


def bf16(x) -> np.ndarray:
    """Round to nearest even bfloat16, returned as float64 (torch's CPU conversion)."""
    import torch
    t = torch.as_tensor(np.asarray(x, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def unpack(params: np.ndarray):
    p = np.asarray(params, dtype=np.float64)
    W1 = p[OFF_W1:OFF_B1].reshape(F, H)
    b1 = p[OFF_B1:OFF_W2]
    W2 = p[OFF_W2:OFF_B2].reshape(H, H)
    b2 = p[OFF_B2:OFF_W3]
    W3 = p[OFF_W3:OFF_B3]
    b3 = p[OFF_B3]
    return W1, b1, W2, b2, W3, b3


def forward(x_bf16: np.ndarray, params: np.ndarray):
    """x_bf16 [n, 256] already rounded; weights rounded here; biases exact.  Returns (y, h1, h2)."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    W1, W2, W3 = bf16(W1), bf16(W2), bf16(W3)
    h1 = bf16(np.maximum(x_bf16 @ W1 + b1, 0.0))
    h2 = bf16(np.maximum(h1 @ W2 + b2, 0.0))
    y = h2 @ W3 + b3
    return y, h1, h2


def loss_grad(y: np.ndarray, t: np.ndarray, quantile: float = 0.0) -> np.ndarray:
    """d loss / d y per sample, loss averaged over the samples."""
    n = y.shape[0]
    if quantile <= 0:
        return 2.0 * (y - t) / n
    return np.where(y > t, 1.0 - quantile, np.where(y < t, -quantile, 0.0)) / n


def loss_value(y: np.ndarray, t: np.ndarray, quantile: float = 0.0) -> float:
    if quantile <= 0:
        return float(np.mean((y - t) ** 2))
    r = t - y
    return float(np.mean(np.maximum(quantile * r, (quantile - 1.0) * r)))


def backward(x_bf16: np.ndarray, params: np.ndarray, h1: np.ndarray, h2: np.ndarray, y: np.ndarray,
             t: np.ndarray, quantile: float = 0.0) -> np.ndarray:
    """Gradient of the loss (see loss_grad) with respect to the parameters, float64."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    W2, W3 = bf16(W2), bf16(W3)
    dy = loss_grad(y, t, quantile)
    d2 = np.outer(dy, W3) * (h2 > 0)
    d1 = (d2 @ W2.T) * (h1 > 0)
    g = np.zeros(N_PARAMS)
    g[OFF_W1:OFF_B1] = (x_bf16.T @ d1).ravel()
    g[OFF_B1:OFF_W2] = d1.sum(0)
    g[OFF_W2:OFF_B2] = (h1.T @ d2).ravel()
    g[OFF_B2:OFF_W3] = d2.sum(0)
    g[OFF_W3:OFF_B3] = h2.T @ dy
    g[OFF_B3] = dy.sum()
    return g


def forward_exact(x: np.ndarray, params: np.ndarray):
    W1, b1, W2, b2, W3, b3 = unpack(params)
    h1 = np.maximum(x @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h2 @ W3 + b3, h1, h2


def backward_exact(x, params, t, quantile: float = 0.0):
    W1, b1, W2, b2, W3, b3 = unpack(params)
    y, h1, h2 = forward_exact(x, params)
    dy = loss_grad(y, t, quantile)
    d2 = np.outer(dy, W3) * (h2 > 0)
    d1 = (d2 @ W2.T) * (h1 > 0)
    g = np.zeros(N_PARAMS)
    g[OFF_W1:OFF_B1] = (x.T @ d1).ravel()
    g[OFF_B1:OFF_W2] = d1.sum(0)
    g[OFF_W2:OFF_B2] = (h1.T @ d2).ravel()
    g[OFF_B2:OFF_W3] = d2.sum(0)
    g[OFF_W3:OFF_B3] = h2.T @ dy
    g[OFF_B3] = dy.sum()
    return g


def loss_exact(x, params, t, quantile: float = 0.0) -> float:
    y, _, _ = forward_exact(x, params)
    return loss_value(y, t, quantile)
