"""Trains the pruning-threshold network on the GPU with the library's own kernels.

    python -m paper_1304_5966_amd.train [--out PATH] [--n-small 4000] [--n-full 200]
    python -m paper_1304_5966_amd.train --label-only --dump labels.npz ...   # labelling only
    python -m paper_1304_5966_amd.train --data a.npz b.npz                   # train on dumps

Training pairs come from the learned-pruning generator with its training seed
(never the evaluation seed): ``n_small`` pairs of 50-400 kbp per side and
``n_full`` pairs of 1-4 Mbp.  Labels are the exact best scores returned by the
library's batched score pass; features come from ``sw_features_dev``;
forward, backward and Adam run as the library's HIP kernels.  Host code only
shuffles, slices mini-batches and computes the standardisation statistics.
The target is y = ln(1 + S); the loss is mean((y_hat - y)^2), or with --quantile q the
mean pinball loss, whose minimiser is the q-quantile of y given the features (a
conservative prediction keeps T = floor(0.9 * S_hat) below the true score more often).
"""
from __future__ import annotations

import argparse
import json
import os
import struct
import sys
import time

import numpy as np

from . import swmi, synth

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "models", "threshold_mlp.bin")


def _bf16_bits(x: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16).view(np.int16)


def save_model(path: str, mean: np.ndarray, inv_std: np.ndarray, params: np.ndarray) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "wb") as f:
        f.write(b"SWMLP001")
        f.write(struct.pack("<ii", 256, 128))
        f.write(np.asarray(mean, dtype="<f4").tobytes())
        f.write(np.asarray(inv_std, dtype="<f4").tobytes())
        f.write(np.asarray(params, dtype="<f4").tobytes())


def load_model_arrays(path: str):
    with open(path, "rb") as f:
        assert f.read(8) == b"SWMLP001"
        assert struct.unpack("<ii", f.read(8)) == (256, 128)
        mean = np.frombuffer(f.read(1024), dtype="<f4").copy()
        inv = np.frombuffer(f.read(1024), dtype="<f4").copy()
        params = np.frombuffer(f.read(4 * swmi.param_count()), dtype="<f4").copy()
    return mean, inv, params


def pairs_to_device(torch, pairs, device):
    a = np.concatenate([p.a for p in pairs])
    b = np.concatenate([p.b for p in pairs])
    oa = np.concatenate(([0], np.cumsum([p.a.size for p in pairs]))).astype(np.int64)
    ob = np.concatenate(([0], np.cumsum([p.b.size for p in pairs]))).astype(np.int64)
    return torch.from_numpy(a).to(device), oa, torch.from_numpy(b).to(device), ob


def label_and_featurize(ctx, pairs, chunk=64, log=print):
    """Exact scores (batched score pass, running-best pruning) and features of every pair."""
    torch = ctx._torch
    dev = torch.device(f"cuda:{ctx.device}")
    scores, feats = [], []
    for k in range(0, len(pairs), chunk):
        part = pairs[k:k + chunk]
        d_a, oa, d_b, ob = pairs_to_device(torch, part, dev)
        res = ctx.batch_dev(d_a, oa, d_b, ob, prune=swmi.PRUNE_BEST)
        scores += [r.score for r in res]
        feats.append(swmi.features_dev(ctx, d_a, oa, d_b, ob).cpu().numpy())
        log(f"labelled {k + len(part)}/{len(pairs)} pairs")
    return np.asarray(scores, dtype=np.int64), np.concatenate(feats)


def init_params(rng) -> np.ndarray:
    p = np.zeros(swmi.param_count(), dtype=np.float32)
    o = 0
    for fan_in, fan_out in ((256, 128), (128, 128), (128, 1)):
        w = rng.normal(scale=np.sqrt(2.0 / fan_in), size=fan_in * fan_out)
        p[o:o + w.size] = w
        o += w.size + fan_out  # bias stays 0
    return p


def thresholds(y_hat: np.ndarray, feats: np.ndarray) -> np.ndarray:
    """The library's threshold rule on predictions (lengths from the two length features)."""
    la = np.exp(feats[:, 254].astype(np.float64) * np.log(4.0e6))
    lb = np.exp(feats[:, 255].astype(np.float64) * np.log(4.0e6))
    t = np.floor(0.9 * np.expm1(y_hat))
    tmin = 0.01 * la * lb / (la + lb)
    return np.where((t < 1) | (t < tmin), 0, t)


def train(ctx, feats, scores, epochs=300, batch=256, lr=2e-3, quantile=0.0, seed=0, log=print):
    torch = ctx._torch
    dev = torch.device(f"cuda:{ctx.device}")
    y = np.log1p(scores.astype(np.float64)).astype(np.float32)
    mean = feats.mean(0).astype(np.float32)
    # Spread floored at 1: the high histogram bins are populated only by long homologous
    # pairs, and dividing by their tiny spread over all pairs blows those inputs up.
    inv = (1.0 / np.maximum(feats.std(0), 1.0)).astype(np.float32)
    rng = np.random.default_rng(seed)
    n = len(y)
    perm = rng.permutation(n)
    n_val = max(1, n // 10)
    val, tr = perm[:n_val], perm[n_val:]
    d_feat = torch.from_numpy(feats.astype(np.float32)).to(dev)
    d_mean = torch.from_numpy(mean).to(dev)
    d_inv = torch.from_numpy(inv).to(dev)
    x_all = swmi.mlp_standardize(ctx, d_feat, d_mean, d_inv).cpu().numpy()
    params = init_params(rng)
    d_p = torch.from_numpy(params.copy()).to(dev)
    d_w = torch.from_numpy(_bf16_bits(params)).to(dev)
    d_m = torch.zeros_like(d_p)
    d_v = torch.zeros_like(d_p)
    x_val = torch.from_numpy(x_all[val]).to(dev)
    step = 0
    hist = []
    for ep in range(epochs):
        order = rng.permutation(tr)
        for k in range(0, len(order), batch):
            idx = order[k:k + batch]
            d_x = torch.from_numpy(x_all[idx]).to(dev)
            d_t = torch.from_numpy(y[idx]).to(dev)
            yh, h1, h2 = swmi.mlp_forward(ctx, d_x, d_w, d_p)
            g = swmi.mlp_backward(ctx, d_x, d_w, h1, h2, yh, d_t, quantile)
            step += 1
            swmi.mlp_adam(ctx, d_p, d_m, d_v, g, step, lr, d_w)
        if ep % 25 == 0 or ep == epochs - 1:
            yv, _, _ = swmi.mlp_forward(ctx, x_val, d_w, d_p)
            yv = yv.cpu().numpy().astype(np.float64)
            vl = float(np.mean((yv - y[val]) ** 2))
            miss = float(np.mean(thresholds(yv, feats[val]) > scores[val]))
            hist.append((ep, vl, miss))
            log(f"epoch {ep} val mse {vl:.4f} val miss rate {miss:.3f}")
    return mean, inv, d_p.cpu().numpy(), hist


def load_dumps(paths):
    feats, scores = [], []
    for path in paths:
        with np.load(path) as d:
            feats.append(d["feats"])
            scores.append(d["scores"])
    return np.concatenate(feats), np.concatenate(scores)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--n-small", type=int, default=4000)
    ap.add_argument("--small-lo", type=int, default=50_000)
    ap.add_argument("--small-hi", type=int, default=400_000)
    ap.add_argument("--n-full", type=int, default=200)
    ap.add_argument("--full-start", type=int, default=0, help="index of the first full-size pair")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--quantile", type=float, default=0.1,
                    help="0: squared error on ln(1+S); q in (0,1): pinball loss (predicts the q-quantile)")
    ap.add_argument("--dump", default=None, help="write features, scores and lengths of the labelled pairs here")
    ap.add_argument("--label-only", action="store_true", help="label and dump, do not train")
    ap.add_argument("--data", nargs="*", default=None,
                    help="train on these dumps instead of labelling (features and exact scores)")
    args = ap.parse_args()

    def log(m):
        print(m, flush=True)

    ctx = swmi.Context(0)
    t0 = time.time()
    if args.data:
        feats, scores = load_dumps(args.data)
        n_pairs = len(scores)
        log(f"loaded {n_pairs} labelled pairs")
    else:
        pairs = [synth.config4_pair(i, synth.SEED_CONFIG4_TRAIN, args.small_lo, args.small_hi)
                 for i in range(args.n_small)]
        pairs += [synth.config4_pair(1_000_000 + i, synth.SEED_CONFIG4_TRAIN)
                  for i in range(args.full_start, args.full_start + args.n_full)]
        n_pairs = len(pairs)
        log(f"generated {n_pairs} training pairs in {time.time() - t0:.1f} s")
        scores, feats = label_and_featurize(ctx, pairs, log=log)
        log(f"labels and features in {time.time() - t0:.1f} s")
        if args.dump:
            np.savez_compressed(args.dump, feats=feats, scores=scores,
                                len_a=np.array([p.a.size for p in pairs]),
                                len_b=np.array([p.b.size for p in pairs]))
        if args.label_only:
            return 0
    mean, inv, params, hist = train(ctx, feats, scores, epochs=args.epochs, lr=args.lr, quantile=args.quantile,
                                    log=log)
    save_model(args.out, mean, inv, params)
    meta = {"pairs": n_pairs, "epochs": args.epochs, "lr": args.lr, "quantile": args.quantile,
            "val_mse": hist[-1][1], "val_miss_rate": hist[-1][2],
            "seconds": round(time.time() - t0, 1)}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(json.dumps(meta))
    return 0


if __name__ == "__main__":
    sys.exit(main())
