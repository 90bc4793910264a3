"""Evaluates the learned pruning threshold on the learned-pruning evaluation set.

    python -m paper_1304_5966_amd.eval_learned [--subset 200] [--part 0/2] [--chunk 10]
                                               [--model PATH] [--out JSON]
    python -m paper_1304_5966_amd.eval_learned --merge part0.json part1.json [--out JSON]

Pairs come from the learned-pruning generator with its evaluation seed (never
the training seed).  ``--subset N`` draws a seeded stratified subset of the
2 000 pairs that keeps the set's mix: round(0.4 N) pairs that carry a
homologous segment and the rest unrelated, each stratum drawn uniformly
without replacement; ``--subset 0`` takes the pairs in index order
(``--pairs``).  ``--part i/k`` evaluates the i-th of k consecutive parts of the
chosen pairs (one GPU command each); ``--merge`` adds the parts' totals.

Each chunk of pairs runs as one batched launch per mode -- no pruning,
running-best pruning, the learned threshold, and the threshold set to each
pair's true score (the ceiling, per-pair thresholds in the same batched
launch) -- and every mode must return the same scores and endpoints.  Reported
per mode: seconds, effective GCUPS (all cells / seconds), the fraction of
cells computed, and for the learned mode the thresholds set and the misses
(pairs whose best fell below the threshold and were rerun).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import swmi, synth
from .train import DEFAULT_OUT, pairs_to_device

MODES = ("none", "best", "learned", "ceiling")
N_EVAL = 2000
SUBSET_SEED = 20240


def stratified_subset(n: int, n_total: int = N_EVAL, seed: int = SUBSET_SEED) -> list:
    """Indices of a stratified subset of the evaluation pairs with the set's homologous share."""
    flags = np.array([synth.config4_meta(i)[2] for i in range(n_total)])
    hom, unrel = np.nonzero(flags)[0], np.nonzero(~flags)[0]
    n_h = int(round(0.4 * n))
    rng = np.random.default_rng(seed)
    pick = np.concatenate([rng.choice(hom, size=min(n_h, hom.size), replace=False),
                           rng.choice(unrel, size=min(n - n_h, unrel.size), replace=False)])
    return sorted(int(i) for i in pick)


def evaluate(ctx, model, indices, chunk: int, log=print) -> dict:
    torch = ctx._torch
    dev = torch.device(f"cuda:{ctx.device}")
    tot = {m: {"s": 0.0, "computed": 0} for m in MODES}
    cells = misses = used = homologous = 0
    for k0 in range(0, len(indices), chunk):
        part = indices[k0:k0 + chunk]
        pairs = [synth.config4_pair(i) for i in part]
        d_a, oa, d_b, ob = pairs_to_device(torch, pairs, dev)
        ref = None
        for mode in MODES:
            kw = {"none": dict(prune=swmi.PRUNE_NONE), "best": dict(prune=swmi.PRUNE_BEST),
                  "learned": dict(prune=swmi.PRUNE_LEARNED, model=model.handle),
                  "ceiling": dict(prune=swmi.PRUNE_LEARNED,
                                  pair_thresholds=[r[0] for r in ref] if ref else None)}[mode]
            ws = ctx.workspace(ctx.batch_workspace_size(oa, ob, **kw))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.batch_dev(d_a, oa, d_b, ob, workspace=ws, **kw)
            dt = time.perf_counter() - t0
            keys = res.keys()
            if ref is None:
                ref = keys
            if keys != ref:
                raise RuntimeError(f"mode {mode} disagrees with the unpruned pass on pairs {part}")
            tot[mode]["s"] += dt
            tot[mode]["computed"] += int(res.array["cells_computed"].sum())
            if mode == "learned":
                misses += int(res.array["fallback"].sum())
                used += int((res.array["threshold"] > 0).sum())
            if mode == "ceiling" and res.array["fallback"].any():
                raise RuntimeError("a threshold equal to the true score missed")
        cells += sum(p.cells for p in pairs)
        homologous += sum(1 for p in pairs if p.homologous)
        log(f"pairs {k0}..{k0 + len(pairs) - 1} of {len(indices)} done: " +
            ", ".join(f"{m} {tot[m]['s']:.1f} s" for m in MODES))
    return {"pairs": len(indices), "indices": list(indices), "homologous": homologous, "cells": cells,
            "thresholds_set": used, "misses": misses,
            "modes": {m: {"s": tot[m]["s"], "computed": tot[m]["computed"]} for m in MODES}}


def summarize(parts: list) -> dict:
    """Totals over parts, with per-mode rates and the comparisons."""
    out = {"pairs": sum(p["pairs"] for p in parts), "homologous": sum(p["homologous"] for p in parts),
           "cells": sum(p["cells"] for p in parts), "thresholds_set": sum(p["thresholds_set"] for p in parts),
           "misses": sum(p["misses"] for p in parts)}
    out["miss_rate"] = round(out["misses"] / max(out["thresholds_set"], 1), 4)
    for m in MODES:
        s = sum(p["modes"][m]["s"] for p in parts)
        c = sum(p["modes"][m]["computed"] for p in parts)
        out[m] = {"s": round(s, 3), "gcups_eff": round(out["cells"] / s / 1e9, 1),
                  "cells_computed_frac": round(c / out["cells"], 4)}
    out["speedup_learned_vs_none"] = round(out["none"]["s"] / out["learned"]["s"], 3)
    out["speedup_learned_vs_best"] = round(out["best"]["s"] / out["learned"]["s"], 3)
    out["speedup_ceiling_vs_best"] = round(out["best"]["s"] / out["ceiling"]["s"], 3)
    out["learned_beats_best"] = out["learned"]["s"] < out["best"]["s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--subset", type=int, default=200, help="stratified subset size (0: index order)")
    ap.add_argument("--pairs", type=int, default=100, help="pairs in index order when --subset 0")
    ap.add_argument("--part", default="0/1", help="i/k: the i-th of k consecutive parts")
    ap.add_argument("--chunk", type=int, default=10)
    ap.add_argument("--model", default=DEFAULT_OUT)
    ap.add_argument("--out", default=None)
    ap.add_argument("--merge", nargs="+", default=None, help="part JSON files to add up")
    args = ap.parse_args()

    def log(m):
        print(m, flush=True)

    if args.merge:
        parts = [json.load(open(p)) for p in args.merge]
        res = summarize(parts)
    else:
        idx = stratified_subset(args.subset) if args.subset else list(range(args.pairs))
        i, k = (int(v) for v in args.part.split("/"))
        lo, hi = len(idx) * i // k, len(idx) * (i + 1) // k
        ctx = swmi.Context(0)
        model = swmi.Model(ctx, args.model)
        res = evaluate(ctx, model, idx[lo:hi], args.chunk, log=log)
        res["summary"] = summarize([res])
        model.close()
    line = json.dumps(res)
    log(line)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
