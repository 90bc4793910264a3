"""Evaluates the learned pruning threshold on the learned-pruning evaluation set.

    python -m paper_1304_5966_amd.eval_learned [--pairs 100] [--chunk 10] [--model PATH] [--out JSON]

Pairs come from the learned-pruning generator with its evaluation seed (never
the training seed), in index order.  Each chunk of pairs runs as one batched
launch per mode -- no pruning, running-best pruning, the learned threshold,
and the threshold set to the true score (the ceiling) -- and every mode must
return the same scores and endpoints.  Reported per mode: seconds, effective
GCUPS (all cells / seconds), the fraction of cells computed, and for the
learned mode the miss rate (pairs whose best fell below the threshold and
were rerun).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import swmi, synth
from .train import DEFAULT_OUT, pairs_to_device

MODES = ("none", "best", "learned", "ceiling")


def evaluate(ctx, model, n_pairs: int, chunk: int, log=print) -> dict:
    torch = ctx._torch
    dev = torch.device(f"cuda:{ctx.device}")
    tot = {m: {"s": 0.0, "computed": 0} for m in MODES}
    cells = misses = used = homologous = 0
    for k0 in range(0, n_pairs, chunk):
        pairs = [synth.config4_pair(i) for i in range(k0, min(n_pairs, k0 + chunk))]
        d_a, oa, d_b, ob = pairs_to_device(torch, pairs, dev)
        ccells = sum(p.cells for p in pairs)
        ref = None
        for mode in MODES:
            if mode == "ceiling":
                # the true scores as thresholds: one call per pair (thresholds differ per pair)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = [ctx.score_dev(d_a[oa[i]:oa[i + 1]], d_b[ob[i]:ob[i + 1]], prune=swmi.PRUNE_LEARNED,
                                     threshold=max(ref[i][0], 1)) for i in range(len(pairs))]
            else:
                kw = {"none": dict(prune=swmi.PRUNE_NONE), "best": dict(prune=swmi.PRUNE_BEST),
                      "learned": dict(prune=swmi.PRUNE_LEARNED, model=model.handle)}[mode]
                ws = ctx.workspace(ctx.batch_workspace_size(oa, ob, **kw))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                res = ctx.batch_dev(d_a, oa, d_b, ob, workspace=ws, **kw)
            dt = time.perf_counter() - t0
            keys = [r.key() for r in res]
            if ref is None:
                ref = keys
            if keys != ref:
                raise RuntimeError(f"mode {mode} disagrees with the unpruned pass on pairs {k0}..")
            tot[mode]["s"] += dt
            tot[mode]["computed"] += sum(r.cells_computed for r in res)
            if mode == "learned":
                misses += sum(r.fallback for r in res)
                used += sum(1 for r in res if r.threshold > 0)
        cells += ccells
        homologous += sum(1 for p in pairs if p.homologous)
        log(f"pairs {k0}..{k0 + len(pairs) - 1} done: " +
            ", ".join(f"{m} {tot[m]['s']:.1f} s" for m in MODES))
    out = {"pairs": n_pairs, "homologous": homologous, "cells": cells,
           "thresholds_set": used, "misses": misses, "miss_rate": misses / max(n_pairs, 1)}
    for m in MODES:
        out[m] = {"s": round(tot[m]["s"], 3), "gcups_eff": round(cells / tot[m]["s"] / 1e9, 1),
                  "cells_computed_frac": round(tot[m]["computed"] / cells, 4)}
    out["speedup_learned_vs_none"] = round(tot["none"]["s"] / tot["learned"]["s"], 3)
    out["speedup_learned_vs_best"] = round(tot["best"]["s"] / tot["learned"]["s"], 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=100)
    ap.add_argument("--chunk", type=int, default=10)
    ap.add_argument("--model", default=DEFAULT_OUT)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()

    def log(m):
        print(m, flush=True)

    ctx = swmi.Context(0)
    model = swmi.Model(ctx, args.model)
    res = evaluate(ctx, model, args.pairs, args.chunk, log=log)
    line = json.dumps(res)
    log(line)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    model.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
