"""Benchmark: GCUPS of the exact affine-gap Smith-Waterman score pass on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one score pass (letters already resident in HBM -> codes -> forward
wavefront pass -> endpoint reduction -> 16-byte result on the host) over the
5 Mbp x 4 Mbp homologous pair (A: iid ACGT; B: a mutated 3.5 Mbp piece of A,
1 % substitutions, 0.1 % indels of geometric mean length 3, in random
flanks; scoring +1 / -3 / open 5 / extend 2, int32).  Prints one JSON line.

Extra legs (reported in the same line, not in ``value``): the same pass with
block pruning, and the CPU oracle timed on a bounded crop of the same pair.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published figures used for the roofline.
N_CU = 256
CLOCK_HZ = 2.4e9
LANES = 64
VALU_PEAK = N_CU * LANES * CLOCK_HZ  # int32 VALU instruction-lanes per second (3.93e13)
# Algorithmic int32 operations per DP cell in the shortest gfx950 form of the
# recurrence: E: subtract + 3-input max (with the zero floor); open-gap value:
# subtract; F: subtract + max; diagonal: add with byte-selected score;
# H: 3-input max; running maximum: max.
OPS_PER_CELL = 8


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(pair, target_s=12.0):
    """The oracle (single-threaded plain C) on a crop of the same pair around its planted piece."""
    import oracle
    pl = pair.planted[0]
    side = 40_000
    a = pair.a[pl.a_off:pl.a_off + side].tobytes()
    b = pair.b[pl.b_off:pl.b_off + side].tobytes()
    t0 = time.perf_counter()
    oracle.sw_score(a, b)
    dt = time.perf_counter() - t0
    if dt < target_s / 3:
        side2 = int(side * (target_s / max(dt, 1e-3)) ** 0.5)
        a = pair.a[pl.a_off:pl.a_off + side2].tobytes()
        b = pair.b[pl.b_off:pl.b_off + side2].tobytes()
        t0 = time.perf_counter()
        oracle.sw_score(a, b)
        dt = time.perf_counter() - t0
        side = side2
    cells = len(a) * len(b)
    return {"value": cells / dt / 1e9, "unit": "GCUPS", "cores": 1, "kind": "oracle",
            "sample": f"{len(a)} x {len(b)} crop of the same pair starting at its planted piece "
                      f"({cells:.3g} cells, {dt:.1f} s, single-threaded C, 64-bit integers)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rows-per-lane", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the score pass is "
              f"not sharded across GPUs in this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1304_5966_amd import swmi, synth

    log("generating the 5 Mbp x 4 Mbp pair")
    pair = synth.config2()
    M, N = pair.a.size, pair.b.size
    dev = torch.device("cuda:0")
    d_a = torch.from_numpy(pair.a).to(dev)
    d_b = torch.from_numpy(pair.b).to(dev)
    ctx = swmi.Context(0)
    opts = dict(rows_per_lane=args.rows_per_lane, waves_per_cu=args.waves_per_cu)
    ws = ctx.workspace(ctx.workspace_size(M, N, **opts))
    stream = torch.cuda.current_stream(dev)

    results = []
    for i in range(args.warmup):
        log(f"warmup {i}")
        results.append(ctx.score_dev(d_a, d_b, workspace=ws, **opts).key())
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        results.append(ctx.score_dev(d_a, d_b, workspace=ws, **opts).key())
        log(f"step {i} done")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1) / args.steps
    assert len(set(results)) == 1, results
    score = results[-1]
    cells = M * N
    ms = wall * 1000 / args.steps
    gcups = cells / (ms / 1000) / 1e9
    achieved = OPS_PER_CELL * cells / (gpu_ms / 1000)
    line = {
        "metric": "GCUPS of score pass (plain vs batched vs learned-pruned), exact vs oracle",
        "value": round(gcups, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "plain score pass, one homologous DNA pair: A = 5 Mbp iid ACGT, "
                               "B = 4 Mbp holding a mutated 3.5 Mbp piece of A (1 % subst, 0.1 % indels)",
                   "len_a": M, "len_b": N, "scoring": [1, 3, 5, 2], "prune": "none",
                   "score": score[0], "end": [score[1], score[2]]},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 3),
                     "peak": round(VALU_PEAK / 1e12, 3), "unit": "Tops/s int32",
                     "frac": round(achieved / VALU_PEAK, 4), "traffic": None,
                     "ops_per_cell": OPS_PER_CELL, "kernel_ms": round(gpu_ms, 3)},
    }
    if not args.no_extra:
        log("pruned pass")
        r = ctx.score_dev(d_a, d_b, workspace=ws, prune=swmi.PRUNE_BEST, **opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r = ctx.score_dev(d_a, d_b, workspace=ws, prune=swmi.PRUNE_BEST, **opts)
        dt = time.perf_counter() - t1
        assert r.key() == score, (r, score)
        line["pruned_best"] = {"gcups_eff": round(cells / dt / 1e9, 2), "ms": round(dt * 1000, 3),
                               "cells_computed_frac": round(r.cells_computed / cells, 4)}
    if not args.no_cpu:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(pair)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
