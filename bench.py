"""Benchmark: GCUPS of the exact affine-gap Smith-Waterman score pass on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one score pass (letters already resident in HBM -> codes -> forward
wavefront pass -> endpoint reduction -> 16-byte result on the host) over the
5 Mbp x 4 Mbp homologous pair (A: iid ACGT; B: a mutated 3.5 Mbp piece of A,
1 % substitutions, 0.1 % indels of geometric mean length 3, in random
flanks; scoring +1 / -3 / open 5 / extend 2, int32).  Prints one JSON line.

Extra legs (reported in the same line, not in ``value``): the same pass with
block pruning; the whole alignment of the pair (score pass, start pass,
Myers-Miller reconstruction) timed by phase; the 20 000-pair batch; the
learned threshold; substitution-matrix (protein) scoring; and the CPU oracle
timed on a bounded crop of the same pair.
``--only batched|learned|align|genome|protein`` runs one leg alone and prints its JSON
(for profiling a leg by itself).  The genome leg is the score pass of the
32 Mbp x 28 Mbp genome-scale pair with running-best pruning, in row slabs.
``--time-budget S`` (default 540 s) bounds the whole run: an extra leg whose
usual duration no longer fits is skipped and named as skipped in the line.
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
# Algorithmic int32 operations per DP cell, counted one operation per arithmetic
# step of the recurrence: H - open (1); E: subtract + max (2); F: subtract + max
# (2); diagonal add (1); substitution select (1); H: two maxima (2); running
# maximum (1).  The kernel fuses several of them (3-input maxima, the
# column-shifted domain), so this count can exceed what the VALU issues.
ALGO_OPS_PER_CELL = 10


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def profiled_counters():
    """Counters of one engine-kernel launch on this workload, from the committed rocprofv3
    summary: HBM bytes per launch and VALU instructions per cell.  ``match`` says whether the
    kernel source is the one that was profiled (sha256 prefix)."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "engine_kernel_5Mx4M_counters.md")
    src = os.path.join(ROOT, "paper_1304_5966_amd", "csrc", "engine.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    keys = ("traffic_bytes", "engine_hip_sha256_prefix", "sq_insts_valu", "cells")
    fields = {}
    for line in text.splitlines():
        k, sep, v = line.partition(": ")
        if sep and k in keys:
            fields[k] = v.strip()
    if not all(k in fields for k in keys):
        return None
    return {"match": fields["engine_hip_sha256_prefix"] == sha,
            "traffic": int(float(fields["traffic_bytes"])),
            "valu_per_cell": float(fields["sq_insts_valu"]) * LANES / float(fields["cells"])}


def roofline(cells, kernel_s, counters):
    """Roofline of the dominant kernel.  ``achieved`` is the VALU lane-instruction rate the
    kernel issues (instructions per cell from the profiled counters, times cells, over the
    live kernel time), so ``frac`` is the VALU issue fraction of the published peak.  The
    algorithmic rate (ALGO_OPS_PER_CELL operations per cell) is reported beside it."""
    algo = ALGO_OPS_PER_CELL * cells / kernel_s
    out = {"bound": "alu", "unit": "Tops/s int32", "peak": round(VALU_PEAK / 1e12, 3),
           "kernel_ms": round(kernel_s * 1000, 3),
           "algorithmic_ops_per_cell": ALGO_OPS_PER_CELL,
           "algorithmic_tops": round(algo / 1e12, 3),
           "algorithmic_frac": round(algo / VALU_PEAK, 4)}
    if counters is None:
        out.update({"achieved": None, "frac": None, "traffic": None, "valu_per_cell": None,
                    "counters": "no counter summary"})
        return out
    if not counters["match"]:  # counted on another kernel source: no instruction count, no traffic
        out.update({"achieved": None, "frac": None, "traffic": None, "valu_per_cell": None,
                    "counters": "profiles/engine_kernel_5Mx4M_counters.md (taken on another kernel source)"})
        return out
    issued = counters["valu_per_cell"] * cells / kernel_s
    out.update({"achieved": round(issued / 1e12, 3), "frac": round(issued / VALU_PEAK, 4),
                "valu_per_cell": round(counters["valu_per_cell"], 3), "traffic": counters["traffic"],
                "counters": "profiles/engine_kernel_5Mx4M_counters.md"})
    return out


def cpu_baseline(pair, target_s=15.0):
    """The oracle (plain C, 64-bit integers, linear space, row stripes on every host core it
    may use) on a crop of the same pair around its planted piece: a short probe run sizes a
    square crop for about target_s seconds of work, which is then timed."""
    import oracle
    pl = pair.planted[0]
    threads = oracle.host_cores()

    def timed(side):
        a = pair.a[pl.a_off:pl.a_off + side].tobytes()
        b = pair.b[pl.b_off:pl.b_off + side].tobytes()
        t0 = time.perf_counter()
        # columns in chunks of 2 048 so that each stripe hands many chunks down the pipeline
        oracle.sw_score_mt(a, b, threads=threads, chunk_cols=2048)
        return a, b, time.perf_counter() - t0

    _, _, dt = timed(40_000)
    side = int(40_000 * (target_s / max(dt, 1e-3)) ** 0.5)
    a, b, dt = timed(side)
    cells = len(a) * len(b)
    return {"value": cells / dt / 1e9, "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": f"{len(a)} x {len(b)} crop of the same pair starting at its planted piece "
                      f"({cells:.3g} cells, {dt:.1f} s; linear-space C oracle, 64-bit integers, "
                      f"row stripes of 512 rows, chunks of 2 048 columns, on {threads} threads)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rows-per-lane", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (shape 8 rows/lane, 8 waves/CU)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the pruned, batched and learned legs")
    ap.add_argument("--learned-pairs", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device-to-device (scale for the FETCH_SIZE/WRITE_SIZE counters)")
    ap.add_argument("--seq-sample", type=int, default=2000)
    ap.add_argument("--no-genome", action="store_true", help="skip the genome-scale leg (about 5 minutes)")
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="seconds the whole run may take: an extra leg whose usual duration no longer fits "
                         "is skipped and reported as such (the CPU baseline always runs)")
    ap.add_argument("--only", choices=("batched", "learned", "align", "genome", "protein"), default=None,
                    help="run one extra leg alone and print its JSON object")
    args = ap.parse_args()
    t_run = time.perf_counter()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the score pass is "
              f"not sharded across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1304_5966_amd import swmi, synth

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "dispatches": 3}), flush=True)
        return

    opts = dict(rows_per_lane=args.rows_per_lane, waves_per_cu=args.waves_per_cu)
    if args.only == "genome":
        print(json.dumps(genome_leg(swmi.Context(0), torch, swmi, synth)), flush=True)
        return
    if args.only == "protein":
        print(json.dumps(protein_leg(swmi.Context(0), torch, swmi, synth)), flush=True)
        return
    if args.only in ("batched", "learned"):
        ctx = swmi.Context(0)
        fixed = bool(args.rows_per_lane or args.waves_per_cu)
        if fixed:  # a fixed shape for the leg's launches instead of the tuner's
            ctx.set_tuning(swmi.TUNE_BATCH, args.rows_per_lane, args.waves_per_cu)
        leg = (batched_leg(ctx, torch, swmi, synth, args.seq_sample, not (args.no_tune or fixed))
               if args.only == "batched"
               else learned_leg(ctx, torch, swmi, synth, args.learned_pairs))
        print(json.dumps(leg), flush=True)
        return

    log("generating the 5 Mbp x 4 Mbp pair")
    pair = synth.config2()
    M, N = pair.a.size, pair.b.size
    dev = torch.device("cuda:0")
    d_a = torch.from_numpy(pair.a).to(dev)
    d_b = torch.from_numpy(pair.b).to(dev)
    ctx = swmi.Context(0)
    if args.only == "align":
        print(json.dumps(alignment_leg(ctx, torch, pair, d_a, d_b, opts)), flush=True)
        return
    tune = None
    if not (args.no_tune or args.rows_per_lane or args.waves_per_cu):
        from paper_1304_5966_amd import autotune
        log("autotuning the engine shape on the pair itself (one pass per candidate)")
        tune = {"sample": "the whole pair, one pass per candidate", "candidates": []}
        tune["chosen"] = autotune.tune_score(ctx, d_a, d_b, use_cache=False, log=log, table=tune["candidates"],
                                             candidates=[(8, 6), (8, 8), (8, 10), (8, 12), (4, 12)])
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
        "roofline": roofline(cells, gpu_ms / 1000, profiled_counters()),
        "engine_shape": tune["chosen"] if tune else {"rows_per_lane": args.rows_per_lane or 8,
                                                      "waves_per_cu": args.waves_per_cu or 8},
    }
    if tune:
        line["autotune"] = tune
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
        legs = [("alignment", lambda: alignment_leg(ctx, torch, pair, d_a, d_b, opts)),
                ("batched", lambda: batched_leg(ctx, torch, swmi, synth, args.seq_sample, not args.no_tune)),
                ("learned_pruned", lambda: learned_leg(ctx, torch, swmi, synth, args.learned_pairs)),
                ("protein", lambda: protein_leg(ctx, torch, swmi, synth))]
        for key, run in legs:
            line[key] = run_leg(key, run, t_run, args.time_budget)
    if not args.no_cpu:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(pair)
    if not (args.no_extra or args.no_genome):
        line["genome_scale"] = run_leg("genome_scale", lambda: genome_leg(ctx, torch, swmi, synth),
                                       t_run, args.time_budget)
    print(json.dumps(line), flush=True)


# Usual wall-clock seconds of each extra leg on one MI355X (pair generation included),
# with some margin: a leg runs only if this much time is left in the run's budget.
LEG_SECONDS = {"alignment": 30, "batched": 75, "learned_pruned": 90, "protein": 45, "genome_scale": 320}


def run_leg(key, run, t_run, budget):
    """Run one extra leg if its usual duration fits in what is left of the time budget."""
    left = budget - (time.perf_counter() - t_run)
    if LEG_SECONDS[key] > left:
        log(f"{key} leg skipped: {left:.0f} s left of the {budget:.0f} s budget, the leg takes about "
            f"{LEG_SECONDS[key]} s")
        return {"skipped": f"time budget: {left:.0f} s left of {budget:.0f} s, the leg takes about "
                           f"{LEG_SECONDS[key]} s (run it with --only or a larger --time-budget)"}
    return run()


def alignment_leg(ctx, torch, pair, d_a, d_b, opts):
    """The three phases on the 5 Mbp x 4 Mbp pair: score pass, start pass, reconstruction.

    ``sw_align`` runs all three on host letters (upload included); the start pass is also
    timed alone through ``sw_start``, and the reconstruction is the remainder."""
    a, b = pair.a.tobytes(), pair.b.tobytes()
    M, N = len(a), len(b)
    log("alignment leg: score pass")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sc = ctx.score_dev(d_a, d_b, **opts)
    t_score = time.perf_counter() - t0
    log("alignment leg: start pass")
    t0 = time.perf_counter()
    sa, sb = ctx.start(a, b, sc.score, sc.end_a, sc.end_b)
    t_start = time.perf_counter() - t0
    log("alignment leg: whole alignment")
    t0 = time.perf_counter()
    al = ctx.align(a, b, **opts)
    t_align = time.perf_counter() - t0
    assert (al.score, al.end_a, al.end_b) == sc.key(), (al, sc)
    assert (al.start_a, al.start_b) == (sa, sb), (al, sa, sb)
    la, lb = al.end_a - al.start_a + 1, al.end_b - al.start_b + 1
    ops = {o: 0 for o in "=XID"}
    n = 0
    for ch in al.cigar:
        if ch.isdigit():
            n = n * 10 + ord(ch) - 48
        else:
            ops[ch] += n
            n = 0
    t_rec = max(t_align - t_score - t_start, 0.0)
    log(f"alignment leg: score {t_score:.2f} s, start {t_start:.2f} s, whole {t_align:.2f} s")
    return {"workload": "the same 5 Mbp x 4 Mbp pair, score + start + Myers-Miller CIGAR",
            "score": al.score, "start": [al.start_a, al.start_b], "end": [al.end_a, al.end_b],
            "rectangle": [la, lb], "cigar_ops": ops, "cigar_runs": sum(1 for ch in al.cigar if not ch.isdigit()),
            "score_pass_s": round(t_score, 3), "start_pass_s": round(t_start, 3),
            "align_total_s": round(t_align, 3), "reconstruction_s": round(t_rec, 3),
            "score_pass_gcups": round(M * N / t_score / 1e9, 1)}


def genome_leg(ctx, torch, swmi, synth):
    """Score pass of the 32 Mbp x 28 Mbp genome-scale pair (letters resident on the device),
    running-best pruning, row slabs of at most 1e14 cells (one launch each)."""
    log("genome leg: generating the 32 Mbp x 28 Mbp pair")
    p = synth.config5()
    d_a, d_b = torch.from_numpy(p.a).cuda(), torch.from_numpy(p.b).cuda()
    cells = p.cells
    slabs = []
    t0 = time.perf_counter()

    def progress(done, total):
        slabs.append(round(time.perf_counter() - t0, 2))
        log(f"genome leg: {done}/{total} rows ({slabs[-1]:.1f} s)")

    ws = ctx.workspace(ctx.workspace_size(p.a.size, p.b.size, prune=swmi.PRUNE_BEST))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.score_dev(d_a, d_b, workspace=ws, prune=swmi.PRUNE_BEST, progress=progress)
    dt = time.perf_counter() - t0
    del ws
    return {"workload": "genome-scale pair: A 32 Mbp with GC-rich islands, B 28 Mbp from 40 shuffled, "
                        "mutated pieces of A (4 reverse-complemented); forward strand, running-best pruning",
            "cells": cells, "s": round(dt, 2), "gcups_eff": round(cells / dt / 1e9, 1),
            "cells_computed_frac": round(r.cells_computed / cells, 4), "slab_ends_s": slabs,
            "score": r.score, "end": [r.end_a, r.end_b]}


def _pack(pairs):
    import numpy as np
    a = np.concatenate([p.a for p in pairs])
    b = np.concatenate([p.b for p in pairs])
    oa = np.concatenate(([0], np.cumsum([p.a.size for p in pairs]))).astype(np.int64)
    ob = np.concatenate(([0], np.cumsum([p.b.size for p in pairs]))).astype(np.int64)
    return a, oa, b, ob


def batched_leg(ctx, torch, swmi, synth, seq_sample, tune):
    """20 000 pairs (100-20 000 bp, half homologous) in one launch vs one call per pair."""
    log("batched leg: generating 20 000 pairs")
    pairs = synth.config3()
    a, oa, b, ob = _pack(pairs)
    d_a, d_b = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    cells = sum(p.cells for p in pairs)
    table = []
    shape = None
    if tune:
        from paper_1304_5966_amd import autotune
        shape = autotune.tune_batch(ctx, d_a, oa, d_b, ob, use_cache=False, log=log, table=table)
    if shape is None:
        R, w = ctx.get_tuning(swmi.TUNE_BATCH)
        shape = {"rows_per_lane": R, "waves_per_cu": w, "tuned": False}
    ws = ctx.workspace(ctx.batch_workspace_size(oa, ob))
    ctx.batch_dev(d_a, oa, d_b, ob, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.batch_dev(d_a, oa, d_b, ob, workspace=ws)
    dt = time.perf_counter() - t0
    # the same launch captured as a HIP graph on a context bound to its own stream
    gstream = torch.cuda.Stream()
    gctx = swmi.Context(0, stream=gstream)
    gctx.set_tuning(swmi.TUNE_BATCH, shape["rows_per_lane"], shape["waves_per_cu"])
    gws = torch.empty(gctx.batch_workspace_size(oa, ob, graph=True), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    gres = gctx.batch_dev(d_a, oa, d_b, ob, workspace=gws, graph=True)   # capture + first replay
    t2 = time.perf_counter()
    gres = gctx.batch_dev(d_a, oa, d_b, ob, workspace=gws, graph=True)
    dtg = time.perf_counter() - t2
    assert [r.key() for r in gres] == [r.key() for r in res]
    gctx.close()
    del gws
    out = {"workload": "20 000 pairs, lengths log-uniform 100-20 000 bp per side, even pairs homologous "
                       "(divergence 5-30 %), odd pairs unrelated; one persistent launch",
           "gcups": round(cells / dt / 1e9, 2), "ms": round(dt * 1000, 2), "cells": cells,
           "graph_replay_gcups": round(cells / dtg / 1e9, 2), "graph_replay_ms": round(dtg * 1000, 2),
           "engine_shape": shape, "autotune_candidates": table}
    if seq_sample <= 0:
        log(f"batched: {cells / dt / 1e9:.1f} GCUPS")
        return out
    # the same pairs, one score call each (a seeded sample of the pairs, scaled)
    import numpy as np
    rng = np.random.default_rng(1)
    idx = np.sort(rng.choice(len(pairs), size=min(seq_sample, len(pairs)), replace=False))
    sample_cells = sum(pairs[i].cells for i in idx)
    dev_pairs = [(torch.from_numpy(pairs[i].a).cuda(), torch.from_numpy(pairs[i].b).cuda()) for i in idx]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    seq = [ctx.score_dev(x, y) for x, y in dev_pairs]
    dts = time.perf_counter() - t1
    for k, i in enumerate(idx):
        assert seq[k].key() == res[i].key(), (i, seq[k], res[i])
    log(f"batched: {cells / dt / 1e9:.1f} GCUPS; per-pair calls: {sample_cells / dts / 1e9:.1f} GCUPS")
    out.update({"per_pair_calls_gcups": round(sample_cells / dts / 1e9, 2), "per_pair_sample": int(len(idx)),
                "speedup_vs_per_pair": round((cells / dt) / (sample_cells / dts), 2)})
    return out


def protein_leg(ctx, torch, swmi, synth):
    """Substitution-matrix scoring (protein): the engine reads its scores from a query profile
    in LDS.  A 1 M x 1 M-letter pair (one launch) and a 20 000-pair batch, plain score pass,
    seeded random 20-letter matrix in the usual protein value range, gaps 11 / 1."""
    import numpy as np
    sc = swmi.MatrixScoring(synth.AMINO, synth.substitution_matrix(synth.SEED_PROTEIN), 11, 1)
    log("protein leg: 1 M x 1 M pair")
    p = synth.protein_pair(synth.SEED_PROTEIN, 1_000_000, 1_000_000, 0.3)
    d_a, d_b = torch.from_numpy(p.a).cuda(), torch.from_numpy(p.b).cuda()
    ws = ctx.workspace(ctx.workspace_size(p.a.size, p.b.size))
    r0 = ctx.score_dev(d_a, d_b, sc, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = ctx.score_dev(d_a, d_b, sc, workspace=ws)
    dt = time.perf_counter() - t0
    assert r.key() == r0.key()
    # the same shape with DNA scoring (row tables instead of the profile), for reference
    q = synth.homologous_pair(synth.SEED_PROTEIN, 1_000_000, 1_000_000, 0.3)
    q_a, q_b = torch.from_numpy(q.a).cuda(), torch.from_numpy(q.b).cuda()
    ctx.score_dev(q_a, q_b, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.score_dev(q_a, q_b, workspace=ws)
    dt_dna = time.perf_counter() - t0
    out = {"matrix": "seeded random 20 x 20, diagonal 4..11, off-diagonal -4..2; gap open 11, extend 1",
           "pair": {"workload": "1 000 000 x 1 000 000 letters, B holding a mutated copy of A (divergence 30 %)",
                    "gcups": round(p.cells / dt / 1e9, 1), "s": round(dt, 3), "score": r.score,
                    "dna_same_shape_gcups": round(q.cells / dt_dna / 1e9, 1)}}
    log("protein leg: 20 000-pair batch")
    pairs = synth.protein_batch()
    a, oa, b, ob = _pack(pairs)
    d_a, d_b = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    cells = sum(q.cells for q in pairs)
    ws = ctx.workspace(ctx.batch_workspace_size(oa, ob, sc))
    first = ctx.batch_dev(d_a, oa, d_b, ob, sc, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.batch_dev(d_a, oa, d_b, ob, sc, workspace=ws)
    dt = time.perf_counter() - t0
    assert np.array_equal(res.array, first.array)
    out["batch"] = {"workload": "20 000 pairs, lengths log-uniform 100-10 000 letters per side, even pairs "
                                "homologous (divergence 10-60 %), odd pairs unrelated; one persistent launch",
                    "cells": cells, "gcups": round(cells / dt / 1e9, 1), "ms": round(dt * 1000, 2)}
    log(f"protein leg: pair {out['pair']['gcups']} GCUPS, batch {out['batch']['gcups']} GCUPS")
    return out


def learned_leg(ctx, torch, swmi, synth, n_pairs):
    """Learned threshold against no pruning, running-best pruning and the true score as
    threshold (the ceiling), all batched, on a stratified draw of the 2 000-pair set."""
    from paper_1304_5966_amd import eval_learned
    path = os.path.join(ROOT, "paper_1304_5966_amd", "models", "threshold_mlp.bin")
    if not os.path.exists(path) or n_pairs <= 0:
        return {"status": "no trained model in the tree"}
    model = swmi.Model(ctx, path)
    idx = eval_learned.stratified_subset(n_pairs, seed=eval_learned.SUBSET_SEED + 1)
    log(f"learned leg: {len(idx)} pairs of 1-4 Mbp")
    part = eval_learned.evaluate(ctx, model, idx, chunk=len(idx), log=log)
    model.close()
    out = eval_learned.summarize([part])
    out["workload"] = (f"{len(idx)} pairs of the 2 000-pair learned-pruning set (1-4 Mbp per side), a seeded "
                       f"draw keeping the set's mix ({part['homologous']} homologous); one batched launch per mode")
    out["indices"] = idx
    return out


if __name__ == "__main__":
    main()
