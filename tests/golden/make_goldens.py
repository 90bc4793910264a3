"""Writes the stored expected results of the full-size workloads, from the CPU oracle only.

    python tests/golden/make_goldens.py config3 [--threads T]
    python tests/golden/make_goldens.py config2 [--threads T]
    python tests/golden/make_goldens.py config4 --index I [--threads T]

config3: score and endpoint of all 20 000 pairs of the batched workload
(seed 13045969), each pair by the single-threaded linear-space oracle, pairs
spread over T threads -> ``config3_score_end.csv``.

config2: score, endpoint and start point of the 5 Mbp x 4 Mbp pair (seed
13045968) by the multi-threaded linear-space oracle (row stripes on T
threads; the start by the anchored reverse pass on the reversed prefixes) ->
``config2.json``.  About 3.5e13 cells: hours on a few cores.

config4: score and endpoint of pair I of the learned-pruning evaluation set
(1-4 Mbp per side; seed 13045971) by the multi-threaded linear-space oracle ->
``config4_pair<I>.json``.

Each file records the SHA-256 of the generated letters, so a test can tell a
changed generator from a wrong result.  Nothing here touches the GPU library.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1304_5966_amd import synth  # noqa: E402


def letters_sha(pairs) -> str:
    h = hashlib.sha256()
    for p in pairs:
        h.update(p.a.tobytes())
        h.update(b"|")
        h.update(p.b.tobytes())
        h.update(b"#")
    return h.hexdigest()


def config3(threads: int) -> None:
    pairs = synth.config3()
    out = [None] * len(pairs)
    t0 = time.time()

    def one(i):
        out[i] = oracle.sw_score(pairs[i].a.tobytes(), pairs[i].b.tobytes())

    # largest pairs first, so the pool does not end on a long one
    order = sorted(range(len(pairs)), key=lambda i: -pairs[i].cells)
    with ThreadPoolExecutor(threads) as ex:
        for k, _ in enumerate(ex.map(one, order)):
            if k % 2000 == 0:
                print(f"config3: {k} pairs, {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(HERE, "config3_score_end.csv")
    with open(path + ".tmp", "w") as f:
        f.write(f"# oracle score and endpoint of the 20 000-pair batched workload (seed {synth.SEED_CONFIG3})\n")
        f.write(f"# letters_sha256 {letters_sha(pairs)}\n")
        f.write("pair,score,end_a,end_b\n")
        for i, (s, ea, eb) in enumerate(out):
            f.write(f"{i},{s},{ea},{eb}\n")
    os.replace(path + ".tmp", path)
    print(f"config3: wrote {path} ({time.time() - t0:.0f} s)", flush=True)


def config2(threads: int) -> None:
    p = synth.config2()
    a, b = p.a.tobytes(), p.b.tobytes()
    path = os.path.join(HERE, "config2.json")
    rec = {"workload": f"5 Mbp x 4 Mbp homologous pair, seed {synth.SEED_CONFIG2}",
           "letters_sha256": letters_sha([p]), "scoring": list(oracle.SCORING), "threads": threads}
    t0 = time.time()
    s, ea, eb = oracle.sw_score_mt(a, b, threads=threads)
    rec.update({"score": s, "end_a": ea, "end_b": eb, "score_pass_s": round(time.time() - t0, 1)})
    print(f"config2: score {s} end ({ea}, {eb}) in {time.time() - t0:.0f} s", flush=True)
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f, indent=1)
    os.replace(path + ".tmp", path)
    t1 = time.time()
    sa, sb = oracle.sw_start_mt(a, b, s, ea, eb, threads=threads)
    rec.update({"start_a": sa, "start_b": sb, "start_pass_s": round(time.time() - t1, 1)})
    print(f"config2: start ({sa}, {sb}) in {time.time() - t1:.0f} s", flush=True)
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f, indent=1)
    os.replace(path + ".tmp", path)


def config4(index: int, threads: int) -> None:
    p = synth.config4_pair(index)
    a, b = p.a.tobytes(), p.b.tobytes()
    path = os.path.join(HERE, f"config4_pair{index}.json")
    t0 = time.time()
    s, ea, eb = oracle.sw_score_mt(a, b, threads=threads)
    rec = {"workload": f"pair {index} of the learned-pruning evaluation set (seed {synth.SEED_CONFIG4_EVAL}), "
                       f"{len(a)} x {len(b)}, homologous segment: {p.homologous}",
           "letters_sha256": letters_sha([p]), "scoring": list(oracle.SCORING), "threads": threads,
           "score": s, "end_a": ea, "end_b": eb, "score_pass_s": round(time.time() - t0, 1)}
    print(f"config4 pair {index}: score {s} end ({ea}, {eb}) in {time.time() - t0:.0f} s", flush=True)
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f, indent=1)
    os.replace(path + ".tmp", path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=("config2", "config3", "config4"))
    ap.add_argument("--threads", type=int, default=oracle.host_cores())
    ap.add_argument("--index", type=int, default=581, help="config4: pair of the evaluation set")
    args = ap.parse_args()
    oracle.build()
    if args.which == "config4":
        config4(args.index, args.threads)
    else:
        (config2 if args.which == "config2" else config3)(args.threads)


if __name__ == "__main__":
    main()
