"""Full-size pairs on the GPU, checked against stored oracle results and through properties.

Stored oracle results (tests/golden/, written by make_goldens.py from the CPU
oracle alone): score and endpoint of all 20 000 batched pairs; score, endpoint
and start of the 5 Mbp x 4 Mbp pair (multi-threaded linear-space oracle).
Each file carries the SHA-256 of the generated letters; a mismatch means the
generator changed, not the library.

Beyond those, the 5 Mbp x 4 Mbp pair is checked by:
the alignment's score and endpoint equal the score pass's; its CIGAR rescores
to the score and lands on the endpoint; the planted alignment bounds the score
from below; and sampled windows of the path are optimal.  The last check rests
on a fact of affine-gap alignment: cut an optimal path at two points that are
each reached by an aligned pair; the piece between them is an optimal global
alignment of its block (a better one, spliced in, would only open the same or
fewer gaps at the cuts and improve the whole path).  The oracle computes each
block's global optimum one by one.

The whole 32 Mbp x 28 Mbp genome-scale pair runs its score pass in row slabs
(a few minutes of GPU time) and is checked by the same properties.
"""
import hashlib
import json
import os
import time

import numpy as np
import pytest

from paper_1304_5966_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def letters_sha(pairs) -> str:
    h = hashlib.sha256()
    for p in pairs:
        h.update(p.a.tobytes())
        h.update(b"|")
        h.update(p.b.tobytes())
        h.update(b"#")
    return h.hexdigest()


def golden_config3(pairs):
    path = os.path.join(GOLDEN, "config3_score_end.csv")
    with open(path) as f:
        lines = f.read().splitlines()
    sha = lines[1].split()[-1]
    assert sha == letters_sha(pairs), "the batch generator changed since the stored results were written"
    rows = [tuple(int(v) for v in ln.split(",")) for ln in lines[3:]]
    assert [r[0] for r in rows] == list(range(len(pairs)))
    return [r[1:] for r in rows]


def golden_config2(pair):
    with open(os.path.join(GOLDEN, "config2.json")) as f:
        g = json.load(f)
    assert g["letters_sha256"] == letters_sha([pair]), "the pair generator changed"
    return g


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


def _check_windows(a, b, al, orc, rng, n_windows=8, span=3000):
    """Rescore path pieces between ends of aligned runs against the oracle's global optimum."""
    runs = orc.parse_cigar(al.cigar)
    i, j, pts = al.start_a, al.start_b, []  # (i, j, run index) after each run of aligned pairs
    for r, (n, o) in enumerate(runs):
        if o in "=X":
            i += n
            j += n
            pts.append((i, j, r))
        elif o == "I":
            j += n
        else:
            i += n
    assert len(pts) > 4
    for k in np.sort(rng.choice(len(pts) - 1, size=min(n_windows, len(pts) - 1), replace=False)):
        i0, j0, r0 = pts[k]
        m = k + 1
        while m + 1 < len(pts) and pts[m + 1][0] - i0 <= span and pts[m + 1][1] - j0 <= span:
            m += 1
        i1, j1, r1 = pts[m]
        cig = "".join(f"{n}{o}" for n, o in runs[r0 + 1:r1 + 1])
        seg, ea, eb = orc.rescore(a[i0:i1], b[j0:j1], 0, 0, cig)
        assert (ea, eb) == (i1 - i0 - 1, j1 - j0 - 1)
        opt = orc.global_score(a[i0:i1], b[j0:j1])
        assert seg == opt, ((i0, j0, i1, j1), seg, opt)


def test_config2_alignment_properties(ctx, orc):
    p = synth.config2()
    a, b = p.a.tobytes(), p.b.tobytes()
    _case("config2 score pass")
    t0 = time.perf_counter()
    sc = ctx.score(a, b)
    _case(f"config2 alignment (score pass {time.perf_counter() - t0:.2f} s)")
    t0 = time.perf_counter()
    al = ctx.align(a, b)
    print(f"config2 alignment {al.score} {al.start_a} {al.start_b} {al.end_a} {al.end_b} "
          f"({time.perf_counter() - t0:.2f} s)", flush=True)
    assert (al.score, al.end_a, al.end_b) == sc.key()
    _case("config2 score pass in four row slabs")
    assert ctx.score(a, b, slab_rows=1_250_000).key() == sc.key()
    g = golden_config2(p) if os.path.exists(os.path.join(GOLDEN, "config2.json")) else {}
    if "score" in g:
        assert sc.key() == (g["score"], g["end_a"], g["end_b"])
    if "start_a" in g:
        assert (al.start_a, al.start_b) == (g["start_a"], g["start_b"])
    assert orc.rescore(a, b, al.start_a, al.start_b, al.cigar) == (al.score, al.end_a, al.end_b)
    pl = p.planted[0]
    planted, _, _ = orc.rescore(a, b, pl.a_off, pl.b_off, pl.transcript.cigar())
    assert al.score >= planted > 0.9 * pl.a_len
    _check_windows(a, b, al, orc, np.random.default_rng(2))


def test_config5_genome_scale_alignment(ctx, orc, capsys):
    """The whole 32 Mbp x 28 Mbp genome-scale pair (8.96e14 cells): the score pass runs as
    row slabs of at most 1e14 cells (one launch each, progress printed between them) with
    running-best pruning, then the start pass and the reconstruction of the best alignment.
    Checked by rescoring, by every planted forward-strand segment as a lower bound, and by
    oracle-optimal windows of the path."""
    from paper_1304_5966_amd import swmi

    def say(msg):  # the test runs for minutes: its progress goes past the output capture
        with capsys.disabled():
            print(msg, flush=True)

    say("[case] config5: generating the pair")
    p = synth.config5()
    a, b = p.a.tobytes(), p.b.tobytes()
    t0 = time.perf_counter()

    def progress(done, total):
        say(f"config5 score pass: {done}/{total} rows ({time.perf_counter() - t0:.1f} s)")

    say("[case] config5 alignment (score pass in row slabs, running-best pruning)")
    al = ctx.align(a, b, prune=swmi.PRUNE_BEST, progress=progress)
    say(f"config5 alignment {al.score} {al.start_a} {al.start_b} {al.end_a} {al.end_b} "
        f"({time.perf_counter() - t0:.2f} s)")
    assert orc.rescore(a, b, al.start_a, al.start_b, al.cigar) == (al.score, al.end_a, al.end_b)
    fwd = [pl for pl in p.planted if pl.strand == 0]
    assert fwd
    for pl in fwd:
        assert al.score >= orc.rescore(a, b, pl.a_off, pl.b_off, pl.transcript.cigar())[0]
    _check_windows(a, b, al, orc, np.random.default_rng(5))


def test_config4_pair_against_stored_oracle(ctx):
    """A 1.06 Mbp x 1.01 Mbp pair of the learned-pruning evaluation set (pair 581, with a
    homologous segment) in every pruning mode, against the oracle's stored score and endpoint."""
    from paper_1304_5966_amd import swmi, train
    path = os.path.join(GOLDEN, "config4_pair581.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle result not written")
    with open(path) as f:
        g = json.load(f)
    p = synth.config4_pair(581)
    assert g["letters_sha256"] == letters_sha([p]), "the pair generator changed"
    exp = (g["score"], g["end_a"], g["end_b"])
    a, b = p.a.tobytes(), p.b.tobytes()
    modes = [dict(prune=swmi.PRUNE_NONE), dict(prune=swmi.PRUNE_BEST),
             dict(prune=swmi.PRUNE_LEARNED, threshold=exp[0]), dict(prune=swmi.PRUNE_LEARNED, threshold=exp[0] + 1)]
    model = swmi.Model(ctx, train.DEFAULT_OUT) if os.path.exists(train.DEFAULT_OUT) else None
    if model:
        modes.append(dict(prune=swmi.PRUNE_LEARNED, model=model.handle))
    for kw in modes:
        _case(f"config4 pair 581 {kw}")
        assert ctx.score(a, b, **kw).key() == exp, kw
    if model:
        model.close()


def test_config3_full_launch(ctx, orc):
    """All 20 000 pairs of the batch workload in one launch, in the shape the benchmark's tuner
    picks (6 rows per lane, 16 waves per CU): invariants on every pair, identical results under
    running-best pruning and on graph replays, and every pair equal to the stored oracle result."""
    import torch
    from paper_1304_5966_amd import swmi

    _case("config3: generating 20 000 pairs")
    pairs = synth.config3()
    a = np.concatenate([p.a for p in pairs])
    b = np.concatenate([p.b for p in pairs])
    oa = np.concatenate(([0], np.cumsum([p.a.size for p in pairs]))).astype(np.int64)
    ob = np.concatenate(([0], np.cumsum([p.b.size for p in pairs]))).astype(np.int64)
    d_a, d_b = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    shape = dict(rows_per_lane=6, waves_per_cu=16)

    _case("config3: one launch, no pruning, R = 6 at 16 waves per CU")
    keys = ctx.batch_dev(d_a, oa, d_b, ob, **shape).keys()
    assert len(keys) == len(pairs)
    for p, (s, ea, eb) in zip(pairs, keys):
        la, lb = p.a.size, p.b.size
        assert 0 <= s <= min(la, lb), p.tag  # match = +1
        if s == 0:
            assert (ea, eb) == (-1, -1), p.tag
        else:
            assert 0 <= ea < la and 0 <= eb < lb, p.tag

    _case("config3: one launch, running-best pruning")
    assert ctx.batch_dev(d_a, oa, d_b, ob, prune=swmi.PRUNE_BEST, **shape).keys() == keys

    _case("config3: captured graph, two replays")
    gstream = torch.cuda.Stream()
    gctx = swmi.Context(0, stream=gstream)
    try:
        gws = torch.empty(gctx.batch_workspace_size(oa, ob, graph=True, **shape), dtype=torch.uint8, device="cuda")
        for _ in range(2):
            assert gctx.batch_dev(d_a, oa, d_b, ob, workspace=gws, graph=True, **shape).keys() == keys
    finally:
        gctx.close()

    _case("config3: every pair against the stored oracle results")
    gold = golden_config3(pairs)
    bad = [i for i in range(len(pairs)) if keys[i] != gold[i]]
    assert not bad, [(i, keys[i], gold[i]) for i in bad[:10]]
