"""The seeded generators: reproducible, rates as specified, transcripts consistent."""
import numpy as np

from paper_1304_5966_amd import synth


def _apply(src, out, tr):
    """Replay a transcript: every '=' base equals its source, every 'X' differs."""
    i = j = 0
    for o, n in zip(tr.ops.tolist(), tr.lens.tolist()):
        o = chr(o)
        if o == "=":
            assert np.array_equal(src[i:i + n], out[j:j + n])
            i += n
            j += n
        elif o == "X":
            assert np.all(src[i:i + n] != out[j:j + n])
            i += n
            j += n
        elif o == "I":
            j += n
        else:
            i += n
    return i, j


def test_reproducible():
    a = synth.config1()
    b = synth.config1()
    assert np.array_equal(a.a, b.a) and np.array_equal(a.b, b.b)
    assert a.a.size == 10_000 and a.b.size == 8_000
    p = synth.config3_pair(17)
    q = synth.config3_pair(17)
    assert np.array_equal(p.a, q.a) and np.array_equal(p.b, q.b)
    assert set(np.unique(p.a).tobytes()) <= set(b"ACGT")


def test_mutation_rates_and_transcript():
    rng = synth.rng_for(5)
    src = synth.random_dna(rng, 200_000)
    out, tr = synth.mutate(rng, src, 0.05, 0.005)
    i, j = _apply(src, out, tr)
    assert i == src.size and j == out.size
    ops = {chr(o): int(n) for o, n in zip(*np.unique(np.repeat(tr.ops, 1), return_counts=True))}
    n_sub = int(tr.lens[tr.ops == ord("X")].sum())
    # binomial 5 % of 200k: sd ~ 97; allow 6 sd
    assert abs(n_sub - 10_000 * (1 - 0.005 * 1.5)) < 700
    n_events = int((tr.ops == ord("I")).sum() + (tr.ops == ord("D")).sum())
    assert 800 < n_events < 1200
    mean_len = tr.lens[(tr.ops == ord("I")) | (tr.ops == ord("D"))].mean()
    assert 2.5 < mean_len < 3.6
    assert ops


def test_planted_transcripts_replay():
    for p in (synth.config1(), synth.config3_pair(0), synth.config3_pair(2)):
        pl = p.planted[0]
        i, j = _apply(p.a[pl.a_off:], p.b[pl.b_off:], pl.transcript)
        assert i == pl.a_len
        assert pl.b_off + j <= p.b.size


def test_config3_shape():
    lens = np.array([[synth.config3_pair(i).a.size, synth.config3_pair(i).b.size]
                     for i in range(0, 400)])
    assert lens.min() >= 100 and lens.max() <= 20_000
    # log-uniform: median near sqrt(100 * 20000) ~ 1414
    assert 900 < np.median(lens) < 2200


def test_genome_scale_planted_copies_on_both_strands():
    """Every planted copy of the genome-scale generator replays against its strand of B:
    forward copies in B, reverse-complemented ones in the reverse complement of B."""
    p = synth.config5(len_a=400_000, len_b=350_000, n_seg=10)
    rcb = synth.reverse_complement(p.b)
    strands = {pl.strand for pl in p.planted}
    assert strands == {0, 1}
    for pl in p.planted:
        bb = p.b if pl.strand == 0 else rcb
        i, j = _apply(p.a[pl.a_off:], bb[pl.b_off:], pl.transcript)
        assert i == pl.a_len


def test_learned_set_metadata_matches_the_pairs():
    for i in (0, 1, 7, 123):
        la, lb, hom = synth.config4_meta(i)
        p = synth.config4_pair(i)
        assert (p.a.size, p.b.size, p.homologous) == (la, lb, hom)


def test_stratified_subset_keeps_the_mix():
    from paper_1304_5966_amd import eval_learned
    idx = eval_learned.stratified_subset(200)
    assert len(idx) == len(set(idx)) == 200 and idx == sorted(idx)
    assert sum(synth.config4_meta(i)[2] for i in idx) == 80
    assert eval_learned.stratified_subset(200) == idx


def test_protein_generators():
    m = synth.substitution_matrix(3)
    assert m.dtype == np.int8 and m.shape == (20, 20) and (m == m.T).all()
    assert (np.diag(m) >= 4).all() and (np.diag(m) <= 11).all()
    off = m[~np.eye(20, dtype=bool)]
    assert off.min() >= -4 and off.max() <= 2
    assert not (synth.substitution_matrix(3, symmetric=False) == synth.substitution_matrix(3, symmetric=False).T).all()
    for la, lb in [(1, 1), (300, 250), (64, 2000), (5000, 80)]:
        p = synth.protein_pair(9, la, lb, 0.3)
        assert (p.a.size, p.b.size) == (la, lb)
        assert set(p.a.tobytes()) <= set(synth.AMINO) and set(p.b.tobytes()) <= set(synth.AMINO)
        q = synth.protein_pair(9, la, lb, 0.3)
        assert (p.a == q.a).all() and (p.b == q.b).all()
    # a low divergence copy shares long exact runs with A
    p = synth.protein_pair(4, 2000, 2000, 0.02)
    assert p.b[100:140].tobytes() in p.a.tobytes() or p.b[1000:1040].tobytes() in p.a.tobytes()
    batch = [synth.protein_batch_pair(i) for i in range(40)]
    assert all(100 <= x.a.size <= 10_000 and 100 <= x.b.size <= 10_000 for x in batch)
    assert [x.homologous for x in batch[:4]] == [True, False, True, False]
