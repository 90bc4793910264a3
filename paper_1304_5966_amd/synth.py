"""Seeded synthetic DNA (and protein) workloads.

This module only *generates sequences*: iid bases, point substitutions,
insertions and deletions, segment shuffles and reverse complements.  The edit
transcript of every mutation is kept as plain bookkeeping (which source base
was copied, changed, dropped, or which bases were inserted).  Nothing here
scores an alignment or runs a dynamic program, so both the CPU oracle and the
GPU path can consume it without sharing any of the method's arithmetic.

Sequences are numpy ``uint8`` arrays of ASCII letters ``ACGT``.  Every
generator takes an integer seed and is reproducible bit for bit
(numpy PCG64 through ``default_rng``).

The workloads stand in for the genome-scale pairs of the paper's Table 1,
which are not available; their shapes follow the benchmark configurations:

* ``config1``: A = 10 kbp, B = 8 kbp holding a mutated 6 kbp piece of A.
* ``config2``: A = 5 Mbp, B = 4 Mbp holding a mutated 3.5 Mbp piece of A.
* ``config3_pair``: 20 000 pairs, log-uniform 100..20 000 bp per side,
  even pairs homologous (divergence 5..30 %), odd pairs unrelated.
* ``config4_pair``: 2 000 pairs of 1..4 Mbp, 40 % carrying a homologous
  segment (divergence 1..15 %, 5..60 % of the shorter length).
* ``config5``: A = 32 Mbp with GC-rich islands, B = 28 Mbp assembled from 40
  shuffled, partly reverse-complemented pieces of A.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ALPHABET = np.frombuffer(b"ACGT", dtype=np.uint8).copy()
_COMPLEMENT = np.zeros(256, dtype=np.uint8)
for _x, _y in zip(b"ACGTacgt", b"TGCAtgca"):
    _COMPLEMENT[_x] = _y

SEED_CONFIG1 = 13045967
SEED_CONFIG2 = 13045968
SEED_CONFIG3 = 13045969
SEED_CONFIG4_TRAIN = 13045970
SEED_CONFIG4_EVAL = 13045971
SEED_CONFIG5 = 13045972

N_CONFIG3 = 20_000
N_CONFIG4 = 2_000


def rng_for(seed: int, *index: int) -> np.random.Generator:
    """Independent stream for (seed, index...) so one pair can be rebuilt alone."""
    return np.random.default_rng(np.random.SeedSequence([int(seed), *[int(i) for i in index]]))


def random_dna(rng: np.random.Generator, n: int, probs=None) -> np.ndarray:
    """n iid bases over ACGT (uniform unless ``probs`` gives P(A,C,G,T))."""
    if n <= 0:
        return np.zeros(0, dtype=np.uint8)
    if probs is None:
        codes = rng.integers(0, 4, size=n, dtype=np.uint8)
    else:
        codes = rng.choice(4, size=n, p=np.asarray(probs, dtype=np.float64)).astype(np.uint8)
    return ALPHABET[codes]


def reverse_complement(seq: np.ndarray) -> np.ndarray:
    return _COMPLEMENT[np.asarray(seq, dtype=np.uint8)[::-1]]


def _codes(seq: np.ndarray) -> np.ndarray:
    lut = np.full(256, 255, dtype=np.uint8)
    for i, ch in enumerate(b"ACGT"):
        lut[ch] = i
        lut[ch + 32] = i
    return lut[seq]


@dataclass
class Transcript:
    """Run-length edit transcript of ``src -> out``: ops in '=XID', A (src) is the reference.

    '=' copied base, 'X' substituted base, 'I' base inserted into ``out``,
    'D' base of ``src`` dropped.
    """
    ops: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.uint8))
    lens: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))

    def cigar(self) -> str:
        return "".join(f"{int(n)}{chr(o)}" for o, n in zip(self.ops, self.lens))


def _runs_of_mask(mask: np.ndarray):
    """Run-length encode a boolean mask (True -> 'X', False -> '=')."""
    n = mask.size
    if n == 0:
        return [], []
    change = np.nonzero(mask[1:] != mask[:-1])[0] + 1
    starts = np.concatenate(([0], change))
    ends = np.concatenate((change, [n]))
    ops = np.where(mask[starts], ord("X"), ord("=")).astype(np.uint8)
    return list(ops), list((ends - starts).astype(np.int64))


def _merge_runs(ops, lens) -> Transcript:
    out_o, out_l = [], []
    for o, n in zip(ops, lens):
        if n <= 0:
            continue
        if out_o and out_o[-1] == o:
            out_l[-1] += int(n)
        else:
            out_o.append(int(o))
            out_l.append(int(n))
    return Transcript(np.asarray(out_o, dtype=np.uint8), np.asarray(out_l, dtype=np.int64))


def mutate(rng: np.random.Generator, src: np.ndarray, sub_rate: float, indel_rate: float,
           mean_indel: float = 3.0, ins_share: float = 0.5):
    """Copy ``src`` with point substitutions and geometric-length indels.

    Per source base: a substitution (to a uniformly chosen *other* base) with
    probability ``sub_rate``; independently an indel event with probability
    ``indel_rate`` -- an insertion of L random bases before the base or a
    deletion of L bases starting at it (insertion with probability
    ``ins_share``), L ~ Geometric(1/mean_indel) on {1, 2, ...}.
    Returns ``(out, transcript)``.
    """
    src = np.asarray(src, dtype=np.uint8)
    n = src.size
    codes = _codes(src)
    sub = rng.random(n) < sub_rate
    newc = codes.copy()
    k = int(sub.sum())
    if k:
        newc[sub] = (codes[sub] + rng.integers(1, 4, size=k, dtype=np.uint8)) % 4
    ev = np.nonzero(rng.random(n) < indel_rate)[0]
    is_ins = rng.random(ev.size) < ins_share
    lens = rng.geometric(1.0 / mean_indel, size=ev.size).astype(np.int64)
    pieces, ops, olens = [], [], []
    pos = 0
    for p, ins, L in zip(ev.tolist(), is_ins.tolist(), lens.tolist()):
        if p < pos:
            continue  # swallowed by an earlier deletion
        pieces.append(newc[pos:p])
        o, l = _runs_of_mask(sub[pos:p])
        ops += o
        olens += l
        if ins:
            pieces.append(rng.integers(0, 4, size=L, dtype=np.uint8))
            ops.append(ord("I"))
            olens.append(L)
            pos = p
        else:
            L = min(L, n - p)
            ops.append(ord("D"))
            olens.append(L)
            pos = p + L
    pieces.append(newc[pos:])
    o, l = _runs_of_mask(sub[pos:])
    ops += o
    olens += l
    out = ALPHABET[np.concatenate(pieces)] if pieces else np.zeros(0, dtype=np.uint8)
    return out, _merge_runs(ops, olens)


@dataclass
class Planted:
    """Where a mutated copy of ``a[a_off : a_off + a_len]`` sits in ``b`` (from ``b_off``).

    strand 1: the copy sits in the reverse complement of ``b`` (``b_off`` and the
    transcript refer to that sequence).
    """
    a_off: int
    a_len: int
    b_off: int
    transcript: Transcript
    strand: int = 0


@dataclass
class Pair:
    a: np.ndarray
    b: np.ndarray
    planted: list = field(default_factory=list)
    homologous: bool = False
    tag: str = ""

    @property
    def cells(self) -> int:
        return int(self.a.size) * int(self.b.size)


def _clip_transcript(tr: Transcript, max_out: int) -> tuple[Transcript, int]:
    """Keep the prefix of a transcript that produces at most ``max_out`` output bases.

    Returns the clipped transcript and the number of source bases it consumes.
    """
    ops, lens = [], []
    out_used = 0
    src_used = 0
    for o, n in zip(tr.ops.tolist(), tr.lens.tolist()):
        consumes_out = o in (ord("="), ord("X"), ord("I"))
        consumes_src = o in (ord("="), ord("X"), ord("D"))
        if consumes_out:
            n = min(n, max_out - out_used)
            if n <= 0:
                break
            out_used += n
        ops.append(o)
        lens.append(n)
        if consumes_src:
            src_used += n
    # a transcript should not end with a dropped-source run after clipping
    while ops and ops[-1] == ord("D"):
        src_used -= lens[-1]
        ops.pop()
        lens.pop()
    return _merge_runs(ops, lens), src_used


def embed_homolog(rng, a: np.ndarray, len_b: int, core_len: int, sub_rate: float,
                  indel_rate: float, mean_indel: float = 3.0, flank: str = "pad") -> Pair:
    """B of length ``len_b``: a mutated copy of a random ``core_len`` piece of A in random flanks.

    If the mutated core is longer than ``len_b`` it is trimmed at its end.
    """
    core_len = min(core_len, a.size)
    a_off = int(rng.integers(0, a.size - core_len + 1))
    core, tr = mutate(rng, a[a_off:a_off + core_len], sub_rate, indel_rate, mean_indel)
    if core.size >= len_b:
        tr, src_used = _clip_transcript(tr, len_b)
        b = core[:len_b].copy()
        return Pair(a, b, [Planted(a_off, src_used, 0, tr)], True)
    left = int(rng.integers(0, len_b - core.size + 1))
    b = np.concatenate((random_dna(rng, left), core, random_dna(rng, len_b - core.size - left)))
    return Pair(a, b, [Planted(a_off, core_len, left, tr)], True)


# --------------------------------------------------------------------------- configs

def config1(seed: int = SEED_CONFIG1) -> Pair:
    """10 kbp x 8 kbp; B holds a 6 kbp piece of A with 5 % substitutions, 0.5 % indels."""
    rng = rng_for(seed)
    a = random_dna(rng, 10_000)
    p = embed_homolog(rng, a, 8_000, 6_000, 0.05, 0.005)
    p.tag = "config1"
    return p


def config2(seed: int = SEED_CONFIG2) -> Pair:
    """5 Mbp x 4 Mbp; B holds a 3.5 Mbp piece of A with 1 % substitutions, 0.1 % indels."""
    rng = rng_for(seed)
    a = random_dna(rng, 5_000_000)
    p = embed_homolog(rng, a, 4_000_000, 3_500_000, 0.01, 0.001)
    p.tag = "config2"
    return p


def loguniform_len(rng, lo: int, hi: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def config3_pair(i: int, seed: int = SEED_CONFIG3) -> Pair:
    """Pair ``i`` of the 20 000-pair batch.

    Lengths log-uniform on [100, 20 000] per side.  Even ``i``: B is a mutated
    copy of min(|A|, |B|) bases of A (divergence d ~ U(0.05, 0.30) edits per
    source base, 90 % substitutions, 10 % indel events of geometric mean 3),
    trimmed or flank-padded to |B|.  Odd ``i``: unrelated iid sequences.
    """
    rng = rng_for(seed, i)
    la = loguniform_len(rng, 100, 20_000)
    lb = loguniform_len(rng, 100, 20_000)
    a = random_dna(rng, la)
    if i % 2 == 0:
        d = rng.uniform(0.05, 0.30)
        p = embed_homolog(rng, a, lb, min(la, lb), 0.9 * d, 0.1 * d)
    else:
        p = Pair(a, random_dna(rng, lb))
    p.tag = f"config3[{i}]"
    return p


def config3(n: int = N_CONFIG3, seed: int = SEED_CONFIG3) -> list:
    return [config3_pair(i, seed) for i in range(n)]


def segment_pair(rng, la: int, lb: int, div: float, indel_share: float, seg_frac: float) -> Pair:
    """Unrelated A and B except for one mutated segment of A written into B.

    The segment has ``seg_frac * min(la, lb)`` source bases; the edits per source
    base total ``div``, a fraction ``indel_share`` of them indel events.
    """
    a = random_dna(rng, la)
    b = random_dna(rng, lb)
    seg_len = max(1, int(seg_frac * min(la, lb)))
    a_off = int(rng.integers(0, la - seg_len + 1))
    core, tr = mutate(rng, a[a_off:a_off + seg_len], div * (1 - indel_share), div * indel_share)
    if core.size > lb:
        tr, used = _clip_transcript(tr, lb)
        core = core[:lb]
        seg_len = used
    b_off = int(rng.integers(0, lb - core.size + 1))
    b[b_off:b_off + core.size] = core
    return Pair(a, b, [Planted(a_off, seg_len, b_off, tr)], True)


def config4_pair(i: int, seed: int = SEED_CONFIG4_EVAL, lo: int = 1_000_000,
                 hi: int = 4_000_000) -> Pair:
    """Pair ``i`` of the learned-pruning set.

    |A|, |B| ~ U(lo, hi); with probability 0.4 the pair carries a homologous
    segment (divergence U(0.01, 0.15), 10 % indel share, segment length
    U(0.05, 0.60) x min(|A|, |B|)); otherwise unrelated.  The training set uses
    the same generator with another seed and shorter lengths.
    """
    rng = rng_for(seed, i)
    la = int(rng.integers(lo, hi + 1))
    lb = int(rng.integers(lo, hi + 1))
    if rng.random() < 0.4:
        p = segment_pair(rng, la, lb, rng.uniform(0.01, 0.15), 0.10, rng.uniform(0.05, 0.60))
    else:
        p = Pair(random_dna(rng, la), random_dna(rng, lb))
    p.tag = f"config4[{seed}:{i}]"
    return p


def config4_meta(i: int, seed: int = SEED_CONFIG4_EVAL, lo: int = 1_000_000,
                 hi: int = 4_000_000) -> tuple:
    """(|A|, |B|, homologous) of ``config4_pair(i)`` without generating its letters
    (the same first draws of the pair's generator)."""
    rng = rng_for(seed, i)
    la = int(rng.integers(lo, hi + 1))
    lb = int(rng.integers(lo, hi + 1))
    return la, lb, bool(rng.random() < 0.4)


def config5(seed: int = SEED_CONFIG5, len_a: int = 32_000_000, len_b: int = 28_000_000,
            n_seg: int = 40) -> Pair:
    """Genome-scale pair: A with GC-rich islands; B from shuffled, partly reverse-complemented pieces of A.

    Islands: regions of U(10 k, 100 k) bp with P(G)=P(C)=0.3 covering ~3 % of A.
    B: ``n_seg`` non-overlapping pieces of A (uniform Dirichlet lengths summing to
    ~|B|), shuffled, 10 % reverse-complemented, then 2 % substitutions and
    0.2 % indels, trimmed or padded to |B|.
    """
    rng = rng_for(seed)
    a = random_dna(rng, len_a)
    covered = 0
    while covered < 0.03 * len_a:
        L = int(rng.integers(10_000, 100_001))
        off = int(rng.integers(0, len_a - L))
        a[off:off + L] = random_dna(rng, L, probs=(0.2, 0.3, 0.3, 0.2))
        covered += L
    seg_lens = np.maximum(1, np.floor(rng.dirichlet(np.ones(n_seg)) * len_b).astype(np.int64))
    gap_total = max(0, len_a - int(seg_lens.sum()))
    gaps = np.floor(rng.dirichlet(np.ones(n_seg + 1)) * gap_total).astype(np.int64)
    offs = []
    pos = 0
    for k in range(n_seg):
        pos += int(gaps[k])
        offs.append(pos)
        pos += int(seg_lens[k])
    order = rng.permutation(n_seg)
    n_rc = max(1, int(round(0.1 * n_seg)))
    rc = np.zeros(n_seg, dtype=bool)
    rc[rng.choice(n_seg, size=n_rc, replace=False)] = True
    pieces, planted, planted_rc = [], [], []
    b_pos = 0
    for k in order.tolist():
        seg = a[offs[k]:offs[k] + int(seg_lens[k])]
        if rc[k]:
            seg = reverse_complement(seg)
        mut, tr = mutate(rng, seg, 0.02, 0.002)
        if not rc[k]:
            planted.append(Planted(offs[k], int(seg_lens[k]), b_pos, tr))
        else:
            # in the reverse complement of B the copy reads forward against A: the transcript
            # reversed (complementing both sides keeps every '=' and 'X')
            rev = Transcript(tr.ops[::-1].copy(), tr.lens[::-1].copy())
            planted_rc.append((offs[k], int(seg_lens[k]), b_pos + mut.size, rev))
        pieces.append(mut)
        b_pos += mut.size
    b = np.concatenate(pieces)
    if b.size >= len_b:
        b = b[:len_b].copy()
        keep = []
        for pl in planted:
            if pl.b_off >= len_b:
                continue
            tr, used = _clip_transcript(pl.transcript, len_b - pl.b_off)
            keep.append(Planted(pl.a_off, used, pl.b_off, tr))
        planted = keep
    else:
        b = np.concatenate((b, random_dna(rng, len_b - b.size)))
    for a_off, a_len, b_end, rev in planted_rc:
        if b_end <= len_b:  # copies cut by the trim are left out
            planted.append(Planted(a_off, a_len, len_b - b_end, rev, strand=1))
    p = Pair(a, b, planted, True)
    p.tag = "config5"
    return p


def random_pair(seed: int, la: int, lb: int, alphabet: bytes = b"ACGT") -> Pair:
    """Unrelated iid pair over ``alphabet`` (used for small parity cases)."""
    rng = rng_for(seed, la, lb)
    al = np.frombuffer(alphabet, dtype=np.uint8)
    return Pair(al[rng.integers(0, al.size, size=la)], al[rng.integers(0, al.size, size=lb)])


def homologous_pair(seed: int, la: int, lb: int, div: float = 0.1) -> Pair:
    """A random; B a mutated copy of min(la, lb) bases of A in flanks (small parity cases)."""
    rng = rng_for(seed, la, lb, 1)
    a = random_dna(rng, la)
    return embed_homolog(rng, a, lb, min(la, lb), 0.9 * div, 0.1 * div)


# --------------------------------------------------------------------------- protein

AMINO = b"ARNDCQEGHILKMFPSTWYV"  # the 20 amino-acid letters


def substitution_matrix(seed: int, k: int = 20, symmetric: bool = True) -> np.ndarray:
    """A seeded k x k int8 matrix in the value range of the usual protein matrices:
    diagonal 4..11, off-diagonal -4..2 (the paper prints no matrix, so tests and the
    benchmark draw one)."""
    rng = np.random.default_rng(seed)
    m = rng.integers(-4, 3, size=(k, k))
    if symmetric:
        m = np.triu(m) + np.triu(m, 1).T
    np.fill_diagonal(m, rng.integers(4, 12, size=k))
    return m.astype(np.int8)


def mutate_letters(rng: np.random.Generator, src: np.ndarray, alphabet: bytes, sub_rate: float,
                   indel_rate: float, mean_indel: float = 3.0) -> np.ndarray:
    """Copy ``src`` (letters of ``alphabet``) with substitutions to a uniform other letter
    and geometric-length insertions of random letters / deletions, as ``mutate`` does for DNA."""
    al = np.frombuffer(alphabet, dtype=np.uint8)
    k = al.size
    lut = np.zeros(256, dtype=np.int64)
    lut[al] = np.arange(k)
    codes = lut[np.asarray(src, dtype=np.uint8)]
    n = codes.size
    sub = rng.random(n) < sub_rate
    if k > 1 and sub.any():
        codes = codes.copy()
        codes[sub] = (codes[sub] + rng.integers(1, k, size=int(sub.sum()))) % k
    pieces, pos = [], 0
    for p in np.nonzero(rng.random(n) < indel_rate)[0].tolist():
        if p < pos:
            continue
        L = int(rng.geometric(1.0 / mean_indel))
        pieces.append(codes[pos:p])
        if rng.random() < 0.5:
            pieces.append(rng.integers(0, k, size=L))
            pos = p
        else:
            pos = min(n, p + L)
    pieces.append(codes[pos:])
    return al[np.concatenate(pieces)] if pieces else np.zeros(0, dtype=np.uint8)


def protein_pair(seed: int, la: int, lb: int, div: float = 0.3, alphabet: bytes = AMINO) -> Pair:
    """A: iid letters of ``alphabet``; B: a mutated copy (divergence ``div``, 90 % substitutions,
    10 % indel events) of min(la, lb) letters of A at a random offset, in random flanks,
    trimmed or padded to lb."""
    rng = rng_for(seed, la, lb, 7)
    al = np.frombuffer(alphabet, dtype=np.uint8)
    a = al[rng.integers(0, al.size, size=la)]
    core_len = min(la, lb)
    off = int(rng.integers(0, la - core_len + 1)) if la else 0
    core = mutate_letters(rng, a[off:off + core_len], alphabet, 0.9 * div, 0.1 * div)[:lb]
    left = int(rng.integers(0, lb - core.size + 1))
    b = np.concatenate((al[rng.integers(0, al.size, size=left)], core,
                        al[rng.integers(0, al.size, size=lb - core.size - left)]))
    return Pair(a, b.astype(np.uint8), [], True, "protein")


SEED_PROTEIN = 13045973
N_PROTEIN = 20_000


def protein_batch_pair(i: int, seed: int = SEED_PROTEIN) -> Pair:
    """Pair i of the protein batch: lengths log-uniform 100..10 000 letters per side; even
    pairs homologous (divergence 10..60 %), odd pairs unrelated."""
    rng = rng_for(seed, i)
    la, lb = loguniform_len(rng, 100, 10_000), loguniform_len(rng, 100, 10_000)
    if i % 2 == 0:
        return protein_pair(int(rng.integers(1 << 62)), la, lb, float(rng.uniform(0.1, 0.6)))
    al = np.frombuffer(AMINO, dtype=np.uint8)
    return Pair(al[rng.integers(0, al.size, size=la)], al[rng.integers(0, al.size, size=lb)], [], False, "protein")


def protein_batch(n: int = N_PROTEIN, seed: int = SEED_PROTEIN) -> list:
    return [protein_batch_pair(i, seed) for i in range(n)]

