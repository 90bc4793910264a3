"""CPU oracle for exact affine-gap local alignment -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the GPU library
(``paper_1304_5966_amd``); the only common dependency is the seeded sequence
generator ``paper_1304_5966_amd.synth``, which holds no alignment arithmetic.

``gotoh.c`` holds the dynamic programs (see its header for the exact
recurrences, following the SW# paper, Section 2); this module loads it with
ctypes and adds CIGAR rescoring.  ``brute.py`` holds the pure-Python
enumerations that pin the C code.

Pins (tests/test_oracle_*.py): brute-force enumeration of every local
alignment of tiny inputs (score, endpoint, start point), a midline-filtered
enumeration of optimal global alignments (canonical CIGAR), closed forms
(self-alignment, a single substitution or gap in otherwise equal aperiodic
strings), textbook reductions (linear gaps, gapless Kadane maxima) and
invariants (swap, joint reversal, complement, alphabet permutation,
extension monotonicity), plus the planted-alignment lower bound at scale.
"""
from __future__ import annotations

import ctypes
import os
import re
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gotoh.c")
_LIB = os.path.join(_HERE, "_liboracle.so")

SCORING = (1, 3, 5, 2)  # match, mismatch penalty, gap open, gap extend (all configs)


class _Scoring(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32),
                ("matrix", ctypes.c_void_p), ("letter_class", ctypes.c_void_p),
                ("size", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class MatrixScoring:
    """Substitution-matrix scoring (protein alignment): s(x, y) = matrix[i][j] for the
    letters alphabet[i], alphabet[j] (case-insensitive); gaps as in the tuple form.

    Indexing like the tuple form: [0] the largest score, [2] gap open, [3] gap extend."""

    def __init__(self, alphabet: bytes, matrix, gap_open: int, gap_extend: int):
        self.alphabet = bytes(alphabet).upper()
        self.matrix = np.ascontiguousarray(matrix, dtype=np.int8)
        k = len(self.alphabet)
        if self.matrix.shape != (k, k) or len(set(self.alphabet)) != k:
            raise ValueError("matrix must be K x K for K distinct letters")
        self.letter_class = np.full(256, -1, dtype=np.int8)
        for i, c in enumerate(self.alphabet):
            self.letter_class[c] = i
            self.letter_class[ord(chr(c).lower())] = i
        self.gap_open, self.gap_extend = int(gap_open), int(gap_extend)

    def s(self, x: int, y: int) -> int:
        return int(self.matrix[self.letter_class[x], self.letter_class[y]])

    def __getitem__(self, i):
        return (int(self.matrix.max()), 0, self.gap_open, self.gap_extend)[i]


def build(force: bool = False) -> str:
    """Compile gotoh.c into _liboracle.so with the host C compiler."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-pthread", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u8p = ctypes.c_char_p
        sp = ctypes.POINTER(_Scoring)
        for name in ("orc_sw_full", "orc_sw_linear"):
            f = getattr(L, name)
            f.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, sp, i64p, i64p, i64p]
            f.restype = ctypes.c_int
        L.orc_sw_linear_mt.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, sp, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_int64, i64p, i64p, i64p]
        L.orc_sw_start_mt.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, sp, ctypes.c_int64,
                                      ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int64,
                                      ctypes.c_int64, i64p, i64p]
        L.orc_sw_matrix.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, sp, ctypes.c_void_p]
        L.orc_sw_start.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, sp, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_int64, i64p, i64p]
        L.orc_mm_align.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, sp, ctypes.c_int64,
                                   ctypes.c_int64, ctypes.c_char_p, ctypes.c_int64, i64p]
        L.orc_global_score.argtypes = [u8p, ctypes.c_int64, u8p, ctypes.c_int64, sp,
                                       ctypes.c_int64, ctypes.c_int64, i64p]
        _lib = L
    return _lib


def _bytes(x) -> bytes:
    if isinstance(x, bytes):
        return x
    if isinstance(x, str):
        return x.encode()
    return np.ascontiguousarray(x, dtype=np.uint8).tobytes()


def _sc(scoring) -> _Scoring:
    if isinstance(scoring, MatrixScoring):
        sc = _Scoring(max(1, int(scoring.matrix.max())), 0, scoring.gap_open, scoring.gap_extend,
                      scoring.matrix.ctypes.data, scoring.letter_class.ctypes.data, len(scoring.alphabet), 0)
        sc._keep = scoring  # the arrays must outlive the call
        return sc
    return _Scoring(*[int(v) for v in scoring], None, None, 0, 0)


def sw_score(a, b, scoring=SCORING, full: bool = False):
    """(S, end_a, end_b); end = lexicographically smallest cell holding S, 0-based; -1 if S = 0."""
    a, b = _bytes(a), _bytes(b)
    s, ea, eb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    f = lib().orc_sw_full if full else lib().orc_sw_linear
    rc = f(a, len(a), b, len(b), ctypes.byref(_sc(scoring)), ctypes.byref(s), ctypes.byref(ea),
           ctypes.byref(eb))
    if rc:
        raise ValueError("oracle: invalid arguments")
    return int(s.value), int(ea.value), int(eb.value)


def host_cores() -> int:
    """Threads the multi-threaded modes use by default: the CPUs this process may run on,
    at most 16 (the host share of one GPU on the benchmark machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def sw_score_mt(a, b, scoring=SCORING, threads: int = 0, stripe_rows: int = 0, chunk_cols: int = 0):
    """sw_score in linear space over row stripes on several threads (same result)."""
    a, b = _bytes(a), _bytes(b)
    s, ea, eb = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    rc = lib().orc_sw_linear_mt(a, len(a), b, len(b), ctypes.byref(_sc(scoring)), threads or host_cores(),
                                stripe_rows, chunk_cols, ctypes.byref(s), ctypes.byref(ea), ctypes.byref(eb))
    if rc:
        raise ValueError("oracle: invalid arguments or out of memory")
    return int(s.value), int(ea.value), int(eb.value)


def sw_start_mt(a, b, score, end_a, end_b, scoring=SCORING, threads: int = 0, stripe_rows: int = 0,
                chunk_cols: int = 0):
    """sw_start over row stripes on several threads (same result)."""
    a, b = _bytes(a), _bytes(b)
    sa, sb = ctypes.c_int64(), ctypes.c_int64()
    if lib().orc_sw_start_mt(a, len(a), b, len(b), ctypes.byref(_sc(scoring)), score, end_a, end_b,
                             threads or host_cores(), stripe_rows, chunk_cols, ctypes.byref(sa),
                             ctypes.byref(sb)):
        raise ValueError("oracle: start not found / invalid arguments")
    return int(sa.value), int(sb.value)


def sw_matrix(a, b, scoring=SCORING) -> np.ndarray:
    a, b = _bytes(a), _bytes(b)
    H = np.zeros((len(a) + 1, len(b) + 1), dtype=np.int64)
    if lib().orc_sw_matrix(a, len(a), b, len(b), ctypes.byref(_sc(scoring)), H.ctypes.data):
        raise ValueError("oracle: invalid arguments")
    return H


def sw_start(a, b, score, end_a, end_b, scoring=SCORING):
    a, b = _bytes(a), _bytes(b)
    sa, sb = ctypes.c_int64(), ctypes.c_int64()
    if lib().orc_sw_start(a, len(a), b, len(b), ctypes.byref(_sc(scoring)), score, end_a, end_b,
                          ctypes.byref(sa), ctypes.byref(sb)):
        raise ValueError("oracle: start not found / invalid arguments")
    return int(sa.value), int(sb.value)


def mm_align(a, b, scoring=SCORING, tb: int = -1, te: int = -1) -> str:
    """Canonical Myers-Miller CIGAR of the global alignment of a x b (tb/te default: g)."""
    a, b = _bytes(a), _bytes(b)
    cap = 4 * (len(a) + len(b)) + 64
    buf = ctypes.create_string_buffer(cap)
    n = ctypes.c_int64()
    rc = lib().orc_mm_align(a, len(a), b, len(b), ctypes.byref(_sc(scoring)), tb, te, buf, cap,
                            ctypes.byref(n))
    if rc:
        raise ValueError("oracle: mm_align failed")
    return buf.value.decode()


def global_score(a, b, scoring=SCORING, tb: int = -1, te: int = -1) -> int:
    a, b = _bytes(a), _bytes(b)
    g = scoring[2] - scoring[3]  # gap open minus extend
    out = ctypes.c_int64()
    if lib().orc_global_score(a, len(a), b, len(b), ctypes.byref(_sc(scoring)),
                              g if tb < 0 else tb, g if te < 0 else te, ctypes.byref(out)):
        raise ValueError("oracle: invalid arguments")
    return int(out.value)


@dataclass
class Alignment:
    score: int
    start_a: int
    start_b: int
    end_a: int
    end_b: int
    cigar: str


def sw_align(a, b, scoring=SCORING) -> Alignment:
    """Score, endpoint, start point and canonical CIGAR (empty alignment when S = 0)."""
    a, b = _bytes(a), _bytes(b)
    s, ea, eb = sw_score(a, b, scoring)
    if s <= 0:
        return Alignment(0, -1, -1, -1, -1, "")
    sa, sb = sw_start(a, b, s, ea, eb, scoring)
    cig = mm_align(a[sa:ea + 1], b[sb:eb + 1], scoring)
    return Alignment(s, sa, sb, ea, eb, cig)


_CIG = re.compile(r"(\d+)([=XID])")


def parse_cigar(cigar: str):
    ops = _CIG.findall(cigar)
    if "".join(n + o for n, o in ops) != cigar:
        raise ValueError(f"malformed CIGAR {cigar!r}")
    return [(int(n), o) for n, o in ops]


def rescore(a, b, start_a, start_b, cigar: str, scoring=SCORING):
    """Score of a CIGAR placed at (start_a, start_b); checks '='/'X' against the letters.

    Returns (score, end_a, end_b).  Each maximal I or D run costs open + extend*(k-1).
    """
    a, b = _bytes(a).upper(), _bytes(b).upper()
    if isinstance(scoring, MatrixScoring):
        subst = scoring.s
        go, ge = scoring.gap_open, scoring.gap_extend
    else:
        match, mismatch, go, ge = scoring

        def subst(x, y):
            return match if x == y else -mismatch
    i, j, s = start_a, start_b, 0
    prev = None
    for n, o in parse_cigar(cigar):
        if o in "=X":
            for _ in range(n):
                eq = a[i] == b[j]
                if eq != (o == "="):
                    raise ValueError(f"CIGAR op {o} disagrees with letters at ({i},{j})")
                s += subst(a[i], b[j])
                i += 1
                j += 1
        else:
            if o == prev:
                raise ValueError("adjacent runs of the same gap op")
            s -= go + ge * (n - 1)
            if o == "I":
                j += n
            else:
                i += n
        prev = o
    return s, i - 1, j - 1
