"""Thin ctypes binding of libswmi.so (declared in include/swmi.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch is used for device memory (workspaces and
device-resident sequences) and for the current HIP stream.  If the library has
not been built, importing this module raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from collections.abc import Sequence
from dataclasses import dataclass

import numpy as np
# torch first: libswmi.so and torch share the HIP runtime library
# (libamdhip64.so.7), and the process must bind to torch's copy so that torch
# streams and allocations are valid inside the library.
import torch  # noqa: F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libswmi.so")

SW_OK, SW_EINVAL, SW_ENOMEM, SW_EDEVICE, SW_EUNSUPPORTED, SW_EINTERNAL = 0, -1, -2, -3, -4, -5
PRUNE_NONE, PRUNE_BEST, PRUNE_LEARNED = 0, 1, 2
TUNE_PAIR_SMALL, TUNE_PAIR_LARGE, TUNE_PAIR_HUGE, TUNE_BATCH = 0, 1, 2, 3
FLAG_GRAPH = 1  # SW_FLAG_GRAPH
FLAG_HALVES = 2  # SW_FLAG_HALVES
FLAG_BOTH_STRANDS = 4  # SW_FLAG_BOTH_STRANDS
SPLIT_NONE, SPLIT_LOWER, SPLIT_UPPER, SPLIT_MIDDLE = 0, 1, 2, 3
DEFAULT_SCORING = (1, 3, 5, 2)


class SwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"swmi status {status}: {msg}")
        self.status = status


class Matrix(ctypes.Structure):
    _fields_ = [("alphabet", ctypes.c_char_p), ("scores", ctypes.c_void_p),
                ("size", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Scoring(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32),
                ("matrix", ctypes.POINTER(Matrix))]


class MatrixScoring:
    """Substitution-matrix scoring (protein alignment): s(x, y) = scores[i][j] for
    x = alphabet[i] in A and y = alphabet[j] in B (letters case-insensitive), gaps as
    in the (match, mismatch, open, extend) form.  Pass it wherever a scoring tuple goes."""

    def __init__(self, alphabet: bytes, scores, gap_open: int, gap_extend: int):
        self.alphabet = bytes(alphabet)
        self.scores = np.ascontiguousarray(scores, dtype=np.int8)
        k = len(self.alphabet)
        if self.scores.shape != (k, k):  # the library reads size x size bytes
            raise ValueError(f"scores must be {k} x {k} for a {k}-letter alphabet, got {self.scores.shape}")
        self.gap_open, self.gap_extend = int(gap_open), int(gap_extend)

    def struct(self) -> Scoring:
        m = Matrix(self.alphabet, self.scores.ctypes.data, len(self.alphabet), 0)
        sc = Scoring(0, 0, self.gap_open, self.gap_extend, ctypes.pointer(m))
        sc._keep = (m, self.scores)  # the matrix stays alive while the struct does
        return sc


def _scoring(scoring):
    """ctypes reference to an sw_scoring for a (match, mismatch, open, extend) tuple or a
    MatrixScoring; the object returned keeps everything it points to alive."""
    sc = scoring.struct() if isinstance(scoring, MatrixScoring) else Scoring(*scoring)
    return ctypes.byref(sc)


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64)


class Options(ctypes.Structure):
    _fields_ = [("prune_mode", ctypes.c_int32), ("threshold", ctypes.c_int32),
                ("model", ctypes.c_void_p), ("rows_per_lane", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("band_width", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("slab_rows", ctypes.c_int32),
                ("progress", PROGRESS_FN), ("progress_user", ctypes.c_void_p),
                ("pair_thresholds", ctypes.POINTER(ctypes.c_int32))]


class ScoreResult(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("threshold", ctypes.c_int32),
                ("end_a", ctypes.c_int64), ("end_b", ctypes.c_int64),
                ("cells_computed", ctypes.c_int64), ("fallback", ctypes.c_int32),
                ("split_case", ctypes.c_int32), ("strand", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class AlignResult(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("strand", ctypes.c_int32),
                ("start_a", ctypes.c_int64), ("start_b", ctypes.c_int64),
                ("end_a", ctypes.c_int64), ("end_b", ctypes.c_int64),
                ("cigar", ctypes.c_void_p), ("cigar_len", ctypes.c_int64)]


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run `python -m paper_1304_5966_amd.build`")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.sw_last_error.restype = ctypes.c_char_p
    L.sw_version.restype = ctypes.c_char_p
    L.sw_context_create.argtypes = [ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.sw_context_destroy.argtypes = [vp]
    L.sw_context_set_tuning.argtypes = [vp, i32, i32, i32]
    L.sw_context_set_max_workspace.argtypes = [vp, ctypes.c_size_t]
    L.sw_context_set_band_width.argtypes = [vp, i32, i32]
    L.sw_context_get_band_width.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.sw_context_get_tuning.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.sw_score.argtypes = [vp, ctypes.c_char_p, i64, ctypes.c_char_p, i64, ctypes.POINTER(Scoring),
                           ctypes.POINTER(Options), ctypes.POINTER(ScoreResult)]
    L.sw_score_workspace_size.argtypes = [vp, i64, i64, ctypes.POINTER(Options)]
    L.sw_score_workspace_size.restype = ctypes.c_size_t
    L.sw_score_dev.argtypes = [vp, vp, i64, vp, i64, ctypes.POINTER(Scoring), ctypes.POINTER(Options),
                               vp, ctypes.c_size_t, ctypes.POINTER(ScoreResult)]
    L.sw_score_dev_noalloc.argtypes = [vp, vp, i64, vp, i64, ctypes.POINTER(Scoring), ctypes.POINTER(Options),
                                       ctypes.POINTER(ScoreResult)]
    L.sw_align.argtypes = [vp, ctypes.c_char_p, i64, ctypes.c_char_p, i64, ctypes.POINTER(Scoring),
                           ctypes.POINTER(Options), ctypes.POINTER(AlignResult)]
    L.sw_align_result_free.argtypes = [ctypes.POINTER(AlignResult)]
    L.sw_align_result_free.restype = None
    L.sw_start.argtypes = [vp, ctypes.c_char_p, i64, ctypes.c_char_p, i64, ctypes.POINTER(Scoring), i32,
                           i64, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.sw_batch.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i64), ctypes.c_char_p,
                           ctypes.POINTER(i64), i32, ctypes.POINTER(Scoring), ctypes.POINTER(Options),
                           ctypes.POINTER(ScoreResult)]
    L.sw_batch_workspace_size.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), i32,
                                          ctypes.POINTER(Scoring), ctypes.POINTER(Options)]
    L.sw_batch_workspace_size.restype = ctypes.c_size_t
    L.sw_batch_dev.argtypes = [vp, vp, ctypes.POINTER(i64), vp, ctypes.POINTER(i64), i32,
                               ctypes.POINTER(Scoring), ctypes.POINTER(Options), vp, ctypes.c_size_t,
                               ctypes.POINTER(ScoreResult)]
    L.sw_mm_host.argtypes = [ctypes.c_char_p, i64, ctypes.c_char_p, i64, ctypes.POINTER(Scoring), i32, i32,
                             i32, i64, ctypes.c_char_p, i64, ctypes.POINTER(i64)]
    L.sw_model_load.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(vp)]
    L.sw_model_free.argtypes = [vp]
    L.sw_mlp_param_count.restype = i64
    L.sw_features_workspace_size.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), i32]
    L.sw_features_workspace_size.restype = ctypes.c_size_t
    L.sw_features_dev.argtypes = [vp, vp, ctypes.POINTER(i64), vp, ctypes.POINTER(i64), i32, vp, vp,
                                  ctypes.c_size_t]
    L.sw_mlp_standardize_dev.argtypes = [vp, vp, i32, vp, vp, vp]
    L.sw_mlp_forward_dev.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp]
    L.sw_mlp_backward_dev.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, ctypes.c_float, vp, vp]
    L.sw_mlp_adam_dev.argtypes = [vp, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, vp]
    for name in ("sw_context_create", "sw_context_destroy", "sw_context_set_tuning",
                 "sw_context_get_tuning", "sw_score", "sw_score_dev", "sw_score_dev_noalloc", "sw_align",
                 "sw_start", "sw_batch", "sw_batch_dev", "sw_mm_host", "sw_model_load", "sw_model_free",
                 "sw_features_dev", "sw_mlp_standardize_dev", "sw_mlp_forward_dev", "sw_mlp_backward_dev",
                 "sw_mlp_adam_dev"):
        getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()

EXPORTED = ("sw_last_error", "sw_version", "sw_context_create", "sw_context_destroy",
            "sw_context_set_tuning", "sw_context_get_tuning", "sw_score",
            "sw_score_workspace_size", "sw_score_dev", "sw_score_dev_noalloc", "sw_align",
            "sw_align_result_free", "sw_start",
            "sw_batch", "sw_batch_workspace_size", "sw_batch_dev", "sw_mm_host", "sw_model_load",
            "sw_model_free", "sw_mlp_param_count", "sw_features_workspace_size", "sw_features_dev",
            "sw_mlp_standardize_dev", "sw_mlp_forward_dev", "sw_mlp_backward_dev", "sw_mlp_adam_dev")


def _check(status: int):
    if status != SW_OK:
        raise SwError(status, lib.sw_last_error().decode(errors="replace"))


def _bytes(x) -> bytes:
    if isinstance(x, bytes):
        return x
    if isinstance(x, str):
        return x.encode()
    return np.ascontiguousarray(x, dtype=np.uint8).tobytes()


def _options(prune=PRUNE_NONE, threshold=0, rows_per_lane=0, waves_per_cu=0, band_width=0,
             model=None, graph=False, slab_rows=0, progress=None, halves=False, both_strands=False,
             pair_thresholds=None) -> Options:
    """progress: optional callable(rows_done, rows_total), called after each row slab.
    pair_thresholds: batch calls in PRUNE_LEARNED mode, one threshold per pair."""
    op = Options(int(prune), int(threshold), model, int(rows_per_lane), int(waves_per_cu),
                 int(band_width), (FLAG_GRAPH if graph else 0) | (FLAG_HALVES if halves else 0)
                 | (FLAG_BOTH_STRANDS if both_strands else 0), int(slab_rows))
    if progress is not None:
        op.progress = PROGRESS_FN(lambda _user, done, total: progress(int(done), int(total)))
    if pair_thresholds is not None:
        arr = np.ascontiguousarray(pair_thresholds, dtype=np.int32)
        op._pair_thresholds = arr  # keeps the array alive as long as the options
        op.pair_thresholds = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    return op


@dataclass
class Score:
    score: int
    end_a: int
    end_b: int
    cells_computed: int = 0
    threshold: int = 0
    fallback: int = 0
    split_case: int = 0
    strand: int = 0

    def key(self):
        return (self.score, self.end_a, self.end_b)


@dataclass
class Alignment:
    score: int
    start_a: int
    start_b: int
    end_a: int
    end_b: int
    cigar: str
    strand: int = 0


def _score_of(r: ScoreResult) -> Score:
    return Score(r.score, r.end_a, r.end_b, r.cells_computed, r.threshold, r.fallback, r.split_case, r.strand)


_SCORE_DTYPE = np.dtype([("score", "<i4"), ("threshold", "<i4"), ("end_a", "<i8"), ("end_b", "<i8"),
                         ("cells_computed", "<i8"), ("fallback", "<i4"), ("split_case", "<i4"),
                         ("strand", "<i4"), ("reserved", "<i4")])
assert _SCORE_DTYPE.itemsize == ctypes.sizeof(ScoreResult)


class BatchResults(Sequence):
    """Per-pair results of a batch call: a numpy view of the library's result
    array (``.array``), turned into Score objects on access."""

    def __init__(self, raw, n: int):
        self._raw = raw  # keeps the ctypes buffer alive
        self.array = np.frombuffer(raw, dtype=_SCORE_DTYPE, count=n) if n else np.zeros(0, _SCORE_DTYPE)

    def __len__(self):
        return len(self.array)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[j] for j in range(*i.indices(len(self)))]
        r = self.array[i]
        return Score(int(r["score"]), int(r["end_a"]), int(r["end_b"]), int(r["cells_computed"]),
                     int(r["threshold"]), int(r["fallback"]), int(r["split_case"]), int(r["strand"]))

    def __eq__(self, other):
        return list(self) == list(other)

    def keys(self):
        """(score, end_a, end_b) per pair."""
        a = self.array
        return list(zip(a["score"].tolist(), a["end_a"].tolist(), a["end_b"].tolist()))


class Context:
    """A library context on one device, bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.sw_context_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.device = device
        self._ws = None

    def close(self):
        if self.handle:
            lib.sw_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_max_workspace(self, nbytes: int):
        """Cap on the device memory of the host-pointer calls (0: none)."""
        _check(lib.sw_context_set_max_workspace(self.handle, int(nbytes)))

    def set_tuning(self, tune_class: int, rows_per_lane: int, waves_per_cu: int):
        _check(lib.sw_context_set_tuning(self.handle, int(tune_class), int(rows_per_lane), int(waves_per_cu)))

    def set_band_width(self, tune_class: int, band_width: int):
        _check(lib.sw_context_set_band_width(self.handle, int(tune_class), int(band_width)))

    def get_band_width(self, tune_class: int) -> int:
        w = ctypes.c_int32()
        _check(lib.sw_context_get_band_width(self.handle, int(tune_class), ctypes.byref(w)))
        return w.value

    def get_tuning(self, tune_class: int):
        R, w = ctypes.c_int32(), ctypes.c_int32()
        _check(lib.sw_context_get_tuning(self.handle, int(tune_class), ctypes.byref(R), ctypes.byref(w)))
        return R.value, w.value

    # -- host-pointer entry points
    def score(self, a, b, scoring=DEFAULT_SCORING, **opts) -> Score:
        a, b = _bytes(a), _bytes(b)
        r = ScoreResult()
        _check(lib.sw_score(self.handle, a, len(a), b, len(b), _scoring(scoring),
                            ctypes.byref(_options(**opts)), ctypes.byref(r)))
        return _score_of(r)

    def align(self, a, b, scoring=DEFAULT_SCORING, **opts) -> Alignment:
        a, b = _bytes(a), _bytes(b)
        r = AlignResult()
        _check(lib.sw_align(self.handle, a, len(a), b, len(b), _scoring(scoring),
                            ctypes.byref(_options(**opts)), ctypes.byref(r)))
        try:
            cig = ctypes.string_at(r.cigar, r.cigar_len).decode() if r.cigar else ""
            return Alignment(r.score, r.start_a, r.start_b, r.end_a, r.end_b, cig, r.strand)
        finally:
            lib.sw_align_result_free(ctypes.byref(r))

    def start(self, a, b, score, end_a, end_b, scoring=DEFAULT_SCORING):
        a, b = _bytes(a), _bytes(b)
        sa, sb = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.sw_start(self.handle, a, len(a), b, len(b), _scoring(scoring),
                            int(score), int(end_a), int(end_b), ctypes.byref(sa), ctypes.byref(sb)))
        return sa.value, sb.value

    def batch(self, pairs, scoring=DEFAULT_SCORING, **opts):
        a_parts = [_bytes(p[0]) for p in pairs]
        b_parts = [_bytes(p[1]) for p in pairs]
        offs_a = np.zeros(len(pairs) + 1, dtype=np.int64)
        offs_b = np.zeros(len(pairs) + 1, dtype=np.int64)
        offs_a[1:] = np.cumsum([len(x) for x in a_parts])
        offs_b[1:] = np.cumsum([len(x) for x in b_parts])
        return self.batch_packed(b"".join(a_parts), offs_a, b"".join(b_parts), offs_b, scoring, **opts)

    def batch_packed(self, seqs_a, offs_a, seqs_b, offs_b, scoring=DEFAULT_SCORING, **opts):
        offs_a = np.ascontiguousarray(offs_a, dtype=np.int64)
        offs_b = np.ascontiguousarray(offs_b, dtype=np.int64)
        n = len(offs_a) - 1
        out = (ScoreResult * max(n, 1))()
        i64p = ctypes.POINTER(ctypes.c_int64)
        _check(lib.sw_batch(self.handle, _bytes(seqs_a), offs_a.ctypes.data_as(i64p), _bytes(seqs_b),
                            offs_b.ctypes.data_as(i64p), n, _scoring(scoring),
                            ctypes.byref(_options(**opts)), out))
        return BatchResults(out, n)

    def batch_dev(self, d_seqs_a, offs_a, d_seqs_b, offs_b, scoring=DEFAULT_SCORING, workspace=None,
                  **opts):
        """d_seqs_*: uint8 CUDA tensors of packed letters; offs_*: host int64 offsets (n + 1)."""
        offs_a = np.ascontiguousarray(offs_a, dtype=np.int64)
        offs_b = np.ascontiguousarray(offs_b, dtype=np.int64)
        n = len(offs_a) - 1
        i64p = ctypes.POINTER(ctypes.c_int64)
        sc = scoring.struct() if isinstance(scoring, MatrixScoring) else Scoring(*scoring)
        op = _options(**opts)
        if workspace is None:  # the library checks a caller's workspace itself
            workspace = self.workspace(int(lib.sw_batch_workspace_size(
                self.handle, offs_a.ctypes.data_as(i64p), offs_b.ctypes.data_as(i64p), n, ctypes.byref(sc),
                ctypes.byref(op))))
        ws = workspace
        out = (ScoreResult * max(n, 1))()
        _check(lib.sw_batch_dev(self.handle, ctypes.c_void_p(d_seqs_a.data_ptr()),
                                offs_a.ctypes.data_as(i64p), ctypes.c_void_p(d_seqs_b.data_ptr()),
                                offs_b.ctypes.data_as(i64p), n, ctypes.byref(sc), ctypes.byref(op),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), out))
        return BatchResults(out, n)

    def batch_workspace_size(self, offs_a, offs_b, scoring=DEFAULT_SCORING, **opts) -> int:
        offs_a = np.ascontiguousarray(offs_a, dtype=np.int64)
        offs_b = np.ascontiguousarray(offs_b, dtype=np.int64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        return int(lib.sw_batch_workspace_size(self.handle, offs_a.ctypes.data_as(i64p),
                                               offs_b.ctypes.data_as(i64p), len(offs_a) - 1,
                                               _scoring(scoring),
                                               ctypes.byref(_options(**opts))))

    # -- device-pointer entry point (torch-owned buffers, no allocation in the library)
    def workspace_size(self, len_a: int, len_b: int, **opts) -> int:
        return int(lib.sw_score_workspace_size(self.handle, len_a, len_b, ctypes.byref(_options(**opts))))

    def workspace(self, nbytes: int):
        torch = self._torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def score_dev(self, d_a, d_b, scoring=DEFAULT_SCORING, workspace=None, **opts) -> Score:
        """d_a, d_b: uint8 CUDA tensors of letters on this context's device."""
        la, lb = int(d_a.numel()), int(d_b.numel())
        need = self.workspace_size(la, lb, **opts)
        ws = workspace if workspace is not None else self.workspace(need)
        r = ScoreResult()
        _check(lib.sw_score_dev(self.handle, ctypes.c_void_p(d_a.data_ptr()), la,
                                ctypes.c_void_p(d_b.data_ptr()), lb, _scoring(scoring),
                                ctypes.byref(_options(**opts)), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel(), ctypes.byref(r)))
        return _score_of(r)


    def score_dev_noalloc(self, d_a, d_b, scoring=DEFAULT_SCORING, **opts) -> Score:
        """score_dev with the library's fixed scratch as workspace (no allocation anywhere)."""
        r = ScoreResult()
        _check(lib.sw_score_dev_noalloc(self.handle, ctypes.c_void_p(d_a.data_ptr()), int(d_a.numel()),
                                        ctypes.c_void_p(d_b.data_ptr()), int(d_b.numel()),
                                        _scoring(scoring), ctypes.byref(_options(**opts)),
                                        ctypes.byref(r)))
        return _score_of(r)


NOALLOC_SCRATCH_BYTES = 256 << 20  # SW_NOALLOC_SCRATCH_BYTES


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Model:
    """A threshold model file loaded for SW_PRUNE_LEARNED (pass ``model=m.handle``)."""

    def __init__(self, ctx: "Context", path: str):
        h = ctypes.c_void_p()
        _check(lib.sw_model_load(ctx.handle, path.encode(), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib.sw_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def param_count() -> int:
    return int(lib.sw_mlp_param_count())


def features_dev(ctx: "Context", d_a, offs_a, d_b, offs_b, out=None):
    """Features [n, 256] (float32 CUDA tensor) of packed device letters with host offsets."""
    torch = ctx._torch
    offs_a = np.ascontiguousarray(offs_a, dtype=np.int64)
    offs_b = np.ascontiguousarray(offs_b, dtype=np.int64)
    n = len(offs_a) - 1
    i64p = ctypes.POINTER(ctypes.c_int64)
    need = int(lib.sw_features_workspace_size(ctx.handle, offs_a.ctypes.data_as(i64p),
                                              offs_b.ctypes.data_as(i64p), n))
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=d_a.device)
    if out is None:
        out = torch.empty((n, 256), dtype=torch.float32, device=d_a.device)
    _check(lib.sw_features_dev(ctx.handle, _ptr(d_a), offs_a.ctypes.data_as(i64p), _ptr(d_b),
                               offs_b.ctypes.data_as(i64p), n, _ptr(out), _ptr(ws), ws.numel()))
    return out


def mlp_standardize(ctx, d_feat, d_mean, d_inv_std):
    torch = ctx._torch
    n = d_feat.shape[0]
    x = torch.empty((n, 256), dtype=torch.int16, device=d_feat.device)
    _check(lib.sw_mlp_standardize_dev(ctx.handle, _ptr(d_feat), n, _ptr(d_mean), _ptr(d_inv_std), _ptr(x)))
    return x


def mlp_forward(ctx, d_x, d_wbf, d_params):
    """d_x: int16 [n, 256] holding BF16 bits; returns (y [n], h1 [n,128], h2 [n,128]) float32."""
    torch = ctx._torch
    n = d_x.shape[0]
    h1 = torch.empty((n, 128), dtype=torch.float32, device=d_x.device)
    h2 = torch.empty((n, 128), dtype=torch.float32, device=d_x.device)
    y = torch.empty(n, dtype=torch.float32, device=d_x.device)
    _check(lib.sw_mlp_forward_dev(ctx.handle, _ptr(d_x), n, _ptr(d_wbf), _ptr(d_params), _ptr(h1), _ptr(h2),
                                  _ptr(y)))
    return y, h1, h2


def mlp_backward(ctx, d_x, d_wbf, h1, h2, y, target, quantile=0.0):
    torch = ctx._torch
    n = d_x.shape[0]
    scratch = torch.empty(64 + 257 * n, dtype=torch.float32, device=d_x.device)
    grad = torch.empty(param_count(), dtype=torch.float32, device=d_x.device)
    _check(lib.sw_mlp_backward_dev(ctx.handle, _ptr(d_x), n, _ptr(d_wbf), _ptr(h1), _ptr(h2), _ptr(y),
                                   _ptr(target), float(quantile), _ptr(scratch), _ptr(grad)))
    return grad


def mlp_adam(ctx, d_params, d_m, d_v, d_grad, step, lr, d_wbf, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib.sw_mlp_adam_dev(ctx.handle, _ptr(d_params), _ptr(d_m), _ptr(d_v), _ptr(d_grad), int(step),
                               float(lr), float(beta1), float(beta2), float(eps), _ptr(d_wbf)))


def mm_host(a, b, scoring=DEFAULT_SCORING, tb=-1, te=-1, score=None) -> str:
    """Host Myers-Miller of the whole of a x b (the reconstruction's CPU part)."""
    a, b = _bytes(a), _bytes(b)
    cap = 4 * (len(a) + len(b)) + 64
    buf = ctypes.create_string_buffer(cap)
    n = ctypes.c_int64()
    _check(lib.sw_mm_host(a, len(a), b, len(b), _scoring(scoring), tb, te,
                          0 if score is None else 1, 0 if score is None else int(score), buf, cap,
                          ctypes.byref(n)))
    return buf.value.decode()


def version() -> str:
    return lib.sw_version().decode()
