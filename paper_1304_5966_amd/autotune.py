"""Tile-shape autotuner for the wavefront engine.

The engine's shape has two knobs: rows per lane R (a stripe is 64*R rows) and
resident stripe waves per CU; long pairs add a third, the column band width.  More waves hide latency but lengthen the
stripe pipeline's fill; larger R cuts the per-cell lane-exchange cost but
needs more registers.  The best pair depends on the workload, so the tuner
times each candidate on the caller's own data (through the C ABI; every
candidate runs the real kernels), installs the winner in the context for the
workload's class (``sw_context_set_tuning``: later calls that leave the shape
at 0 use it) and caches it per (architecture, CU count, class) in a JSON file.

    from paper_1304_5966_amd import autotune
    autotune.tune_score(ctx, d_a, d_b)          # one long pair
    autotune.tune_batch(ctx, d_a, oa, d_b, ob)  # many pairs
    ctx.score_dev(d_a, d_b)                     # runs with the tuned shape
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import swmi

# (rows per lane, waves per CU).  R = 8 and R = 6 run a 256-VGPR build up to 8 waves per CU
# and a 168-VGPR build (3 waves per SIMD) above; R = 4 a 128-VGPR build (up to 16 per CU).
CANDIDATES = [(4, 8), (4, 12), (4, 16), (6, 12), (6, 16), (8, 4), (8, 6), (8, 8), (8, 10), (8, 12)]
CACHE = os.environ.get("SWMI_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "swmi", "autotune.json"))


def _device_key(ctx) -> str:
    torch = ctx._torch
    p = torch.cuda.get_device_properties(ctx.device)
    return f"{getattr(p, 'gcnArchName', 'gfx')}:{p.multi_processor_count}"


CLASS_NAMES = {swmi.TUNE_PAIR_SMALL: "pair-small", swmi.TUNE_PAIR_LARGE: "pair-large",
               swmi.TUNE_PAIR_HUGE: "pair-huge", swmi.TUNE_BATCH: "batch"}


def workload_class(cells: float, n_pairs: int) -> int:
    """The library's class of a launch (sw_tune_class): by mean cells per pair."""
    per = cells / max(n_pairs, 1)
    if per >= 1e12:
        return swmi.TUNE_PAIR_HUGE
    if per >= 1e10:
        return swmi.TUNE_PAIR_LARGE
    return swmi.TUNE_BATCH if n_pairs > 1 else swmi.TUNE_PAIR_SMALL


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key, value):
    data = _load()
    data[key] = value
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    except OSError:
        pass


def _key(ctx, cls: int) -> str:
    return f"{_device_key(ctx)}:{CLASS_NAMES[cls]}"


def cached(ctx, cls: int):
    v = _load().get(_key(ctx, cls))
    if v is None:
        return None
    out = {"rows_per_lane": v["rows_per_lane"], "waves_per_cu": v["waves_per_cu"]}
    if "band_width" in v:
        out["band_width"] = v["band_width"]
    return out


def _install(ctx, cls: int, best: dict) -> dict:
    ctx.set_tuning(cls, best["rows_per_lane"], best["waves_per_cu"])
    if "band_width" in best:
        ctx.set_band_width(cls, best["band_width"])
    return best


def band_candidates(n_cols: int, grid: int, max_slot_bytes: float = 96 * 2**30) -> list:
    """Column band widths to try for a pair of n_cols columns: the automatic width (0) and
    the widths that cut the columns into 1, 3 and 4 equal bands, while the hand-off slots
    (about one row of 8-byte entries per resident wave) stay within max_slot_bytes."""
    out = [0]
    for k in (1, 3, 4):
        w = -(-n_cols // k)
        w = -(-w // 64) * 64
        if (grid + 1) * (w + 192) * 8 <= max_slot_bytes and w not in out:
            out.append(w)
    return out


def _time(fn, reps, warm=True):
    torch = swmi.torch
    if warm:
        fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune_score(ctx, d_a, d_b, crop: int | None = None, reps: int = 1, use_cache: bool = True, log=None,
               table=None, candidates=None, tune_bands: bool = True) -> dict:
    """Best shape for one pair, timed on the pair (or its leading crop x crop); for pairs of
    10^10 cells and more, then the best column band width at that shape.

    ``table``, if a list, receives one dict per candidate (shape, seconds, GCUPS)."""
    la, lb = int(d_a.numel()), int(d_b.numel())
    cls = workload_class(float(la) * lb, 1)
    if use_cache and (hit := cached(ctx, cls)):
        return _install(ctx, cls, hit)
    a, b = (d_a, d_b) if crop is None else (d_a[:min(la, crop)], d_b[:min(lb, crop)])
    rows = []
    for R, w in candidates or CANDIDATES:
        opts = dict(rows_per_lane=R, waves_per_cu=w)
        ws = ctx.workspace(ctx.workspace_size(a.numel(), b.numel(), **opts))
        t = _time(lambda: ctx.score_dev(a, b, workspace=ws, **opts), reps, warm=a.numel() * b.numel() < 1e11)
        rows.append((t, R, w))
        if table is not None:
            table.append(dict(opts, s=round(t, 4), gcups=round(a.numel() * b.numel() / t / 1e9, 1)))
        if log:
            log(f"autotune {CLASS_NAMES[cls]} R={R} waves/CU={w}: {a.numel() * b.numel() / t / 1e9:.1f} GCUPS")
    t, R, w = min(rows)
    best = {"rows_per_lane": R, "waves_per_cu": w}
    if tune_bands and cls in (swmi.TUNE_PAIR_LARGE, swmi.TUNE_PAIR_HUGE):
        # then the column band width at that shape (wide bands keep the stripe pipeline full;
        # fewer, narrower bands take less slot memory)
        grid = swmi.torch.cuda.get_device_properties(ctx.device).multi_processor_count * w
        bands = []
        for bw in band_candidates(b.numel(), grid):
            opts = dict(rows_per_lane=R, waves_per_cu=w, band_width=bw)
            tb = t if bw == 0 else _time(lambda: ctx.score_dev(a, b, workspace=ctx.workspace(
                ctx.workspace_size(a.numel(), b.numel(), **opts)), **opts), reps, warm=a.numel() * b.numel() < 1e11)
            bands.append((tb, bw))
            if table is not None:
                table.append(dict(opts, s=round(tb, 4), gcups=round(a.numel() * b.numel() / tb / 1e9, 1)))
            if log:
                log(f"autotune {CLASS_NAMES[cls]} R={R} waves/CU={w} band {bw or 'auto'}: "
                    f"{a.numel() * b.numel() / tb / 1e9:.1f} GCUPS")
        t, bw = min(bands)
        best["band_width"] = bw
    _store(_key(ctx, cls), dict(best, gcups=a.numel() * b.numel() / t / 1e9,
                                 sample=f"{a.numel()}x{b.numel()}"))
    return _install(ctx, cls, best)


def tune_batch(ctx, d_a, offs_a, d_b, offs_b, reps: int = 1, use_cache: bool = True, log=None,
               table=None) -> dict:
    """Best shape for a batch, timed on the batch itself."""
    offs_a = np.asarray(offs_a, dtype=np.int64)
    offs_b = np.asarray(offs_b, dtype=np.int64)
    cells = float(np.sum(np.diff(offs_a) * np.diff(offs_b)))
    cls = workload_class(cells, len(offs_a) - 1)
    if use_cache and (hit := cached(ctx, cls)):
        return _install(ctx, cls, hit)
    rows = []
    for R, w in CANDIDATES:
        opts = dict(rows_per_lane=R, waves_per_cu=w)
        ws = ctx.workspace(ctx.batch_workspace_size(offs_a, offs_b, **opts))
        t = _time(lambda: ctx.batch_dev(d_a, offs_a, d_b, offs_b, workspace=ws, **opts), reps)
        rows.append((t, R, w))
        if table is not None:
            table.append(dict(opts, s=round(t, 4), gcups=round(cells / t / 1e9, 1)))
        if log:
            log(f"autotune {CLASS_NAMES[cls]} R={R} waves/CU={w}: {cells / t / 1e9:.1f} GCUPS")
    t, R, w = min(rows)
    best = {"rows_per_lane": R, "waves_per_cu": w}
    _store(_key(ctx, cls), dict(best, gcups=cells / t / 1e9, pairs=len(offs_a) - 1))
    return _install(ctx, cls, best)
