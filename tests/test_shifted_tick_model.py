"""CPU model of one row-and-column-shifted tick of the engine (R = 4 and 8 rows per lane).

The engine's fast ticks keep every value of cell (stripe row r, tick column t) plus
(r + t) * gap_extend, so that E and F each take one maximum per cell; the local
zeros and the running maximum live in register windows indexed by anti-diagonal.
This test runs the same steps on the host for a 64-lane wave (numpy over lanes):
entry conversion, lane exchange, the per-cell updates, the windows, the exit
conversion, lane 63's outputs and the tick's maximum, and checks every result
against the plain affine-gap recurrence of the same cells (Gotoh, paper section 2),
written out cell by cell.
"""
import numpy as np
import pytest

LANES = 64
STEPS = 64
NEG = -(1 << 30)


def plain_region(rng, R, local, match, mismatch, gopen, ext):
    """Plain recurrence over stripe rows 0..64R-1 and columns -70..63, from random
    borders: H of row -1, the F entering row 0, and H/E of column -71."""
    rows, c0, c1 = LANES * R, -70, STEPS
    ncol = c1 - c0
    a = rng.integers(0, 4, rows)
    b = rng.integers(0, 4, ncol)
    hi = 40 if local else 400
    lo = 0 if local else -400
    top = rng.integers(lo, hi, ncol + 1)  # H(-1, c) for c = c0-1 .. c1-1
    fin = rng.integers(lo - 50, hi - 20, ncol)  # F entering row 0 at column c
    left_h = rng.integers(lo, hi, rows)
    left_e = np.minimum(left_h - gopen, rng.integers(lo - 50, hi - 20, rows))
    if local:
        left_e = np.maximum(left_e, 0)
    H = np.zeros((rows, ncol), np.int64)
    E = np.zeros((rows, ncol), np.int64)
    F = np.zeros((rows, ncol), np.int64)   # F entering row r at column c
    Fo = np.zeros(ncol, np.int64)          # F entering row 64R (leaves the stripe)
    for r in range(rows):
        for j in range(ncol):
            hl, el = (left_h[r], left_e[r]) if j == 0 else (H[r, j - 1], E[r, j - 1])
            e = max(el - ext, hl - gopen)
            if local:
                e = max(e, 0)
            f = fin[j] if r == 0 else max(F[r - 1, j] - ext, H[r - 1, j] - gopen)
            diag = top[j] if r == 0 else (left_h[r - 1] if j == 0 else H[r - 1, j - 1])
            s = match if a[r] == b[j] else -mismatch
            H[r, j], E[r, j], F[r, j] = max(diag + s, e, f), e, f
    for j in range(ncol):
        Fo[j] = max(F[rows - 1, j] - ext, H[rows - 1, j] - gopen)
    return dict(a=a, b=b, top=top, fin=fin, H=H, E=E, F=F, Fo=Fo, c0=c0)


def shifted_tick(reg, R, local, match, mismatch, gopen, ext):
    """The engine's shifted tick, step by step, vectorised over the 64 lanes."""
    H, E, F, Fo, c0 = reg["H"], reg["E"], reg["F"], reg["Fo"], reg["c0"]
    a, b, top, fin = reg["a"], reg["b"], reg["top"], reg["fin"]
    g = gopen - ext
    lane = np.arange(LANES)
    rbase = lane * R
    col = lambda c: c - c0  # column index into the region arrays

    # carried state at step -1: lane l sits at column -1 - l
    cprev = col(-1 - lane)
    sH = np.stack([H[rbase + k, cprev] for k in range(R)])
    sE = np.stack([E[rbase + k, cprev] for k in range(R)])
    # the diagonal of row 0 at step 0: H of the row above, one column left of step 0's column
    hup = np.where(lane == 0, top[col(-1 - lane) + 1], H[np.maximum(rbase - 1, 0), cprev])
    hl = sH[R - 1].copy()
    gl = np.where(rbase + R < LANES * R, F[np.minimum(rbase + R, LANES * R - 1), cprev], Fo[cprev])

    off = (rbase - lane - 1) * ext
    for k in range(R):
        sH[k] += off + k * ext
        sE[k] += off + k * ext
    HA = sH - g
    hup = hup + off - ext
    hl = hl + off + (R - 1) * ext
    gl = gl + off + R * ext
    zw = [(rbase - lane + j) * ext for j in range(R)]
    aw = [np.full(LANES, NEG, np.int64) for _ in range(R)]
    out = np.zeros((STEPS, 2), np.int64)
    # lane 0's inputs, shifted: H of stripe row -1 with -ext, F entering row 0
    in_x = np.array([top[col(m) + 1] for m in range(STEPS)]) + (np.arange(STEPS) - 1) * ext
    in_y = np.array([fin[col(m)] for m in range(STEPS)]) + np.arange(STEPS) * ext
    for m in range(STEPS):
        j0 = m % R
        upH = np.concatenate(([in_x[m]], hl[:-1]))
        upG = np.concatenate(([in_y[m]], gl[:-1]))
        diag, hup = hup, upH
        f = upG
        cc = m - lane
        for k in range(R):
            s2 = np.where(a[rbase + k] == b[col(cc)], match, -mismatch) + 2 * ext
            hd = diag + s2
            en = np.maximum(sE[k], HA[k])
            if local:
                en = np.maximum(en, zw[(j0 + k) % R])
            hn = np.maximum(np.maximum(hd, en), f)
            han = hn - g
            f = np.maximum(f, han)
            diag = sH[k].copy()
            sH[k], sE[k], HA[k] = hn, en, han
            aw[(j0 + k) % R] = np.maximum(aw[(j0 + k) % R], hn)
        if local:
            zw[j0] = zw[j0] + R * ext
        aw[j0] = aw[j0] + R * ext
        hl, gl = sH[R - 1].copy(), f
        out[m] = (hl[LANES - 1], gl[LANES - 1])
    back = (STEPS - 1 - lane) * ext
    for k in range(R):
        sH[k] -= back + (rbase + k) * ext
        sE[k] -= back + (rbase + k) * ext
    hup = hup - (back + (rbase - 1) * ext)
    hl = hl - (back + (rbase + R - 1) * ext)
    gl = gl - (back + (rbase + R) * ext)
    tmax = np.max(np.stack([aw[j] - (rbase - lane + STEPS + j) * ext for j in range(R)]), axis=0).max()
    # lane 63's output of step m loses its column shift (m - 63) and its row shift
    m = np.arange(STEPS)
    out[:, 0] -= (m - (STEPS - 1) + (LANES * R - 1)) * ext
    out[:, 1] -= (m - (STEPS - 1) + LANES * R) * ext
    return sH, sE, hup, hl, gl, out, tmax


@pytest.mark.parametrize("R", [4, 8])
@pytest.mark.parametrize("local", [True, False])
@pytest.mark.parametrize("scoring", [(1, 3, 5, 2), (2, 3, 7, 1), (5, 4, 10, 3)])
def test_shifted_tick_equals_plain_recurrence(R, local, scoring):
    match, mismatch, gopen, ext = scoring
    rng = np.random.default_rng(1000 * R + 10 * local + match)
    reg = plain_region(rng, R, local, match, mismatch, gopen, ext)
    sH, sE, hup, hl, gl, out, tmax = shifted_tick(reg, R, local, match, mismatch, gopen, ext)
    H, E, F, Fo, c0 = reg["H"], reg["E"], reg["F"], reg["Fo"], reg["c0"]
    lane = np.arange(LANES)
    clast = STEPS - 1 - lane - c0  # lane l ends the tick at column 63 - l
    for k in range(R):
        r = lane * R + k
        assert np.array_equal(sH[k], H[r, clast]), k
        assert np.array_equal(sE[k], E[r, clast]), k
    rows = LANES * R
    assert np.array_equal(hl, H[lane * R + R - 1, clast])
    want_gl = np.where(lane * R + R < rows, F[np.minimum(lane * R + R, rows - 1), clast], Fo[clast])
    assert np.array_equal(gl, want_gl)
    want_hup = np.where(lane == 0, reg["top"][clast + 1], H[np.maximum(lane * R - 1, 0), clast])
    assert np.array_equal(hup, want_hup)
    cols = np.arange(STEPS) - (STEPS - 1) - c0  # lane 63 at step m sits at column m - 63
    assert np.array_equal(out[:, 0], H[rows - 1, cols])
    assert np.array_equal(out[:, 1], Fo[cols])
    # the tick's maximum over every cell it computed
    cells = [H[l * R + k, m - l - c0] for l in range(LANES) for k in range(R) for m in range(STEPS)]
    assert tmax == max(cells)

