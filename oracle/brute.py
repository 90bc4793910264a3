"""Brute-force enumerations that pin the C oracle on tiny inputs -- TEST INFRASTRUCTURE ONLY.

Nothing here runs a dynamic program.  Alignments are enumerated as explicit
edit paths and scored one by one from the affine-gap definition (a maximal
gap run of length k costs open + extend*(k-1)), so a dropped term, a wrong
sign or a transposed operand in ``gotoh.c`` shows up as a disagreement.
"""
from __future__ import annotations


def _s(x: int, y: int, sc) -> int:
    if hasattr(sc, "s"):  # substitution matrix
        return sc.s(x, y)
    return sc[0] if (x & 0xDF) == (y & 0xDF) else -sc[1]


def local_alignments(a: bytes, b: bytes, sc):
    """Yield (score, sa, sb, ea, eb) for every local alignment that begins and ends with an aligned pair.

    An optimal local alignment never begins or ends with a gap (dropping it
    would raise the score), so these are all the candidates for the optimum.
    Gap runs may follow each other only if they differ in kind (an I run may
    be followed directly by a D run and vice versa), which is every path of
    the edit graph written as maximal runs.
    """
    m, n = len(a), len(b)
    go, ge = sc[2], sc[3]
    for sa in range(m):
        for sb in range(n):
            stack = [(sa + 1, sb + 1, _s(a[sa], b[sb], sc), "M")]
            while stack:
                i, j, v, last = stack.pop()
                if last == "M":
                    yield v, sa, sb, i - 1, j - 1
                if i < m and j < n:
                    stack.append((i + 1, j + 1, v + _s(a[i], b[j], sc), "M"))
                if last != "I":
                    for k in range(1, n - j + 1):
                        stack.append((i, j + k, v - (go + ge * (k - 1)), "I"))
                if last != "D":
                    for k in range(1, m - i + 1):
                        stack.append((i + k, j, v - (go + ge * (k - 1)), "D"))


def local_best(a: bytes, b: bytes, sc):
    """(S, start_a, start_b, end_a, end_b) by enumeration.

    End = lexicographically smallest (end_a, end_b) among optimal alignments;
    start = lexicographically largest (start_a, start_b) among optimal
    alignments with that end.  All -1 when S = 0.
    """
    best = 0
    ends = {}
    for v, sa, sb, ea, eb in local_alignments(a, b, sc):
        if v > best:
            best = v
            ends = {}
        if v == best and v > 0:
            ends.setdefault((ea, eb), set()).add((sa, sb))
    if best == 0:
        return 0, -1, -1, -1, -1
    end = min(ends)
    start = max(ends[end])
    return best, start[0], start[1], end[0], end[1]


def global_paths(M: int, N: int):
    """Every path (0,0) -> (M,N) of the edit graph as a string over 'M' (pair), 'I' (B only), 'D' (A only)."""
    out = []

    def rec(i, j, acc):
        if i == M and j == N:
            out.append("".join(acc))
            return
        if i < M and j < N:
            acc.append("M")
            rec(i + 1, j + 1, acc)
            acc.pop()
        if j < N:
            acc.append("I")
            rec(i, j + 1, acc)
            acc.pop()
        if i < M:
            acc.append("D")
            rec(i + 1, j, acc)
            acc.pop()

    rec(0, 0, [])
    return out


def path_score(A: bytes, B: bytes, path: str, sc, tb: int, te: int) -> int:
    """Score of a global path with gap cost g + h*k (g = open - extend, h = extend).

    A deletion run that leaves (0,0) opens at ``tb`` and one that ends at (M,N)
    opens at ``te`` (the smaller of the two if it does both); every other run
    opens at g.
    """
    g, h = sc[2] - sc[3], sc[3]
    i = j = 0
    v = 0
    k = 0
    n = len(path)
    while k < n:
        op = path[k]
        if op == "M":
            v += _s(A[i], B[j], sc)
            i += 1
            j += 1
            k += 1
            continue
        r = k
        while r < n and path[r] == op:
            r += 1
        L = r - k
        if op == "I":
            v -= g + h * L
            j += L
        else:
            starts = (k == 0)
            ends = (r == n)
            if starts and ends:
                o = min(tb, te)
            elif starts:
                o = tb
            elif ends:
                o = te
            else:
                o = g
            v -= o + h * L
            i += L
        k = r
    return v


def _crossing(path: str, mid: int):
    """(j, type) where the path meets vertex row ``mid``: first column, type 2 if it passes straight down."""
    i = j = 0
    for k, op in enumerate(path):
        if i == mid:
            entered_down = k > 0 and path[k - 1] == "D"
            leaves_down = op == "D"
            return j, (2 if entered_down and leaves_down else 1)
        if op == "M":
            i += 1
            j += 1
        elif op == "I":
            j += 1
        else:
            i += 1
    return j, 1


def canonical_global(A: bytes, B: bytes, sc, tb: int, te: int) -> str:
    """Canonical optimal global path by enumeration plus the midline rule.

    The midline (row M//2) is chosen as the smallest (column, type) over all
    optimal paths, a plain crossing ranked before a straight vertical pass;
    the two halves are solved again the same way with the gap-open
    conventions of the split.  Base cases: N = 0 all deletions; M = 0 all
    insertions; M = 1 the optimal path that aligns A_0 to the leftmost
    possible B_k, else the deletion next to the cheaper open side (first
    unless te < tb).  Returns the op string over 'MID'.
    """
    M, N = len(A), len(B)
    g = sc[2] - sc[3]
    if N == 0:
        return "D" * M
    if M == 0:
        return "I" * N
    paths = global_paths(M, N)
    scores = [path_score(A, B, p, sc, tb, te) for p in paths]
    best = max(scores)
    opt = [p for p, v in zip(paths, scores) if v == best]
    if M == 1:
        with_pair = [p for p in opt if "M" in p]
        if with_pair:
            return min(with_pair, key=lambda p: p.index("M"))
        first = "D" + "I" * N
        last = "I" * N + "D"
        pick = last if te < tb else first
        if pick not in opt:
            raise AssertionError("base case preference is not optimal")
        return pick
    mid = M // 2
    cj, ct = min(_crossing(p, mid) for p in opt)
    if ct == 1:
        return (canonical_global(A[:mid], B[:cj], sc, tb, g)
                + canonical_global(A[mid:], B[cj:], sc, g, te))
    return (canonical_global(A[:mid - 1], B[:cj], sc, tb, 0) + "DD"
            + canonical_global(A[mid + 1:], B[cj:], sc, 0, te))


def best_global(A: bytes, B: bytes, sc, tb: int, te: int) -> int:
    return max(path_score(A, B, p, sc, tb, te) for p in global_paths(len(A), len(B)))


def ops_to_cigar(A: bytes, B: bytes, ops: str) -> str:
    """'MID' path -> run-length CIGAR with '=' / 'X' split by the letters."""
    out = []
    i = j = 0
    for op in ops:
        if op == "M":
            o = "=" if (A[i] & 0xDF) == (B[j] & 0xDF) else "X"
            i += 1
            j += 1
        elif op == "I":
            o = "I"
            j += 1
        else:
            o = "D"
            i += 1
        if out and out[-1][1] == o:
            out[-1][0] += 1
        else:
            out.append([1, o])
    return "".join(f"{n}{o}" for n, o in out)
