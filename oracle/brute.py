"""Brute-force DTW by enumeration of every warping path (test infrastructure only).

Pure Python, for M, N <= 8.  It shares nothing with the C oracle: it walks the
definition of a warping path (Sec. 2.1 of Tralie & Dempsey, arXiv 2008.02734:
W_1 = (0,0), W_K = (M-1,N-1), steps (0,1), (1,0), (1,1)) and the objective of
Eq. 1 (sum of the frame cost along the path) directly, with no recurrence.

The number of warping paths of an M x N grid is the Delannoy number
D(M-1, N-1) = sum_k binom(M-1,k) binom(N-1,k) 2^k, which pins the enumerator.

Tie rule: among all minimisers, the path whose move sequence read backwards
from (M-1,N-1) is lexicographically smallest under DIAG < UP < LEFT, with
UP = (i-1,j) and LEFT = (i,j-1).  A greedy backtrace that prefers DIAG, then
UP, then LEFT yields exactly this path (and one that prefers LEFT, then UP,
then DIAG the smallest under the reversed ranking).
"""
from __future__ import annotations

import math
from math import comb

DIAG, UP, LEFT = 0, 1, 2


def delannoy(m: int, n: int) -> int:
    """Delannoy number D(m, n): lattice paths from (0,0) to (m,n) with steps E, N, NE."""
    return sum(comb(m, k) * comb(n, k) * 2**k for k in range(min(m, n) + 1))


def frame_cost(x, y) -> float:
    """Euclidean distance between two frames (Sec. 4.1), summed in dimension order."""
    s = 0.0
    for a, b in zip(x, y):
        e = float(a) - float(b)
        s += e * e
    return math.sqrt(s)


def enumerate_paths(M: int, N: int):
    """Yield every warping path of an M x N grid as a tuple of (i, j) cells."""
    def rec(i, j, acc):
        if i == M - 1 and j == N - 1:
            yield tuple(acc)
            return
        for di, dj in ((1, 1), (1, 0), (0, 1)):
            a, b = i + di, j + dj
            if a < M and b < N:
                acc.append((a, b))
                yield from rec(a, b, acc)
                acc.pop()

    yield from rec(0, 0, [(0, 0)])


def backward_moves(path):
    """Move labels read from the end of the path back to its start."""
    out = []
    for q in range(len(path) - 1, 0, -1):
        (i, j), (pi, pj) = path[q], path[q - 1]
        if (i - pi, j - pj) == (1, 1):
            out.append(DIAG)
        elif (i - pi, j - pj) == (1, 0):
            out.append(UP)
        else:
            out.append(LEFT)
    return tuple(out)


def brute_dtw(X, Y, cost=frame_cost, order=(DIAG, UP, LEFT)):
    """Return (optimal cost, tie-broken optimal path, number of paths enumerated).

    Path costs are summed sequentially from (0,0), in path order.  `order`
    lists the moves from most to least preferred; among minimisers the path
    whose backward move sequence is lexicographically smallest under that
    ranking wins (the default is DIAG, then UP, then LEFT; (LEFT, UP, DIAG)
    is the reversed rule of Sec. 4.2).
    """
    M, N = len(X), len(Y)
    if M > 8 or N > 8:
        raise ValueError("brute force is limited to M, N <= 8")
    rank = {mv: r for r, mv in enumerate(order)}
    C = [[cost(X[i], Y[j]) for j in range(N)] for i in range(M)]
    best = math.inf
    best_path = None
    count = 0
    for p in enumerate_paths(M, N):
        count += 1
        s = 0.0
        for (i, j) in p:
            s += C[i][j]
        if s < best or (s == best and [rank[m] for m in backward_moves(p)] <
                        [rank[m] for m in backward_moves(best_path)]):
            best, best_path = s, p
    return best, best_path, count


def brute_dtw_f32(X, Y):
    """Binary32 brute force for one-dimensional frames: every path's cost is the
    sequential float32 sum of float32 frame costs sqrt(e*e), e = x - y with x
    and y rounded to float32 (with one dimension the frame cost involves a
    single rounded product, so no fused operation is needed).  Returns the
    smallest such sum as a float.  Because float addition is monotone, the
    float32 recurrence reaches exactly this value."""
    import numpy as np
    M, N = len(X), len(Y)
    if M > 8 or N > 8:
        raise ValueError("brute force is limited to M, N <= 8")
    xs = [np.float32(float(np.ravel(x)[0])) for x in X]
    ys = [np.float32(float(np.ravel(y)[0])) for y in Y]
    if any(np.size(x) != 1 for x in X) or any(np.size(y) != 1 for y in Y):
        raise ValueError("one-dimensional frames only")
    C = [[np.sqrt((xs[i] - ys[j]) * (xs[i] - ys[j])) for j in range(N)] for i in range(M)]
    best = None
    for p in enumerate_paths(M, N):
        s = np.float32(0.0)
        for (i, j) in p:
            s = np.float32(s + C[i][j])
        if best is None or s < best:
            best = s
    return float(best)


def brute_edit(a, b, sub=1, gap=1):
    """Weighted edit distance by enumeration of every lattice path of nodes
    (0,0) -> (M,N), M, N <= 7 (the moves of an (M+1) x (N+1) warping grid).
    A DIAG move into node (i,j) costs 0 when a[i-1] == b[j-1], else `sub`;
    UP and LEFT moves cost `gap`.  Returns (least cost, the minimiser whose
    backward move sequence is smallest under DIAG < UP < LEFT, number of
    optimal paths)."""
    M, N = len(a), len(b)
    if M > 7 or N > 7:
        raise ValueError("brute force is limited to M, N <= 7")
    rank = {DIAG: 0, UP: 1, LEFT: 2}
    best, best_path, n_best = None, None, 0
    for p in enumerate_paths(M + 1, N + 1):
        s = 0
        for q in range(1, len(p)):
            (i, j), (pi, pj) = p[q], p[q - 1]
            if (i - pi, j - pj) == (1, 1):
                s += 0 if a[i - 1] == b[j - 1] else sub
            else:
                s += gap
        if best is None or s < best:
            best, best_path, n_best = s, p, 1
        elif s == best:
            n_best += 1
            if [rank[m] for m in backward_moves(p)] < [rank[m] for m in backward_moves(best_path)]:
                best_path = p
    return best, best_path, n_best


def brute_lcs(a, b):
    """Length of a longest common subsequence, by trying every subsequence of
    the shorter string (length <= 12) against the other."""
    from itertools import combinations
    if len(a) > len(b):
        a, b = b, a
    if len(a) > 12:
        raise ValueError("brute force is limited to 12 characters")

    def is_subseq(s, t):
        it = iter(t)
        return all(ch in it for ch in s)

    for k in range(len(a), 0, -1):
        for idx in combinations(range(len(a)), k):
            if is_subseq([a[i] for i in idx], b):
                return k
    return 0


def brute_local(a, b, match=2, mismatch=1, gap=1):
    """Smith-Waterman by enumeration: the best score of a global alignment
    (every lattice path) of every pair of substrings a[i0:i1], b[j0:j1],
    M, N <= 5, and the end (i1, j1) of the first best pair in row-major order
    of the end cell ((0, 0) for score 0; an empty pair scores 0)."""
    M, N = len(a), len(b)
    if M > 5 or N > 5:
        raise ValueError("brute force is limited to M, N <= 5")
    best, end = 0, (0, 0)
    for i1 in range(1, M + 1):
        for j1 in range(1, N + 1):
            for i0 in range(i1):
                for j0 in range(j1):
                    sa, sb = a[i0:i1], b[j0:j1]
                    for p in enumerate_paths(len(sa) + 1, len(sb) + 1):
                        s = 0
                        for q in range(1, len(p)):
                            (i, j), (pi, pj) = p[q], p[q - 1]
                            if (i - pi, j - pj) == (1, 1):
                                s += match if sa[i - 1] == sb[j - 1] else -mismatch
                            else:
                                s -= gap
                        if s > best:
                            best, end = s, (i1, j1)
    return best, end
