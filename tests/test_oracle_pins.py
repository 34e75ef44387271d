"""Pins for the CPU oracle: it is checked against things other than itself.

Each test cites the passage of Tralie & Dempsey (arXiv 2008.02734) that fixes
the expected value.  Together they are meant to fail on any plausible slip in
the oracle (dropped term, wrong tie order, wrong boundary, transposed operand,
wrong split arithmetic); test_oracle_mutants.py plants such slips and checks
that these pins catch them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.brute import brute_dtw, delannoy, enumerate_paths
from paper_2008_02734_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def valid_path(path, M, N):
    """Warping-path definition of Sec. 2.1."""
    p = np.asarray(path)
    if p.shape[0] < 1 or tuple(p[0]) != (0, 0) or tuple(p[-1]) != (M - 1, N - 1):
        return False
    steps = np.diff(p, axis=0)
    ok = {(0, 1), (1, 0), (1, 1)}
    return all(tuple(s) in ok for s in steps)


# ---------------------------------------------------------------- enumerator

@pytest.mark.parametrize("m,n,expected", [(3, 3, 63), (7, 7, 48639), (2, 5, 61), (1, 1, 3)])
def test_delannoy_textbook_values(m, n, expected):
    # Published Delannoy numbers: D(1,1)=3, D(2,5)=61, D(3,3)=63, D(7,7)=48639.
    assert delannoy(m, n) == expected


@pytest.mark.parametrize("M,N", [(1, 1), (1, 5), (4, 1), (3, 3), (4, 6), (6, 5), (8, 8)])
def test_enumerator_counts_delannoy(M, N):
    paths = list(enumerate_paths(M, N))
    assert len(paths) == delannoy(M - 1, N - 1)
    assert len(set(paths)) == len(paths)
    assert all(valid_path(p, M, N) for p in paths)


def test_lemma1_every_path_hits_two_adjacent_diagonals():
    # Lemma 1 (Sec. 3.2): any warping path meets any 3 adjacent diagonals;
    # steps advance i+j by 1 or 2, so it even meets any 2 adjacent ones.
    M, N = 5, 6
    for p in enumerate_paths(M, N):
        ks = {i + j for i, j in p}
        for k in range(M + N - 2):
            assert k in ks or (k + 1) in ks


# ---------------------------------------------------------------- golden

def test_hand_worked_examples():
    ex = json.load(open(GOLDEN))["examples"]
    for e in ex:
        X, Y = np.array(e["X"], float), np.array(e["Y"], float)
        cost, path, F = oracle.full(X, Y, return_table=True)
        for i in range(X.shape[0]):
            for j in range(Y.shape[0]):
                assert oracle.frame_cost(X[i], Y[j]) == e["C"][i][j]
        assert F.tolist() == e["F"], e["name"]
        assert path.tolist() == e["path"], e["name"]
        assert cost == e["cost"], e["name"]


# ---------------------------------------------------------------- brute force

def _cases(kind, n):
    rng = np.random.default_rng([77, 1 if kind == "normal" else 2])
    for s in range(n):
        M, N = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        d = int(rng.integers(1, 4)) if kind == "normal" else 1
        yield (s, M, N, d)


@pytest.mark.parametrize("s,M,N,d", list(_cases("normal", 40)))
def test_full_equals_brute_continuous(s, M, N, d):
    X, Y = synth.random_pair(100 + s, M, N, d, "normal")
    cost, path = oracle.full(X, Y)
    b, bp, count = brute_dtw(X, Y)
    assert count == delannoy(M - 1, N - 1)
    assert path.tolist() == [list(c) for c in bp]
    assert abs(cost - b) <= 1e-12 * max(1.0, abs(b))
    assert valid_path(path, M, N)


@pytest.mark.parametrize("s,M,N,d", list(_cases("int3", 60)))
def test_full_equals_brute_ties(s, M, N, d):
    # Integer frames with d=1: C = |x-y| is exact and every sum is exact, so
    # ties are exact and the DIAG > UP > LEFT lexicographic path is pinned.
    X, Y = synth.random_pair(500 + s, M, N, d, "int3")
    cost, path = oracle.full(X, Y)
    b, bp, _ = brute_dtw(X, Y)
    assert cost == b
    assert path.tolist() == [list(c) for c in bp]


# ------------------------------------------- Sec. 4.2: 32-bit and tie-rule references

@pytest.mark.parametrize("s,M,N,d", list(_cases("int3", 40)))
def test_left_first_equals_brute_under_reversed_order(s, M, N, d):
    # Integer frames make ties exact; the reversed tie rule (LEFT, then UP,
    # then DIAG) must give the backward-lexicographic minimiser under that
    # ranking, with the same optimal cost as the default rule.
    from oracle.brute import DIAG, LEFT, UP
    X, Y = synth.random_pair(700 + s, M, N, d, "int3")
    cost, path = oracle.full_left_first(X, Y)
    b, bp, _ = brute_dtw(X, Y, order=(LEFT, UP, DIAG))
    assert cost == b == oracle.full(X, Y)[0]
    assert path.tolist() == [list(c) for c in bp]


def test_left_first_differs_from_default_on_a_tie():
    # X = Y = (0, 0): every path costs 0.  DIAG first steps from (1,1)
    # straight back to (0,0); LEFT first steps to (1,0), whose only move (column
    # 0) is UP to (0,0).
    X = np.zeros((2, 1))
    assert oracle.full(X, X)[1].tolist() == [[0, 0], [1, 1]]
    assert oracle.full_left_first(X, X)[1].tolist() == [[0, 0], [1, 0], [1, 1]]


@pytest.mark.parametrize("s,M,N", [(s, 1 + s % 7, 1 + (3 * s) % 8) for s in range(30)])
def test_f32_equals_float32_brute_force(s, M, N):
    # One-dimensional frames: the float32 table's optimum equals the smallest
    # sequential float32 sum over all warping paths (float addition is
    # monotone, so the recurrence reaches it exactly), and the returned path's
    # float32 sum is that value.
    from oracle.brute import brute_dtw_f32
    X, Y = synth.random_pair(900 + s, M, N, 1, "normal")
    cost, path = oracle.full_f32(X, Y)
    assert cost == brute_dtw_f32(X, Y)
    x32, y32 = X.astype(np.float32)[:, 0], Y.astype(np.float32)[:, 0]
    acc = np.float32(0.0)
    for i, j in path:
        acc = np.float32(acc + np.sqrt((x32[i] - y32[j]) * (x32[i] - y32[j])))
    assert float(acc) == cost
    assert valid_path(path, M, N)


@pytest.mark.parametrize("seed", range(8))
def test_f32_equals_f64_on_exact_inputs(seed):
    # Small integer frames (d = 1): every frame cost |x - y| and every partial
    # sum is an integer below 2^24, exact in both formats, so the float32
    # table must reproduce the FP64 optimum and path exactly.
    X, Y = synth.random_pair(950 + seed, 30 + seed, 25 + 2 * seed, 1, "int3")
    c32, p32 = oracle.full_f32(X, Y)
    c64, p64 = oracle.full(X, Y)
    assert c32 == c64 and p32.tolist() == p64.tolist()


@pytest.mark.parametrize("seed", range(6))
def test_f32_within_rounding_bound_of_f64(seed):
    # Continuous 12-dimensional frames: each float32 frame cost is within
    # (d + 3) units of 2^-24 of the exact one (input rounding, d fused steps,
    # the square root) and each of the K path additions adds one more, so the
    # optimum moves by at most (K + d + 3) * 2^-24 relative (plus a slack of
    # 2); a dropped term or a wrong operand is far outside this.
    X, Y = synth.make_pair(1, seed, 60 + 10 * seed, 50 + 7 * seed, 12, "gaussian_walk")
    c32, p32 = oracle.full_f32(X, Y)
    c64, _ = oracle.full(X, Y)
    K = X.shape[0] + Y.shape[0] - 1
    assert abs(c32 - c64) <= 2 * (K + 12 + 3) * 2.0 ** -24 * c64
    assert abs(c32 - c64) > 0 or seed > 0  # float32 rounding is visible on the first pair
    assert valid_path(p32, X.shape[0], Y.shape[0])


# ------------------------------------------- Sec. 4.1: the cosine frame cost

def _cos_cost_py(x, y):
    # 1 - cos(angle), written out independently of the oracle (plain products
    # and sums, math.sqrt), clamped at 0 like the oracle's definition
    nx = math.sqrt(sum(float(v) * float(v) for v in x))
    ny = math.sqrt(sum(float(v) * float(v) for v in y))
    if nx == 0.0 or ny == 0.0:
        return 1.0
    return max(0.0, 1.0 - sum(float(a) * float(b) for a, b in zip(x, y)) / (nx * ny))


def test_cosine_cost_closed_forms():
    e1, e2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    assert oracle.frame_cost(e1, e2, cost="cosine") == 1.0          # orthogonal
    assert oracle.frame_cost(e1, -e1, cost="cosine") == 2.0         # opposite
    assert oracle.frame_cost(e1, 5 * e1, cost="cosine") == 0.0      # parallel
    assert oracle.frame_cost(np.zeros(3), e1, cost="cosine") == 1.0  # a zero frame
    assert oracle.frame_cost(e1, np.zeros(3), cost="cosine") == 1.0
    x, y = np.array([3.0, 4.0]), np.array([6.0, 8.0])
    assert oracle.frame_cost(x, y, cost="cosine") <= 4e-16          # parallel, inexact quotients
    # 60 degrees: cos = 1/2
    a, b = np.array([1.0, 0.0]), np.array([0.5, math.sqrt(3) / 2])
    assert oracle.frame_cost(a, b, cost="cosine") == pytest.approx(0.5, abs=1e-15)
    # the Euclidean default is untouched afterwards
    assert oracle.frame_cost(e1, e2) == math.sqrt(2.0)


@pytest.mark.parametrize("s,M,N,d", list(_cases("normal", 30)))
def test_cosine_full_equals_brute(s, M, N, d):
    d = max(d, 2)
    X, Y = synth.random_pair(1100 + s, M, N, d, "normal")
    for i in range(X.shape[0]):
        for j in range(Y.shape[0]):
            assert oracle.frame_cost(X[i], Y[j], cost="cosine") == pytest.approx(_cos_cost_py(X[i], Y[j]),
                                                                                  abs=2e-15)
    cost, path = oracle.full(X, Y, cost="cosine")
    b, bp, _ = brute_dtw(X, Y, cost=_cos_cost_py)
    assert abs(cost - b) <= 1e-12 * max(1.0, b)
    assert path.tolist() == [list(c) for c in bp]


@pytest.mark.parametrize("seed", range(4))
def test_cosine_ignores_frame_scale(seed):
    # the cosine cost depends on directions only: scaling every frame by a
    # power of two leaves each normalised frame, hence every cost, path and
    # accumulated value, bit for bit unchanged
    X, Y = synth.make_pair(6, seed, 40 + seed, 33 + seed, 12, "chroma")
    c, p = oracle.full(X, Y, cost="cosine")
    rng = np.random.default_rng(seed)
    Xs = X * 2.0 ** rng.integers(-6, 7, (X.shape[0], 1))
    Ys = Y * 2.0 ** rng.integers(-6, 7, (Y.shape[0], 1))
    c2, p2 = oracle.full(Xs, Ys, cost="cosine")
    assert c2 == c and p2.tolist() == p.tolist()


@pytest.mark.parametrize("seed,m", [(0, 3), (1, 8), (2, 16)])
def test_cosine_linmdtw_equals_full_and_diag_equals_table(seed, m):
    # the divide and conquer and the sweep under the cosine cost: the same
    # identities as for the Euclidean cost (Lemma 2 gives the textbook path
    # on tie-free inputs; DiagDTW equals the table bit for bit)
    X, Y = synth.make_pair(6, 10 + seed, 70 + 9 * seed, 55 + 5 * seed, 12, "chroma")
    c, p, F = oracle.full(X, Y, return_table=True, cost="cosine")
    r = oracle.linmdtw(X, Y, min_block=m, cost="cosine")
    assert r["path"].tolist() == p.tolist()
    assert abs(r["cost"] - c) <= 1e-12 * c
    assert oracle.path_cost(X, Y, p, cost="cosine") == pytest.approx(c, rel=1e-12)
    M, N = X.shape[0], Y.shape[0]
    kstop = (M + N) // 2
    out = oracle.diag(X, Y, 0, 0, M - 1, N - 1, 0, kstop, cost="cosine")
    for q in range(3):
        for a in range(M):
            b = kstop - 2 + q - a
            if 0 <= b < N:
                assert out[q, a] == F[a, b]


# ---------------------------------------------------------------- closed forms

def test_single_row_and_column_are_forced():
    # M = 1 or N = 1: the only warping path walks the single row/column, and the
    # boundary equation makes D the prefix sum of C (Sec. 2.1, Eq. 3).
    rng = np.random.default_rng(5)
    X = rng.standard_normal((1, 4))
    Y = rng.standard_normal((9, 4))
    cost, path = oracle.full(X, Y)
    assert path.tolist() == [[0, j] for j in range(9)]
    s = 0.0
    for j in range(9):
        s += oracle.frame_cost(X[0], Y[j])
    assert cost == s
    cost2, path2 = oracle.full(Y, X)
    assert path2.tolist() == [[i, 0] for i in range(9)]
    assert cost2 == s


def test_identical_sequences_diagonal_zero():
    X = synth.random_pair(3, 30, 30, 5)[0]
    cost, path = oracle.full(X, X)
    assert cost == 0.0
    assert path.tolist() == [[i, i] for i in range(30)]


def test_repeated_frames_staircase():
    # Y repeats every frame of X r times: the unique zero-cost path is the
    # staircase that holds each X frame for r Y frames.
    X = synth.random_pair(4, 12, 1, 3)[0]
    r = 3
    Y = np.repeat(X, r, axis=0)
    cost, path = oracle.full(X, Y)
    assert cost == 0.0
    assert path.tolist() == [[j // r, j] for j in range(12 * r)]


def test_euclidean_not_squared():
    # Sec. 4.1: Euclidean distance.  A 3-4-5 triangle gives 5, not 25.
    assert oracle.frame_cost([0.0, 0.0], [3.0, 4.0]) == 5.0
    X = np.array([[0.0, 0.0]])
    Y = np.array([[3.0, 4.0], [6.0, 8.0]])
    assert oracle.full(X, Y)[0] == 15.0


@pytest.mark.parametrize("seed", range(6))
def test_reversal_and_transpose_invariance(seed):
    # Sec. 3.2 (proof of Lemma 2): reversing both series leaves the optimal cost
    # unchanged; swapping X and Y transposes the table.  Exact on integer costs.
    X, Y = synth.random_pair(900 + seed, 9, 13, 1, "int3")
    c = oracle.full(X, Y)[0]
    assert oracle.full(X[::-1], Y[::-1])[0] == c
    assert oracle.full(Y, X)[0] == c
    Xc, Yc = synth.random_pair(950 + seed, 9, 13, 3, "normal")
    c, p = oracle.full(Xc, Yc)
    ct, pt = oracle.full(Yc, Xc)
    assert abs(ct - c) <= 1e-12 * c
    assert pt[:, ::-1].tolist() == p.tolist()


# ---------------------------------------------------------------- Lemma 2

@pytest.mark.parametrize("kind", ["int3", "normal"])
def test_lemma2_split_cost(kind):
    # Lemma 2 (read as S = F + B - C, R3): on every cell of an optimal path the
    # forward cost plus the reversed cost minus C equals the optimum, and
    # everywhere else it is no smaller.
    for seed in range(5):
        d = 1 if kind == "int3" else 3
        X, Y = synth.random_pair(1200 + seed, 14, 11, d, kind)
        M, N = X.shape[0], Y.shape[0]
        D, path, F = oracle.full(X, Y, return_table=True)
        _, _, FR = oracle.full(X[::-1].copy(), Y[::-1].copy(), return_table=True)
        B = FR[::-1, ::-1]
        C = np.array([[oracle.frame_cost(X[i], Y[j]) for j in range(N)] for i in range(M)])
        S = (F + B) - C
        tol = 0.0 if kind == "int3" else 1e-12 * D
        for i, j in path:
            assert abs(S[i, j] - D) <= tol
        assert (S >= D - tol).all()


# ---------------------------------------------------------------- DiagDTW

@pytest.mark.parametrize("shape", [(7, 5), (5, 9), (12, 12), (3, 20), (31, 17)])
def test_diag_sweep_matches_full_table(shape):
    # Algorithm 1 fills the same table in a different order; min is exact and
    # each cell is one rounded add, so the diagonals equal the row-major table
    # bit for bit.  The reversed sweep equals the table of the reversed series.
    M, N = shape
    X, Y = synth.random_pair(sum(shape), M, N, 4, "normal")
    _, _, F = oracle.full(X, Y, return_table=True)
    _, _, FR = oracle.full(X[::-1].copy(), Y[::-1].copy(), return_table=True)
    for kstop in range(2, M + N - 1):
        for rev, T in ((0, F), (1, FR)):
            out = oracle.diag(X, Y, 0, 0, M - 1, N - 1, rev, kstop)
            for q in range(3):
                k = kstop - 2 + q
                for a in range(M):
                    b = k - a
                    if 0 <= b < N:
                        assert out[q, a] == T[a, b]
                    else:
                        assert math.isnan(out[q, a])


def test_diag_sweep_on_sub_block():
    X, Y = synth.random_pair(42, 30, 25, 3, "normal")
    i0, j0, i1, j1 = 4, 7, 20, 19
    _, _, F = oracle.full(X[i0:i1 + 1], Y[j0:j1 + 1], return_table=True)
    _, _, FR = oracle.full(X[i0:i1 + 1][::-1].copy(), Y[j0:j1 + 1][::-1].copy(), return_table=True)
    for rev, T in ((0, F), (1, FR)):
        out = oracle.diag(X, Y, i0, j0, i1, j1, rev, 15)
        for q in range(3):
            for a in range(i1 - i0 + 1):
                b = 13 + q - a
                if 0 <= b <= j1 - j0:
                    assert out[q, a] == T[a, b]


# ---------------------------------------------------------------- linmdtw

@pytest.mark.parametrize("seed,M,N,m", [(s, 20 + 7 * s, 15 + 11 * s, m)
                                        for s in range(6) for m in (3, 5, 16)])
def test_linmdtw_equals_full_tie_free(seed, M, N, m):
    # Algorithm 2 reaches the textbook optimum exactly.  On continuous inputs
    # (tie-free with probability 1) the path must be the textbook path.
    X, Y = synth.random_pair(3000 + seed, M, N, 3, "normal")
    c, p = oracle.full(X, Y)
    r = oracle.linmdtw(X, Y, min_block=m)
    assert r["path"].tolist() == p.tolist()
    assert abs(r["cost"] - c) <= 1e-12 * c
    assert abs(r["s_min"] - c) <= 1e-12 * c


@pytest.mark.parametrize("seed", range(20))
def test_linmdtw_optimal_on_ties(seed):
    # With exact ties the pivot rule may pick another optimal path (R5); the
    # cost must still be the optimum exactly and the path must be valid.
    rng = np.random.default_rng(seed)
    M, N = int(rng.integers(3, 40)), int(rng.integers(3, 40))
    X, Y = synth.random_pair(4000 + seed, M, N, 1, "int3")
    c, _ = oracle.full(X, Y)
    r = oracle.linmdtw(X, Y, min_block=3)
    assert valid_path(r["path"], M, N)
    assert r["cost"] == c
    assert oracle.path_cost(X, Y, r["path"]) == c


def test_linmdtw_leaf_only_is_textbook():
    # M < m or N < m: Algorithm 2 returns the brute-force path directly.
    X, Y = synth.config_pair(1)
    c, p = oracle.full(X, Y)
    r = oracle.linmdtw(X, Y, min_block=500)
    assert r["path"].tolist() == p.tolist()
    assert r["cost"] == c
    assert r["cells"] == 500 * 400
    assert len(r["pivots"]) == 0


def test_linmdtw_config1_small_blocks():
    X, Y = synth.config_pair(1)
    c, p = oracle.full(X, Y)
    for m in (3, 16, 64):
        r = oracle.linmdtw(X, Y, min_block=m)
        assert r["path"].tolist() == p.tolist()
        assert abs(r["cost"] - c) <= 1e-12 * c
        # pivots lie on the path
        ps = {tuple(x) for x in p.tolist()}
        assert all(tuple(v) in ps for v in r["pivots"].tolist())


def _replay_recursion(M, N, m, pivots):
    """Rebuild Algorithm 2's recursion tree from the depth-first pivot list and
    return (cells of both half sweeps + leaf tables, band cells of all splits)."""
    it = iter([tuple(v) for v in pivots.tolist()])

    def dlen(Mb, Nb, k):
        return max(0, min(Mb - 1, k) - max(0, k - Nb + 1) + 1)

    def rec(i0, j0, i1, j1):
        Mb, Nb = i1 - i0 + 1, j1 - j0 + 1
        if Mb < m or Nb < m:
            return Mb * Nb, 0
        K = Mb + Nb - 1
        kf = (K + 1) // 2
        kb = kf + (K % 2 == 0)
        cells = sum(dlen(Mb, Nb, k) for k in range(kf + 1)) + sum(dlen(Mb, Nb, k) for k in range(kb + 1))
        band = sum(dlen(Mb, Nb, k) for k in range(kf - 2, kf + 1))
        pi, pj = next(it)
        assert i0 <= pi <= i1 and j0 <= pj <= j1 and kf - 2 <= (pi - i0) + (pj - j0) <= kf
        c1, b1 = rec(i0, j0, pi, pj)
        c2, b2 = rec(pi, pj, i1, j1)
        return cells + c1 + c2, band + b1 + b2

    return rec(0, 0, M - 1, N - 1)


@pytest.mark.parametrize("m", [3, 16, 64])
def test_cells_processed_bound(m):
    # Sec. 3.2 complexity: at most 2MN + (M+N) log2(M+N) cells once the three
    # band diagonals that both half sweeps evaluate are counted once more, and
    # Sec. 4.4 (Fig. "Cell"): the ratio to MN is close to 2 for warped pairs.
    X, Y = synth.make_pair(1, 7, 600, 480, 6, "gaussian_walk")
    M, N = 600, 480
    r = oracle.linmdtw(X, Y, min_block=m)
    cells, band = _replay_recursion(M, N, m, r["pivots"])
    assert cells == r["cells"]
    assert r["cells"] <= 2 * M * N + (M + N) * math.log2(M + N) + band
    assert 1.8 <= r["cells"] / (M * N) <= 2.1


@pytest.mark.parametrize("M,N", [(40, 33), (33, 40), (57, 57), (64, 31)])
def test_pivot_tie_rule_all_zero_costs(M, N):
    # With X and Y constant every cell costs 0, so every split cost on the band
    # ties at 0; the tie rule (R5: smallest diagonal, then smallest row) picks
    # the first cell of diagonal kf-2, with kf = ceil(K/2), K = M+N-1 (Alg. 2).
    r = oracle.linmdtw(np.zeros((M, 1)), np.zeros((N, 1)), min_block=3)
    K = M + N - 1
    k = (K + 1) // 2 - 2
    a = max(0, k - (N - 1))
    assert tuple(r["pivots"][0]) == (a, k - a)
    assert r["cost"] == 0.0


def test_linmdtw_rejects_small_m():
    X, Y = synth.random_pair(1, 5, 5, 2)
    with pytest.raises(RuntimeError):
        oracle.linmdtw(X, Y, min_block=2)


# ---------------------------------------------------------------- path cost

def test_path_cost_rejects_invalid_paths():
    X, Y = synth.random_pair(2, 4, 4, 2)
    assert math.isnan(oracle.path_cost(X, Y, [[0, 0], [2, 2], [3, 3]]))
    assert math.isnan(oracle.path_cost(X, Y, [[0, 0], [1, 1], [2, 2]]))
    assert math.isnan(oracle.path_cost(X, Y, [[0, 1], [1, 2], [2, 3], [3, 3]]))
    c, p = oracle.full(X, Y)
    assert oracle.path_cost(X, Y, p) == c


# ------------------------------------------- tie-exact divide and conquer (not in the paper)
#
# The split of each block is read from labels carried by a forward table
# that starts from the origin's accumulated cost in the whole problem; the
# concatenated path must be the textbook backtrace (ties DIAG, UP, LEFT) on
# every input, also where exact ties make Algorithm 2's split ambiguous.

def _last_cell_at_or_before(path, kf):
    cells = [tuple(c) for c in path.tolist() if c[0] + c[1] <= kf]
    return cells[-1]


@pytest.mark.parametrize("fam,d", [("int3", 1), ("normal", 3), ("int3", 2)])
def test_tie_pivot_is_the_textbook_paths_cell(fam, d):
    # the label read at the end cell names the textbook path's last cell on
    # or before diagonal kf, and its accumulated cost is the table's, bit for bit
    for seed in range(40):
        rng = np.random.default_rng(7000 + seed)
        M, N = (int(v) for v in rng.integers(3, 40, 2))
        X, Y = synth.random_pair(7000 + seed, M, N, d, fam)
        c, p, F = oracle.full(X, Y, return_table=True)
        K = M + N - 1
        kf = (K + 1) // 2
        a, k, f = oracle.tie_pivot(X, Y, 0, 0, M - 1, N - 1, F[0, 0])
        assert (a, k - a) == _last_cell_at_or_before(p, kf)
        assert k in (kf - 1, kf)
        assert f == F[a, k - a]


def test_tie_pivot_of_a_child_block_keeps_the_whole_tables_values():
    # the right child of the top split starts from the pivot's value; its own
    # pivot is again a textbook path cell whose value equals the whole
    # table's (a child's table can only be larger off the path)
    for seed in range(30):
        X, Y = synth.random_pair(7100 + seed, 45, 38, 1, "int3")
        c, p, F = oracle.full(X, Y, return_table=True)
        a, k, f = oracle.tie_pivot(X, Y, 0, 0, 44, 37, F[0, 0])
        i0, j0 = a, k - a
        a2, k2, f2 = oracle.tie_pivot(X, Y, i0, j0, 44, 37, f)
        cell = (i0 + a2, j0 + k2 - a2)
        assert cell in [tuple(q) for q in p.tolist()]
        assert f2 == F[cell]


@pytest.mark.parametrize("fam,d,m", [("int3", 1, 3), ("int3", 1, 8), ("int3", 2, 5), ("normal", 3, 3),
                                     ("normal", 4, 16), ("zeros", 2, 4)])
def test_tie_exact_recursion_equals_textbook(fam, d, m):
    differs = 0
    for seed in range(60):
        rng = np.random.default_rng(7200 + seed)
        M, N = (int(v) for v in rng.integers(3, 70, 2))
        if fam == "zeros":  # every frame cost 0: every path is optimal
            X, Y = np.zeros((M, d)), np.zeros((N, d))
        else:
            X, Y = synth.random_pair(7200 + seed, M, N, d, fam)
        c, p = oracle.full(X, Y)
        r = oracle.linmdtw_tie(X, Y, min_block=m)
        assert r["path"].tolist() == p.tolist()
        assert r["cost"] == oracle.path_cost(X, Y, p)
        differs += oracle.linmdtw(X, Y, min_block=m)["path"].tolist() != p.tolist()
    if fam != "normal":
        # the inputs do exercise ties: Algorithm 2's own split leaves the
        # textbook path on some of them
        assert differs > 0
