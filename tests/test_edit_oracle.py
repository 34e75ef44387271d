"""Pins of the edit-distance oracle (CPU): hand-worked tables, brute force,
closed forms, metric properties, the row sweeps against sub-block tables,
the linear-memory recursion against the textbook table, and planted mistakes.

The paper names edit distance as a problem with the same dynamic-programming
structure (Sec. 6) without defining an algorithm for it; the definitions
pinned here are the lattice, move costs and row split of oracle/edit_oracle.c.
"""
import json
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from oracle import edit
from oracle.brute import brute_edit, brute_lcs, delannoy, enumerate_paths
from paper_2008_02734_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden", "edit_examples.json")

COSTS = [(1, 1), (2, 1), (3, 2), (1, 3), (0, 1), (5, 2)]


def _rand(seed, M, N, k):
    rng = np.random.default_rng([11, seed])
    return rng.integers(0, k, M).astype(np.uint8), rng.integers(0, k, N).astype(np.uint8)


def test_golden_tables_and_paths():
    ex = json.load(open(GOLDEN))
    for e in ex["examples"]:
        d, p, E = edit.full(e["a"], e["b"], e["sub"], e["gap"], return_table=True)
        assert E.tolist() == e["E"], e["name"]
        assert p.tolist() == e["path"], e["name"]
        assert d == e["dist"], e["name"]
    for e in ex["classic"]:
        assert edit.full(e["a"], e["b"], e["sub"], e["gap"])[0] == e["dist"]
        assert edit.linear(e["a"], e["b"], e["sub"], e["gap"], leaf_rows=2)["dist"] == e["dist"]


def test_enumerator_counts_node_paths():
    # node paths (0,0) -> (M,N) are the warping paths of an (M+1) x (N+1) grid
    for M in range(4):
        for N in range(4):
            assert sum(1 for _ in enumerate_paths(M + 1, N + 1)) == delannoy(M, N)


@pytest.mark.parametrize("sub,gap", COSTS)
def test_table_equals_brute_force(sub, gap):
    # every size up to 5 x 5, binary and 3-letter alphabets (many exact ties):
    # the distance, and the backtrace's path is the brute force's tie path
    for M in range(0, 6):
        for N in range(0, 6):
            for k in (2, 3):
                a, b = _rand(100 * M + 10 * N + k, M, N, k)
                d, p = edit.full(a, b, sub, gap)
                bd, bp, _ = brute_edit(a.tolist(), b.tolist(), sub, gap)
                assert d == bd
                assert p.tolist() == [list(q) for q in bp]


@pytest.mark.parametrize("gap", [1, 2, 3])
def test_indel_only_distance_is_lcs(gap):
    # with sub >= 2 gap a substitution never beats a deletion plus an
    # insertion, so the distance is gap (M + N - 2 LCS)
    for s in range(40):
        rng = np.random.default_rng([12, s])
        M, N = (int(v) for v in rng.integers(0, 10, 2))
        a, b = _rand(1000 + s, M, N, 3)
        assert edit.full(a, b, 2 * gap + s % 3, gap)[0] == gap * (M + N - 2 * brute_lcs(a.tolist(), b.tolist()))


def test_closed_forms():
    a, _ = _rand(5, 37, 1, 4)
    for sub, gap in COSTS:
        d, p = edit.full(a, a, sub, gap)
        assert d == 0 and p.tolist() == [[i, i] for i in range(38)]
        assert edit.full(a, b"", sub, gap)[0] == 37 * gap
        assert edit.full(b"", a, sub, gap)[0] == 37 * gap
        d, p = edit.full(b"", b"", sub, gap)
        assert d == 0 and p.tolist() == [[0, 0]]
        # disjoint alphabets: min(M,N) substitutions (or two gaps each) plus |M-N| gaps
        x = np.full(9, 1, np.uint8)
        y = np.full(14, 2, np.uint8)
        assert edit.full(x, y, sub, gap)[0] == 9 * min(sub, 2 * gap) + 5 * gap


def test_metric_properties():
    for s in range(30):
        rng = np.random.default_rng([13, s])
        M, N, P = (int(v) for v in rng.integers(0, 40, 3))
        a, b = _rand(2000 + s, M, N, 4)
        c, _ = _rand(3000 + s, P, 1, 4)
        for sub, gap in ((1, 1), (2, 1), (3, 2)):  # sub <= 2 gap: a metric
            dab = edit.full(a, b, sub, gap)[0]
            assert dab == edit.full(b, a, sub, gap)[0]
            assert dab == edit.full(a[::-1].copy(), b[::-1].copy(), sub, gap)[0]
            assert edit.full(a, c, sub, gap)[0] <= dab + edit.full(b, c, sub, gap)[0]
            assert dab <= gap * (M + N)


def test_row_sweeps_against_block_tables():
    # forward: the last row of the block's own table; backward: entry j is the
    # distance of the sub-block from (i0, j) to (i1, j1), solved on its own
    a, b = _rand(77, 30, 26, 3)
    for (i0, j0, i1, j1) in ((0, 0, 30, 26), (3, 5, 17, 20), (10, 0, 11, 26), (4, 9, 29, 9)):
        for sub, gap in ((1, 1), (3, 2)):
            f = edit.row(a, b, i0, j0, i1, j1, sub, gap, rev=False)
            _, _, E = edit.full(a[i0:i1], b[j0:j1], sub, gap, return_table=True)
            assert f.tolist() == E[-1].tolist()
            r = edit.row(a, b, i0, j0, i1, j1, sub, gap, rev=True)
            assert r.tolist() == [edit.full(a[i0:i1], b[j:j1], sub, gap)[0] for j in range(j0, j1 + 1)]


def test_levels():
    for M in range(0, 300):
        for h in (2, 3, 7, 64):
            L = edit.levels(M, h)
            assert -(-M // (1 << L)) <= h
            assert L == 0 or -(-M // (1 << (L - 1))) > h


@pytest.mark.parametrize("h", [2, 3, 8, 64])
def test_linear_distance_and_path(h):
    for s in range(25):
        rng = np.random.default_rng([14, s, h])
        M, N = (int(v) for v in rng.integers(0, 150, 2))
        a, b = synth.string_pair(4000 + s, M, N, k=int(rng.integers(2, 5)), p=0.3)
        sub, gap = COSTS[s % len(COSTS)]
        d, p = edit.full(a, b, sub, gap)
        r = edit.linear(a, b, sub, gap, leaf_rows=h)
        assert r["dist"] == d
        assert edit.path_cost(a, b, r["path"], sub, gap) == d
        assert r["path"].shape[0] >= max(M, N) + 1


def test_linear_takes_the_unique_optimal_path():
    seen = 0
    for s in range(300):
        rng = np.random.default_rng([15, s])
        M, N = (int(v) for v in rng.integers(1, 8, 2))
        a, b = _rand(5000 + s, M, N, 4)
        sub, gap = COSTS[s % 4]
        bd, bp, nb = brute_edit(a.tolist(), b.tolist(), sub, gap)
        if nb != 1:
            continue
        seen += 1
        for h in (2, 3):
            assert edit.linear(a, b, sub, gap, leaf_rows=h)["path"].tolist() == [list(q) for q in bp]
    assert seen > 50


def test_pivots_lie_on_optimal_paths():
    # each split node (mid, j) of the top level: best cost through it equals the distance
    a, b = synth.string_pair(6000, 300, 280, k=4, p=0.2)
    for sub, gap in ((1, 1), (2, 3)):
        d, _, E = edit.full(a, b, sub, gap, return_table=True)
        r = edit.linear(a, b, sub, gap, leaf_rows=4, pivots=True)
        L0, k, mid, j = r["pivots"][0].tolist()
        assert (L0, k, mid) == (0, 0, 150)
        tail = edit.full(a[mid:], b[j:], sub, gap)[0]
        assert E[mid, j] + tail == d
        assert [mid, j] in r["path"].tolist()
        assert len(r["pivots"]) == 2 ** edit.levels(300, 4) - 1


# ------------------------------------------------------------------ local alignment (Smith-Waterman)

LOCAL_SCORES = [(2, 1, 1), (1, 1, 1), (3, 2, 2), (1, 3, 1), (2, 0, 0), (5, 1, 3)]


@pytest.mark.parametrize("match,mismatch,gap", LOCAL_SCORES)
def test_local_score_equals_brute_force(match, mismatch, gap):
    # every size up to 5 x 5 on 2- and 3-letter alphabets: the best score over
    # all substring pairs and all their alignments, and its first end cell
    from oracle.brute import brute_local
    for M in range(0, 6):
        for N in range(0, 6):
            for k in (2, 3):
                a, b = _rand(700 + 100 * M + 10 * N + k, M, N, k)
                sc, i, j = edit.local_score(a, b, match, mismatch, gap)
                bs, (bi, bj) = brute_local(a.tolist(), b.tolist(), match, mismatch, gap)
                assert (sc, i, j) == (bs, bi, bj)


def test_local_score_closed_forms():
    a, _ = _rand(21, 57, 1, 4)
    for match, mismatch, gap in LOCAL_SCORES:
        # a string against itself: every letter matched, ending at (M, M)
        assert edit.local_score(a, a, match, mismatch, gap) == (match * 57, 57, 57)
        # no common letter: nothing scores above 0
        assert edit.local_score(np.full(9, 1, np.uint8), np.full(12, 2, np.uint8), match, mismatch, gap) == (0, 0, 0)
        assert edit.local_score(a, b"", match, mismatch, gap) == (0, 0, 0)
        # one common letter at the end of both: a single match
        x = np.array([1, 1, 1, 3], np.uint8)
        y = np.array([2, 2, 3], np.uint8)
        assert edit.local_score(x, y, match, mismatch, gap) == (match, 4, 3)
        # a planted common substring in unrelated text scores at least its matches
        p = np.arange(40, 40 + 30, dtype=np.uint8)
        u = np.concatenate([np.full(50, 1, np.uint8), p, np.full(20, 2, np.uint8)])
        w = np.concatenate([np.full(35, 3, np.uint8), p, np.full(10, 4, np.uint8)])
        assert edit.local_score(u, w, match, mismatch, gap) == (30 * match, 80, 65)


def test_local_score_symmetry_and_global_bound():
    # the score is symmetric in a and b, and at least the global alignment
    # score of the whole strings: with m, x, g the match score and the two
    # penalties, 2 x global score = m (M + N) - d, d the edit distance with
    # sub = 2 (m + x) and gap = 2 g + m (matches + mismatches + gaps/2 = (M+N)/2)
    for s in range(30):
        rng = np.random.default_rng([16, s])
        M, N = (int(v) for v in rng.integers(0, 60, 2))
        a, b = synth.string_pair(7000 + s, M, N, k=4, p=0.3)
        for m, x, g in ((2, 1, 1), (3, 2, 2)):
            sc, i, j = edit.local_score(a, b, m, x, g)
            assert sc == edit.local_score(b, a, m, x, g)[0]
            d = edit.full(a, b, 2 * (m + x), 2 * g + m)[0]
            assert 2 * sc >= m * (M + N) - d
            assert sc >= 0 and 0 <= i <= M and 0 <= j <= N


# ------------------------------------------------------------------ planted mistakes

MUTANTS = {
    "diag_costs_gap": ("int64_t dg = E[(i - 1) * ld + j - 1] + move_sub(a[i0 + i - 1], b[j0 + j - 1], sub);",
                       "int64_t dg = E[(i - 1) * ld + j - 1] + gap;"),
    "match_costs_sub": ("return x == y ? 0 : sub;", "return x == y ? sub : 0;"),
    "row0_no_prefix": ("for (int64_t j = 0; j <= W; ++j) E[j] = j * (int64_t)gap;",
                       "for (int64_t j = 0; j <= W; ++j) E[j] = 0;"),
    "col0_no_prefix": ("E[i * ld] = i * (int64_t)gap;", "E[i * ld] = 0;"),
    "backtrace_up_first": ("if (i > 0 && j > 0 && e == E[(i - 1) * ld + j - 1]",
                           "if (i > 0 && j > 0 && e != E[(i - 1) * ld + j] + gap && e == E[(i - 1) * ld + j - 1]"),
    "row_sweep_no_left_boundary": ("row[0] = r * (int64_t)gap;", "row[0] = 0;"),
    "backward_not_reversed": ("const uint8_t x = rev ? a[i1 - r] : a[i0 + r - 1];",
                              "const uint8_t x = a[i0 + r - 1];"),
    "split_forward_only": ("const int64_t s = c->F[j - j0] + c->B[j - j0];", "const int64_t s = c->F[j - j0];"),
    "leaf_node_duplicated": ("c->n += c->n > 0 ? m - 1 : m;", "c->n += m;"),
    "local_no_floor_at_zero": ("      if (h < 0) h = 0;\n", "      if (h < -1000000) h = 0;\n"),
    "local_mismatch_added": ("const int64_t s = a[i - 1] == b[j - 1] ? match : -(int64_t)mismatch;",
                             "const int64_t s = a[i - 1] == b[j - 1] ? match : (int64_t)mismatch;"),
    "local_end_last_maximum": ("      if (h > best) {\n        best = h;", "      if (h >= best && h > 0) {\n        best = h;"),
    "reversed_row_not_flipped": ("for (int64_t p = 0, q = W; p < q; ++p, --q) {\n      int64_t t = row[p];",
                                 "for (int64_t p = 0, q = -1; p < q; ++p, --q) {\n      int64_t t = row[p];"),
}

CHECKS = textwrap.dedent(r'''
    import sys, json, numpy as np
    sys.path.insert(0, sys.argv[2])
    from oracle import edit
    from oracle.brute import brute_edit
    from paper_2008_02734_amd import synth
    L = edit.load(sys.argv[1])
    fails = []
    def check(name, ok):
        if not ok: fails.append(name)
    ex = json.load(open(sys.argv[2] + "/tests/golden/edit_examples.json"))
    for e in ex["examples"]:
        d, p, E = edit.full(e["a"], e["b"], e["sub"], e["gap"], return_table=True, L=L)
        check("golden", E.tolist() == e["E"] and p.tolist() == e["path"] and d == e["dist"])
    for s in range(30):
        rng = np.random.default_rng([11, s])
        M, N = int(rng.integers(0, 6)), int(rng.integers(0, 6))
        a = rng.integers(0, 2, M).astype(np.uint8); b = rng.integers(0, 2, N).astype(np.uint8)
        for sub, gap in ((1, 1), (3, 2)):
            d, p = edit.full(a, b, sub, gap, L=L)
            bd, bp, _ = brute_edit(a.tolist(), b.tolist(), sub, gap)
            check("brute", d == bd and p.tolist() == [list(q) for q in bp])
    for s in range(8):
        a, b = synth.string_pair(4000 + s, 60 + 7 * s, 55 + 5 * s, k=3, p=0.3)
        for sub, gap in ((1, 1), (2, 3)):
            d, _ = edit.full(a, b, sub, gap, L=L)
            r = edit.linear(a, b, sub, gap, leaf_rows=3, L=L)
            check("linear", r["dist"] == d and r["path"].shape[0] >= max(a.size, b.size) + 1
                  and edit.path_cost(a, b, r["path"], sub, gap, L=L) == d)
            rr = edit.row(a, b, 5, 3, 40, 50, sub, gap, rev=True, L=L)
            check("row_rev", rr.tolist() == [edit.full(a[5:40], b[j:50], sub, gap, L=L)[0] for j in range(3, 51)])
    from oracle.brute import brute_local
    for s in range(40):
        rng = np.random.default_rng([17, s])
        M, N = int(rng.integers(0, 6)), int(rng.integers(0, 6))
        a = rng.integers(0, 3, M).astype(np.uint8); b = rng.integers(0, 3, N).astype(np.uint8)
        for m, x, gp in ((2, 1, 1), (1, 3, 1)):
            bs, (bi, bj) = brute_local(a.tolist(), b.tolist(), m, x, gp)
            check("local_brute", edit.local_score(a, b, m, x, gp, L=L) == (bs, bi, bj))
    # a common substring after unrelated text: the best alignment starts where
    # every earlier cell has fallen to zero
    p = np.arange(40, 70, dtype=np.uint8)
    u = np.concatenate([np.full(50, 1, np.uint8), p, np.full(20, 2, np.uint8)])
    w = np.concatenate([np.full(35, 3, np.uint8), p, np.full(10, 4, np.uint8)])
    check("local_planted", edit.local_score(u, w, 2, 1, 1, L=L) == (60, 80, 65))
    print(json.dumps(fails))
''')


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = edit.source()
    assert src.count(old) == 1, name
    lib = edit.build_variant(src.replace(old, new), str(tmp_path / f"m_{name}.so"))
    r = subprocess.run([sys.executable, "-c", CHECKS, lib, ROOT], capture_output=True, text=True, timeout=300)
    fails = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 and r.stdout.strip() else ["crash"]
    assert fails, f"planted mistake {name} survived every check"


def test_unmodified_oracle_passes_the_mutant_checks(tmp_path):
    lib = edit.build_variant(edit.source(), str(tmp_path / "clean.so"))
    r = subprocess.run([sys.executable, "-c", CHECKS, lib, ROOT], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert json.loads(r.stdout.strip().splitlines()[-1]) == []
