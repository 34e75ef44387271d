"""Edit distance on the GPU (dtw_edit_align) against the oracle.

Bit-exact: the distance equals the textbook table's, and the path equals the
oracle's linear-memory recursion (same row partition, same split and leaf
tie rules) node for node.  At the benchmark size (200000 x 160000) the
oracle's recursion is too slow for a test, so the path is checked for
validity and for its cost, and prefixes and suffixes of it are checked
against the oracle's distances of the matching prefixes and suffixes of the
strings (every part of an optimal path is optimal)."""
import numpy as np
import pytest
import torch

from oracle import edit
from paper_2008_02734_amd import dtw, synth

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _dist(a, b, sub=1, gap=1):
    # the oracle's distance in linear memory (its last row)
    return int(edit.row(a, b, 0, 0, len(a), len(b), sub, gap)[-1])


def _gpu(a, b, sub, gap, h):
    d, p = dtw.edit_align(_dev(a), _dev(b), sub, gap, h)
    return d, p.cpu().numpy()


# (M, N, alphabet, mutation rate, sub, gap, leaf_rows)
CASES = [
    (0, 0, 4, 0.1, 1, 1, 64), (0, 7, 4, 0.1, 1, 1, 64), (9, 0, 4, 0.1, 1, 1, 2), (1, 1, 4, 0.1, 1, 1, 2),
    (63, 64, 4, 0.1, 1, 1, 64), (65, 64, 4, 0.1, 1, 1, 64), (257, 300, 2, 0.3, 1, 1, 2),
    (1000, 700, 4, 0.2, 1, 1, 64), (3000, 2500, 4, 0.1, 2, 1, 32), (4099, 4097, 20, 0.05, 3, 2, 17),
    (5000, 50, 4, 0.1, 1, 1, 64), (50, 20000, 4, 0.1, 1, 1, 64), (2000, 2000, 4, 0.0, 1, 1, 64),
    (20000, 16000, 4, 0.1, 1, 1, 64), (60000, 50000, 4, 0.1, 1, 1, 64),
]


@pytest.mark.parametrize("M,N,k,p,sub,gap,h", CASES)
def test_edit_equals_oracle(M, N, k, p, sub, gap, h):
    print(f"edit {M}x{N} k={k} sub={sub} gap={gap} leaf_rows={h}", flush=True)
    a, b = synth.string_pair(9000 + M + 3 * N, M, N, k=k, p=p)
    d, path = _gpu(a, b, sub, gap, h)
    r = edit.linear(a, b, sub, gap, leaf_rows=h)
    assert d == r["dist"]
    assert path.tolist() == r["path"].tolist()
    if (M + 1) * (N + 1) <= 5e6:
        assert d == edit.full(a, b, sub, gap)[0]


@pytest.mark.parametrize("sub,gap", [(0, 0), (0, 1), (1, 0), (5, 1), (1, 5), (1 << 10, 7)])
def test_edit_cost_corner_cases(sub, gap):
    # free substitutions, free gaps, everything free (every path optimal:
    # the tie rules decide), substitutions dearer than two gaps
    a, b = synth.string_pair(77, 700, 610, k=3, p=0.3)
    d, path = _gpu(a, b, sub, gap, 8)
    r = edit.linear(a, b, sub, gap, leaf_rows=8)
    assert d == r["dist"] == edit.full(a, b, sub, gap)[0]
    assert path.tolist() == r["path"].tolist()


def test_edit_full_size_properties():
    M, N = 200000, 160000
    a, b = synth.string_pair(6, M, N, k=4, p=0.1)
    d, path = _gpu(a, b, 1, 1, 64)
    assert edit.path_cost(a, b, path, 1, 1) == d
    steps = np.diff(path, axis=0)
    assert ((steps >= 0) & (steps <= 1)).all() and (steps.sum(axis=1) >= 1).all()
    assert d >= abs(M - N)
    # prefixes and suffixes of an optimal path are optimal: the cost of the
    # path up to a node equals the distance of the two prefixes
    cost = np.concatenate([[0], np.cumsum([
        (0 if a[i - 1] == b[j - 1] else 1) if (i - pi, j - pj) == (1, 1) else 1
        for (pi, pj), (i, j) in zip(path[:-1].tolist(), path[1:].tolist())])])
    for q in (len(path) // 97, len(path) // 31, len(path) // 19):
        i, j = path[q]
        assert cost[q] == _dist(a[:i], b[:j])
        i2, j2 = path[-1 - q]
        assert cost[-1] - cost[-1 - q] == _dist(a[i2:], b[j2:])


def test_edit_aligner_reuse():
    a, b = synth.string_pair(11, 5000, 4000, k=4, p=0.2)
    a2, b2 = synth.string_pair(12, 5000, 4000, k=4, p=0.4)
    al = dtw.EditAligner(5000, 4000, 64)
    outs = []
    for x, y in ((a, b), (a2, b2), (a, b)):
        al.run(_dev(x), _dev(y), 1, 1)
        n = int(al.plen.item())
        outs.append((int(al.dist.item()), al.path[:n].cpu().numpy().tolist()))
    assert outs[0] == outs[2]
    r = edit.linear(a2, b2, 1, 1, leaf_rows=64)
    assert outs[1] == (r["dist"], r["path"].tolist())


def test_edit_rejects_bad_arguments():
    a, b = _dev(np.zeros(10, np.uint8)), _dev(np.zeros(12, np.uint8))
    for kw in (dict(leaf_rows=1), dict(leaf_rows=65), dict(sub=-1), dict(gap=1 << 21)):
        with pytest.raises(dtw.DtwError):
            dtw.edit_align(a, b, **{"sub": 1, "gap": 1, "leaf_rows": 64, **kw})


# ------------------------------------------------------------------ local alignment score
#
# The device launch of dtw_local_score is switched off: its first launch (the
# 1 x 1 case below) did not finish, and no cause has been shown.  Its kernels
# run to the oracle's results in the CPU model (tests/test_edit_cpu_model.py);
# these tests stay skipped until a cause is found and fixed.

LOCAL_OFF = "dtw_local_score's device launch is switched off: its first launch did not finish on the device, cause not found"


def test_local_score_reports_unsupported():
    # the switched-off entry point checks its arguments and launches nothing
    x = _dev(np.zeros(10, np.uint8))
    with pytest.raises(dtw.DtwError) as e:
        dtw.local_score(x, x, 2, 1, 1)
    assert e.value.status == -8  # DTW_ERR_UNSUPPORTED
    with pytest.raises(dtw.DtwError) as e:
        dtw.local_score(x, x, 0, 1, 1)
    assert e.value.status == -1  # DTW_ERR_INVALID_ARG: a match score below 1



@pytest.mark.skip(reason=LOCAL_OFF)
@pytest.mark.parametrize("M,N,p", [(0, 0, 0.1), (0, 9, 0.1), (9, 0, 0.1), (1, 1, 0.1), (63, 64, 0.3), (257, 300, 0.3),
                                   (1000, 700, 0.2), (5000, 50, 0.1), (50, 20000, 0.1), (2000, 2000, 0.0),
                                   (20000, 16000, 0.1), (60000, 50000, 0.1)])
def test_local_score_equals_oracle(M, N, p):
    print(f"local {M}x{N}", flush=True)
    a, b = synth.string_pair(9500 + M + 3 * N, M, N, k=4, p=p)
    for match, mismatch, gap in ((2, 1, 1), (1, 3, 2)):
        assert dtw.local_score(_dev(a), _dev(b), match, mismatch, gap) == edit.local_score(a, b, match, mismatch, gap)


@pytest.mark.skip(reason=LOCAL_OFF)
def test_local_score_planted_substring():
    # a common substring inside unrelated text, found at its end
    rng = np.random.default_rng(3)
    p = rng.integers(0, 4, 5000).astype(np.uint8)
    u = np.concatenate([rng.integers(10, 14, 30000).astype(np.uint8), p, rng.integers(10, 14, 4000).astype(np.uint8)])
    w = np.concatenate([rng.integers(20, 24, 12000).astype(np.uint8), p, rng.integers(20, 24, 900).astype(np.uint8)])
    assert dtw.local_score(_dev(u), _dev(w), 2, 1, 1) == (10000, 35000, 17000)
    assert edit.local_score(u, w, 2, 1, 1) == (10000, 35000, 17000)


@pytest.mark.skip(reason=LOCAL_OFF)
def test_local_score_reuse_and_bad_arguments():
    a, b = synth.string_pair(31, 3000, 2500, k=4, p=0.2)
    sc = dtw.LocalScorer(3000, 2500)
    outs = []
    for m in (2, 3, 2):
        sc.run(_dev(a), _dev(b), m, 1, 1)
        outs.append(tuple(sc.out.cpu().tolist()))
    assert outs[0] == outs[2] == edit.local_score(a, b, 2, 1, 1)
    assert outs[1] == edit.local_score(a, b, 3, 1, 1)
    x = _dev(np.zeros(10, np.uint8))
    for args in ((0, 1, 1), (2, -1, 1), (2, 1, 1 << 21)):
        with pytest.raises(dtw.DtwError):
            dtw.local_score(x, x, *args)
