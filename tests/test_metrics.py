"""The alignment discrepancy of Sec. 4.4, checked on hand-made paths."""
import numpy as np

from paper_2008_02734_amd import metrics


def test_identical_paths_have_zero_error():
    p = np.array([[0, 0], [1, 1], [1, 2], [2, 3]])
    e = metrics.discrepancy(p, p)
    assert e.shape == (8,) and not e.any()


def test_hand_example():
    # path: diagonal (0,0)->(3,3); ref: right along row 0 then down column 3
    p = np.array([[0, 0], [1, 1], [2, 2], [3, 3]])
    ref = np.array([[0, 0], [0, 1], [0, 2], [0, 3], [1, 3], [2, 3], [3, 3]])
    e = metrics.discrepancy(p, ref)
    # row errors: row 0 of ref spans j 0..3 -> 0; row 1 -> |1-3| = 2; row 2 -> 1; row 3 -> 0
    # column errors: column 0 of ref is i = 0 -> 0; column 1 -> |1-0| = 1; column 2 -> 2; column 3 spans 0..3 -> 0
    assert e.tolist() == [0, 2, 1, 0, 0, 1, 2, 0]
    s = metrics.summary(p, ref)
    assert s["max_frames"] == 2 and abs(s["mean_frames"] - 0.75) < 1e-12
    assert s["frac_le_1"] == 0.75 and s["frac_le_2"] == 1.0


def test_symmetry_of_definition():
    rng = np.random.default_rng(3)
    def rand_path(M, N):
        i = j = 0
        cells = [(0, 0)]
        while (i, j) != (M - 1, N - 1):
            moves = [(1, 1), (1, 0), (0, 1)]
            ok = [(di, dj) for di, dj in moves if i + di < M and j + dj < N]
            di, dj = ok[rng.integers(len(ok))]
            i, j = i + di, j + dj
            cells.append((i, j))
        return np.array(cells)
    for _ in range(20):
        a, b = rand_path(30, 25), rand_path(30, 25)
        # transposing both paths swaps the roles of row and column errors
        ea = np.sort(metrics.discrepancy(a, b))
        eb = np.sort(metrics.discrepancy(a[:, ::-1], b[:, ::-1]))
        assert ea.tolist() == eb.tolist()
