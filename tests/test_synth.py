"""Input generators: seeded, deterministic, and shaped as stated."""
import numpy as np
import pytest

from paper_2008_02734_amd import synth


def test_deterministic_per_seed():
    a = synth.make_pair(2, 0, 300, 250, 12, "chroma")
    b = synth.make_pair(2, 0, 300, 250, 12, "chroma")
    c = synth.make_pair(2, 1, 300, 250, 12, "chroma")
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[0], c[0])


@pytest.mark.parametrize("M,N", [(500, 400), (20000, 16000), (1000, 1400), (1400, 1000), (7, 5)])
def test_warp_monotone_with_bounded_slopes(M, N):
    w = synth.warp(np.random.default_rng(1), M, N)
    assert w[0] == 0.0 and w[-1] == M - 1
    s = np.diff(w)
    assert (s >= 0.5 - 1e-9).all() and (s <= 2.0 + 1e-9).all()


@pytest.mark.parametrize("family", ["gaussian_walk", "chroma", "embedding"])
def test_families(family):
    X, Y = synth.make_pair(7, 3, 400, 330, 24, family)
    assert X.shape == (400, 24) and Y.shape == (330, 24)
    assert X.dtype == np.float64 and np.isfinite(X).all() and np.isfinite(Y).all()
    if family in ("chroma", "embedding"):
        assert np.allclose(np.linalg.norm(X, axis=1), 1.0)
        assert np.allclose(np.linalg.norm(Y, axis=1), 1.0)
    if family == "chroma":
        assert (X >= 0).all() and (Y >= 0).all()


def test_batch_shapes_ratio():
    sh = synth.batch_shapes(64)
    assert len(sh) == 64
    for M, N in sh:
        assert 1000 <= M <= 30000 and 1000 <= N <= 30000
        assert 0.7 <= N / M <= 1.4
