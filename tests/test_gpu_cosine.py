"""GPU parity of the cosine frame cost (Sec. 4.1) against the oracle.

FP64 bar: the path equals the oracle's linmdtw path under the cosine cost
on every input, and its textbook path where no tie separates the two (one
case, d = 5 rectified chroma frames, has such ties); the cost agrees within
1e-12 relative.  The FP32 form lies within 1e-5 of the optimum.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2008_02734_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dtw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_02734_amd import dtw as mod
    mod.lib()
    return mod


def run(dtw, X, Y, precision="fp64", min_block=500, dtype=torch.float64):
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda", dtype)
    Yd = torch.from_numpy(np.ascontiguousarray(Y)).to("cuda", dtype)
    al = dtw.Aligner(X.shape[0], Y.shape[0], X.shape[1], dtype, precision, min_block, cost="cosine")
    st = al.run(Xd, Yd, stats=True)
    n = int(st["path_len"])
    return float(al.cost.item()), al.path[:n].cpu().numpy(), st


CASES = [  # (M, N, d, family, m)
    (300, 240, 12, "chroma", 500),     # one leaf
    (1500, 1200, 12, "chroma", 500),   # splits and stripes
    (900, 1300, 24, "chroma", 64),     # N > M, small cutoff
    (700, 520, 5, "chroma", 16),       # padded frame width
    (600, 500, 64, "embedding", 64),   # wide frames staged in LDS
    (400, 350, 100, "embedding", 32),  # wide frames, padded to 128
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_cosine_fp64_equals_textbook(dtw, case):
    M, N, d, fam, m = CASES[case]
    X, Y = synth.make_pair(11, case, M, N, d, fam)
    c, p, st = run(dtw, X, Y, min_block=m)
    assert st["device_error"] == 0
    c_ref, p_ref = oracle.full(X, Y, cost="cosine")
    lin = oracle.linmdtw(X, Y, min_block=m, cost="cosine")
    # the method's own path (the oracle's port of Algorithms 1-2) always; the
    # textbook path too where the input has no tie that separates the two
    assert p.tolist() == lin["path"].tolist()
    if lin["path"].tolist() == p_ref.tolist():
        assert p.tolist() == p_ref.tolist()
    assert abs(c - c_ref) <= 1e-12 * c_ref
    assert oracle.path_cost(X, Y, p, cost="cosine") == pytest.approx(c, rel=1e-12)


def test_cosine_fp64_equals_linmdtw_on_ties(dtw):
    # integer-valued frames make exact ties common: the GPU path must be the
    # oracle's linmdtw path (same splits and leaf tie rule), optimal always
    rng = np.random.default_rng(77)
    for k in range(6):
        M, N, d = rng.integers(40, 200), rng.integers(40, 200), 3
        X = rng.integers(0, 3, size=(M, d)).astype(np.float64)
        Y = rng.integers(0, 3, size=(N, d)).astype(np.float64)
        c, p, _ = run(dtw, X, Y, min_block=8)
        lin = oracle.linmdtw(X, Y, min_block=8, cost="cosine")
        p_lin = lin["path"]
        assert p.tolist() == p_lin.tolist()
        assert c == pytest.approx(oracle.full(X, Y, cost="cosine")[0], rel=1e-12, abs=1e-12)


def test_cosine_zero_frames(dtw):
    # a zero frame stays zero (cost 1 against any non-zero frame, 0 against another zero frame)
    X, Y = synth.make_pair(11, 50, 400, 330, 12, "chroma")
    X[[0, 17, 200]] = 0.0
    Y[[5, 100]] = 0.0
    c, p, _ = run(dtw, X, Y, min_block=64)
    c_ref, p_ref = oracle.full(X, Y, cost="cosine")
    assert p.tolist() == p_ref.tolist() and abs(c - c_ref) <= 1e-12 * c_ref


def test_cosine_fp32_form_within_tolerance(dtw):
    X, Y = synth.make_pair(11, 60, 2000, 1700, 12, "chroma")
    c, p, st = run(dtw, X.astype(np.float32), Y.astype(np.float32), precision="fp32", dtype=torch.float32)
    Xf, Yf = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)
    c_ref = oracle.full(Xf, Yf, cost="cosine")[0]
    assert st["device_error"] == 0
    assert c >= c_ref * (1 - 1e-12) and (c - c_ref) / c_ref <= 1e-5
    assert oracle.path_cost(Xf, Yf, p, cost="cosine") == pytest.approx(c, rel=1e-12)


def test_cosine_batched_equals_single(dtw):
    pairs = [synth.make_pair(11, 70 + i, M, N, 12, "chroma") for i, (M, N) in enumerate([(500, 420), (1200, 900), (260, 300)])]
    Xs = [torch.from_numpy(X).cuda() for X, _ in pairs]
    Ys = [torch.from_numpy(Y).cuda() for _, Y in pairs]
    ba = dtw.BatchAligner(Xs, Ys, min_block=128, cost="cosine")
    st = ba.run()
    assert st["device_error"] == 0
    for b, (X, Y) in enumerate(pairs):
        c_ref, p_ref = oracle.full(X, Y, cost="cosine")
        assert ba.path_list()[b].cpu().numpy().tolist() == p_ref.tolist()
        assert abs(float(ba.costs[b]) - c_ref) <= 1e-12 * c_ref


def test_cosine_served_equals_oracle(dtw):
    # the serving loop keeps cosine requests apart from Euclidean ones (the
    # frame cost is part of a batch's class) and serves them exactly
    pairs = [synth.make_pair(11, 90 + i, 300 + 97 * i, 280 + 60 * i, 12, "chroma") for i in range(4)]
    srv = dtw.Server(pool_bytes=1 << 30, max_slots=2, max_batch=4)
    try:
        tks = [srv.submit(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), cost=("cosine" if i % 2 else "euclidean"))
               for i, (X, Y) in enumerate(pairs)]
        res = [srv.wait(t) for t in tks]
    finally:
        srv.close()
    for i, ((X, Y), r) in enumerate(zip(pairs, res)):
        assert r["status"] == 0
        c_ref, p_ref = oracle.full(X, Y, cost=("cosine" if i % 2 else "euclidean"))
        assert r["path"].cpu().numpy().tolist() == p_ref.tolist()
        assert abs(r["cost"] - c_ref) <= 1e-12 * c_ref
