"""GPU parity of the cosine frame cost (Sec. 4.1) against the oracle.

FP64 bar: the path equals the oracle's linmdtw path under the cosine cost
on every input, and its textbook path where no tie separates the two (one
case, d = 5 rectified chroma frames, has such ties); the cost agrees within
1e-12 relative.  The FP32 form lies within 1e-5 of the optimum.  The
BF16/FP16 Gram forms are checked against bounds derived from their
arithmetic (below).
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


# ---------------------------------------------------------------- Gram forms
#
# The cosine cost on the matrix-core tile: the frames are normalised in FP64,
# rounded to FP32 and then to bf16 or fp16, and the cost is max(0, 1 - dot)
# with FP32 accumulation.  Two checks, each with a bound derived from that
# arithmetic:
#  * the internal FP32 optimum (cost_lowp) against an FP64 DP over the costs
#    of the same rounded frames: the products of 16-bit values are exact in
#    FP32, so each cell's dot differs from the FP64 one by at most d * 2^-24
#    (unit vectors: the absolute products sum to at most about 1), and the
#    FP32 recurrence adds at most K * 2^-24 relative (K = M + N - 1 cells on
#    any path);
#  * the FP64 cosine cost of the returned path against the oracle's optimum:
#    a path optimal for costs C~ is within 2 * K * max|C~ - C| (plus the FP32
#    slack above) of the optimum for C, with max|C~ - C| measured on the
#    instance.

def _normalise_round(A, kind):
    n = np.sqrt((A * A).sum(axis=1, keepdims=True))
    U = np.divide(A, n, out=np.zeros_like(A), where=n > 0)
    U32 = U.astype(np.float32)
    if kind == "bf16":
        u = U32.view(np.uint32).astype(np.uint64)
        u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    return U32.astype(np.float16).astype(np.float64)


def _dp_optimum(C):
    """Textbook DTW optimum of a cost matrix, anti-diagonal by anti-diagonal."""
    M, N = C.shape
    F = np.full((M, N), np.inf)
    F[0, 0] = C[0, 0]
    for k in range(1, M + N - 1):
        i = np.arange(max(0, k - N + 1), min(M - 1, k) + 1)
        j = k - i
        best = np.full(i.shape, np.inf)
        m = (i > 0) & (j > 0)
        best[m] = F[i[m] - 1, j[m] - 1]
        m = i > 0
        best[m] = np.minimum(best[m], F[i[m] - 1, j[m]])
        m = j > 0
        best[m] = np.minimum(best[m], F[i[m], j[m] - 1])
        F[i, j] = best + C[i, j]
    return F[M - 1, N - 1]


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("M,N,d,m", [(700, 600, 128, 500), (1500, 1300, 64, 64), (900, 1000, 40, 16)])
def test_gram_cosine(dtw, prec, M, N, d, m):
    X, Y = synth.make_pair(12, M + d, M, N, d, "embedding")
    c, p, st = run(dtw, X, Y, precision=prec, min_block=m, dtype=torch.float32)
    assert st["device_error"] == 0
    K = M + N - 1
    assert p.shape[0] <= K and p[0].tolist() == [0, 0] and p[-1].tolist() == [M - 1, N - 1]
    assert np.all(np.diff(p, axis=0) >= 0) and np.all(np.diff(p, axis=0).sum(axis=1) >= 1)
    X32, Y32 = X.astype(np.float32).astype(np.float64), Y.astype(np.float32).astype(np.float64)  # the caller's frames
    assert oracle.path_cost(X32, Y32, p, cost="cosine") == pytest.approx(c, rel=1e-12)
    # (1) the kernels' arithmetic: the FP32 optimum against the FP64 DP on the rounded frames
    Xr, Yr = _normalise_round(X32, prec), _normalise_round(Y32, prec)
    Ct = np.maximum(1.0 - Xr @ Yr.T, 0.0)
    ft = _dp_optimum(Ct)
    u32 = 2.0 ** -24
    assert abs(st["cost_lowp"] - ft) <= K * d * u32 + K * u32 * ft, (st["cost_lowp"], ft)
    # (2) the precision form against the exact optimum
    c_ref, _ = oracle.full(X32, Y32, cost="cosine")
    nx = np.sqrt((X32 * X32).sum(1))
    ny = np.sqrt((Y32 * Y32).sum(1))
    C = np.maximum(1.0 - (X32 @ Y32.T) / np.outer(nx, ny), 0.0)
    e_max = float(np.max(np.abs(Ct - C)))
    c32 = c
    slack = 2 * K * e_max + K * d * u32 + K * u32 * ft
    assert -1e-12 * c_ref <= c32 - c_ref <= slack, (c32, c_ref, slack)
    print(f"{prec} {M}x{N} d={d}: rel err {(c32 - c_ref) / c_ref:.2e} (bound {slack / c_ref:.2e}), "
          f"lowp vs rounded-frame DP {abs(st['cost_lowp'] - ft) / ft:.2e}")
