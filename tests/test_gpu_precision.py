"""Reduced-precision forms (FP32 Euclidean, BF16 and FP16 Gram cost) against the FP64 oracle.

FP32 form: frame costs and the accumulated-cost recurrence in FP32 on the
VALU; band sums S = F + B - C and the argmin in FP64 (the FP32 values
widened); the returned cost is the FP64 sum of FP64 frame costs along the
returned path.  The gate is the relative error of that cost against the
oracle's optimum, <= 1e-5.  The frame deviation of the path from the FP64
path (Sec. 4.4 discrepancy) is reported.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2008_02734_amd import metrics, synth

pytestmark = pytest.mark.gpu

FP32_REL_TOL = 1e-5


@pytest.fixture(scope="module")
def dtw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_02734_amd import dtw as mod
    mod.lib()
    return mod


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def check_path(p, M, N):
    assert tuple(p[0]) == (0, 0) and tuple(p[-1]) == (M - 1, N - 1)
    steps = {tuple(s) for s in np.diff(p, axis=0).tolist()}
    assert steps <= {(0, 1), (1, 0), (1, 1)}


def fp32_case(dtw, X, Y, m, in_dtype=torch.float64):
    M, N = X.shape[0], Y.shape[0]
    cost, path, st = dtw.align(dev(X, in_dtype), dev(Y, in_dtype), precision="fp32", min_block=m)
    p = path.cpu().numpy()
    check_path(p, M, N)
    Xo = X.astype(np.float64) if in_dtype == torch.float64 else X.astype(np.float32).astype(np.float64)
    Yo = Y.astype(np.float64) if in_dtype == torch.float64 else Y.astype(np.float32).astype(np.float64)
    c_ref, p_ref = oracle.full(Xo, Yo)
    # the returned cost is the FP64 cost of the returned path
    assert abs(cost - oracle.path_cost(Xo, Yo, p)) <= 1e-12 * c_ref
    rel = (cost - c_ref) / c_ref
    assert -1e-12 <= rel <= FP32_REL_TOL, rel
    dev_ = metrics.summary(p, p_ref)
    lowp_rel = abs(st["cost_lowp"] - c_ref) / c_ref
    print(f"M={M} N={N} m={m}: rel cost err {rel:.2e}, internal FP32 cost err {lowp_rel:.2e}, "
          f"frame deviation mean {dev_['mean_frames']:.3f} max {dev_['max_frames']}")
    return rel, dev_, st


def test_fp32_config2_pair(dtw):
    X, Y = synth.config_pair(2)
    rel, dv, st = fp32_case(dtw, X, Y, 500)
    assert st["device_error"] == 0 and st["levels"] >= 5
    assert st["cost_lowp"] > 0


@pytest.mark.parametrize("m", [500, 64, 16])
def test_fp32_config1_pair(dtw, m):
    X, Y = synth.config_pair(1)
    fp32_case(dtw, X, Y, m)


@pytest.mark.parametrize("p", range(4))
def test_fp32_chroma_d24_float_inputs(dtw, p):
    # the batched form's frames: d = 24 chroma-like, FP32 inputs
    M, N = synth.batch_shapes(4, lo=1000, hi=6000)[p]
    X, Y = synth.make_pair(4, p, M, N, 24, "chroma")
    fp32_case(dtw, X.astype(np.float32), Y.astype(np.float32), 500, in_dtype=torch.float32)


@pytest.mark.parametrize("M,N,d", [(3000, 2500, 128), (1500, 1800, 64)])
def test_fp32_wide_embedding(dtw, M, N, d):
    # wide frames on the VALU in FP32 (the Euclidean form at d = 64..128)
    X, Y = synth.make_pair(3, 400 + d, M, N, d, "embedding")
    fp32_case(dtw, X.astype(np.float32), Y.astype(np.float32), 500, in_dtype=torch.float32)


def test_fp32_batched_equals_single(dtw):
    shapes = synth.batch_shapes(6, lo=500, hi=3000)
    Xs, Ys = [], []
    for p, (M, N) in enumerate(shapes):
        X, Y = synth.make_pair(4, 100 + p, M, N, 24, "chroma")
        Xs.append(dev(X.astype(np.float32), torch.float32))
        Ys.append(dev(Y.astype(np.float32), torch.float32))
    costs, paths, st = dtw.align_batched(Xs, Ys, precision="fp32", min_block=500)
    assert st["device_error"] == 0
    for b in range(len(shapes)):
        c1, p1, _ = dtw.align(Xs[b], Ys[b], precision="fp32", min_block=500)
        assert costs[b].item() == c1
        assert torch.equal(paths[b], p1)


# ------------------------------------------------------------------ BF16 Gram form
#
# Frame costs sqrt(max(0, |x|^2 + |y|^2 - 2 x.y)) from frames rounded to bf16
# (dot products on the matrix cores, FP32 accumulation), recurrence in FP32,
# band sums and argmin in FP64; gate: relative cost error <= 1e-2.

BF16_REL_TOL = 1e-2


def bf16_round(a):
    """Round to bf16 (nearest even) through FP32, as the input staging does."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_case(dtw, X, Y, m):
    M, N = X.shape[0], Y.shape[0]
    cost, path, st = dtw.align(dev(X), dev(Y), precision="bf16", min_block=m)
    assert st["device_error"] == 0
    p = path.cpu().numpy()
    check_path(p, M, N)
    c_ref, p_ref = oracle.full(X, Y)
    assert abs(cost - oracle.path_cost(X, Y, p)) <= 1e-12 * c_ref
    rel = (cost - c_ref) / c_ref
    assert -1e-12 <= rel <= BF16_REL_TOL, rel
    dv = metrics.summary(p, p_ref)
    print(f"bf16 M={M} N={N} d={X.shape[1]} m={m}: rel cost err {rel:.2e}, internal cost err "
          f"{abs(st['cost_lowp'] - c_ref) / c_ref:.2e}, frame deviation mean {dv['mean_frames']:.3f} "
          f"max {dv['max_frames']} within 1 frame {dv['frac_le_1']:.4f}")
    return rel, dv, st


@pytest.mark.parametrize("M,N", [(3000, 2500), (6000, 4800)])
def test_bf16_embedding_d128(dtw, M, N):
    X, Y = synth.make_pair(3, M, M, N, 128, "embedding")
    bf16_case(dtw, X, Y, 500)


@pytest.mark.parametrize("d,m", [(20, 16), (64, 500), (100, 64)])
def test_bf16_other_widths(dtw, d, m):
    X, Y = synth.make_pair(3, 1000 + d, 700, 560, d, "embedding")
    bf16_case(dtw, X, Y, m)


def test_bf16_sweep_band_against_gram_reference(dtw):
    # one sweep (Algorithm 1) in the Gram form against an FP64 DP on the Gram
    # costs of the bf16-rounded frames: only FP32 dot/recurrence rounding differs
    M, N, d = 300, 260, 128
    X, Y = synth.make_pair(3, 77, M, N, d, "embedding")
    Xr, Yr = bf16_round(X), bf16_round(Y)
    nx = (Xr * Xr).sum(1)
    ny = (Yr * Yr).sum(1)
    C = np.sqrt(np.maximum(nx[:, None] + ny[None, :] - 2.0 * Xr @ Yr.T, 0.0))
    F = np.full((M, N), np.inf)
    F[0, 0] = C[0, 0]
    for i in range(M):
        for j in range(N):
            if i == 0 and j == 0:
                continue
            best = min(F[i - 1, j - 1] if i and j else np.inf, F[i - 1, j] if i else np.inf,
                       F[i, j - 1] if j else np.inf)
            F[i, j] = best + C[i, j]
    K = M + N - 1
    kstop = (K + 1) // 2
    got = dtw.diag(dev(X), dev(Y), 0, 0, M - 1, N - 1, 0, kstop, precision="bf16").cpu().numpy()
    for q in range(3):
        k = kstop - 2 + q
        for a in range(max(0, k - N + 1), min(M - 1, k) + 1):
            ref = F[a, k - a]
            assert abs(got[q, a] - ref) <= 2e-5 * ref, (q, a, got[q, a], ref)


def test_bf16_batched_equals_single(dtw):
    shapes = [(800, 700), (1500, 1300), (300, 420)]
    Xs, Ys = [], []
    for p, (M, N) in enumerate(shapes):
        X, Y = synth.make_pair(3, 200 + p, M, N, 128, "embedding")
        Xs.append(dev(X.astype(np.float32), torch.float32))
        Ys.append(dev(Y.astype(np.float32), torch.float32))
    costs, paths, st = dtw.align_batched(Xs, Ys, precision="bf16", min_block=500)
    assert st["device_error"] == 0
    for b in range(len(shapes)):
        c1, p1, _ = dtw.align(Xs[b], Ys[b], precision="bf16", min_block=500)
        assert costs[b].item() == c1
        assert torch.equal(paths[b], p1)


# ------------------------------------------------------------------ FP16 Gram form
#
# The same Gram form from frames rounded to fp16 (round to nearest even,
# subnormals kept): eight times finer than bf16 at the same matrix-core rate;
# gate: relative cost error <= 1e-5.

FP16_REL_TOL = 1e-5


def fp16_round(a):
    """Round to fp16 (nearest even, subnormals kept) through FP32, as the input staging does."""
    return np.ascontiguousarray(a, dtype=np.float32).astype(np.float16).astype(np.float64)


@pytest.mark.parametrize("M,N", [(3000, 2500), (6000, 4800)])
def test_fp16_embedding_d128(dtw, M, N):
    X, Y = synth.make_pair(3, M + 1, M, N, 128, "embedding")
    cost, path, st = dtw.align(dev(X), dev(Y), precision="fp16", min_block=500)
    assert st["device_error"] == 0
    p = path.cpu().numpy()
    check_path(p, M, N)
    c_ref, p_ref = oracle.full(X, Y)
    assert abs(cost - oracle.path_cost(X, Y, p)) <= 1e-12 * c_ref
    rel = (cost - c_ref) / c_ref
    assert -1e-12 <= rel <= FP16_REL_TOL, rel
    dv = metrics.summary(p, p_ref)
    print(f"fp16 M={M} N={N}: rel cost err {rel:.2e}, frame deviation mean {dv['mean_frames']:.3f} "
          f"max {dv['max_frames']}")


@pytest.mark.parametrize("scale", [1.0, 3e-4])
def test_fp16_sweep_band_against_gram_reference(dtw, scale):
    # one sweep in the FP16 Gram form against an FP64 DP on the Gram costs of
    # the fp16-rounded frames; scale 3e-4 puts most elements in fp16's
    # subnormal range
    M, N, d = 260, 300, 128
    X, Y = synth.make_pair(3, 78, M, N, d, "embedding")
    X, Y = X * scale, Y * scale
    Xr, Yr = fp16_round(X), fp16_round(Y)
    nx = (Xr * Xr).sum(1)
    ny = (Yr * Yr).sum(1)
    C = np.sqrt(np.maximum(nx[:, None] + ny[None, :] - 2.0 * Xr @ Yr.T, 0.0))
    F = np.full((M, N), np.inf)
    for i in range(M):
        for j in range(N):
            if i == 0 and j == 0:
                F[0, 0] = C[0, 0]
                continue
            best = min(F[i - 1, j - 1] if i and j else np.inf, F[i - 1, j] if i else np.inf,
                       F[i, j - 1] if j else np.inf)
            F[i, j] = best + C[i, j]
    K = M + N - 1
    kstop = (K + 1) // 2
    got = dtw.diag(dev(X), dev(Y), 0, 0, M - 1, N - 1, 0, kstop, precision="fp16").cpu().numpy()
    for q in range(3):
        k = kstop - 2 + q
        for a in range(max(0, k - N + 1), min(M - 1, k) + 1):
            ref = F[a, k - a]
            assert abs(got[q, a] - ref) <= 2e-5 * ref, (q, a, got[q, a], ref)


# ------------------------------------------------------------------ full-size workloads
#
# At the benchmark's sizes the oracle's full table is out of reach for the
# 200000 x 160000 pair, so these check what holds at any size: a valid path,
# its reported cost equal to the oracle's FP64 cost of that path, the exact
# FP64 GPU path no more costly, and the precision form within its bound of
# it.  The batch is checked pair by pair on the pairs the oracle can solve in
# seconds.


def test_long_pair_full_size_precision_forms(dtw):
    X, Y = synth.make_pair(3, 0, 200000, 160000, 128, "embedding")
    M, N = X.shape[0], Y.shape[0]
    Xd, Yd = dev(X), dev(Y)  # FP64 inputs: every form's reported cost is on the same frames
    c64, p64, st64 = dtw.align(Xd, Yd)
    assert st64["device_error"] == 0
    p64 = p64.cpu().numpy()
    check_path(p64, M, N)
    assert abs(c64 - oracle.path_cost(X, Y, p64)) <= 1e-12 * c64
    for prec, tol in (("bf16", BF16_REL_TOL), ("fp16", FP16_REL_TOL)):
        c, p, st = dtw.align(Xd, Yd, precision=prec)
        assert st["device_error"] == 0
        p = p.cpu().numpy()
        check_path(p, M, N)
        assert abs(c - oracle.path_cost(X, Y, p)) <= 1e-12 * c64
        rel = (c - c64) / c64
        assert -1e-12 <= rel <= tol, (prec, rel)
        print(f"{prec} 200000x160000 d=128: rel cost err vs the FP64 path {rel:.2e}")


def test_batch_full_size_fp32_sampled_against_oracle(dtw):
    shapes = synth.batch_shapes(512)
    Xs, Ys = [], []
    for p, (M, N) in enumerate(shapes):
        X, Y = synth.make_pair(4, p, M, N, 24, "chroma")
        Xs.append(X)
        Ys.append(Y)
    costs, paths, st = dtw.align_batched([dev(X.astype(np.float32), torch.float32) for X in Xs],
                                         [dev(Y.astype(np.float32), torch.float32) for Y in Ys], precision="fp32")
    assert st["device_error"] == 0
    costs = costs.cpu().numpy()
    order = np.argsort([M * N for M, N in shapes])
    for b in order[:12]:  # the smallest pairs: the oracle's table in well under a second each
        Xr = Xs[b].astype(np.float32).astype(np.float64)
        Yr = Ys[b].astype(np.float32).astype(np.float64)
        c_ref, _ = oracle.full(Xr, Yr)
        p = paths[b].cpu().numpy()
        check_path(p, *shapes[b])
        assert abs(costs[b] - oracle.path_cost(Xr, Yr, p)) <= 1e-12 * c_ref
        assert -1e-12 <= (costs[b] - c_ref) / c_ref <= FP32_REL_TOL


def test_batch_full_size_fp32_every_pair_against_fp64(dtw):
    # every one of the 512 pairs, at sizes the oracle's table cannot reach in
    # the test: a valid warping path whose reported cost is the oracle's FP64
    # cost of that path, no cheaper than the exact FP64 path of the same
    # batch (its optimum) and within the FP32 tolerance of it; the FP64
    # batch's own costs are the oracle's FP64 costs of its paths
    shapes = synth.batch_shapes(512)
    Xs, Ys = [], []
    for p, (M, N) in enumerate(shapes):
        X, Y = synth.make_pair(4, p, M, N, 24, "chroma")
        Xs.append(X.astype(np.float32).astype(np.float64))
        Ys.append(Y.astype(np.float32).astype(np.float64))
    c32, p32, st32 = dtw.align_batched([dev(X, torch.float32) for X in Xs], [dev(Y, torch.float32) for Y in Ys],
                                       precision="fp32")
    c64, p64, st64 = dtw.align_batched([dev(X) for X in Xs], [dev(Y) for Y in Ys])
    assert st32["device_error"] == 0 and st64["device_error"] == 0
    c32, c64 = c32.cpu().numpy(), c64.cpu().numpy()
    for b, (M, N) in enumerate(shapes):
        q32, q64 = p32[b].cpu().numpy(), p64[b].cpu().numpy()
        check_path(q32, M, N)
        check_path(q64, M, N)
        assert abs(c32[b] - oracle.path_cost(Xs[b], Ys[b], q32)) <= 1e-12 * c64[b]
        assert abs(c64[b] - oracle.path_cost(Xs[b], Ys[b], q64)) <= 1e-12 * c64[b]
        assert -1e-12 <= (c32[b] - c64[b]) / c64[b] <= FP32_REL_TOL, b
