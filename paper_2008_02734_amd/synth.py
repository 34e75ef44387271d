"""Seeded synthetic inputs: time-warped feature sequences.

This module holds no DTW arithmetic; it only draws input sequences, so both
the GPU tests and the CPU oracle tests take their inputs from here.

The paper aligns audio features at about 43 frames per second (22050 Hz,
hop 512; Sec. 4.1): 12-d chroma-like DLNC0/CENS frames and ~100-d
MFCC-style frames.  The orchestral recordings are not available, so these
generators stand in for them:

  gaussian_walk   X_0 ~ N(0, I_d), X_t = X_{t-1} + N(0, step^2 I_d)
  chroma_like     AR(1) walk Z_t = rho Z_{t-1} + sqrt(1-rho^2) N(0, I_d),
                  rectified (max(Z, 0)) and L2-normalised per frame; an
                  all-zero frame becomes the constant 1/sqrt(d) frame
  embedding_like  gaussian_walk normalised to unit L2 norm per frame

  warp            random monotone piecewise-linear map w: [0, N-1] -> [0, M-1]
                  with max(4, N // 100) equal segments, slopes drawn
                  U[0.5, 2], rescaled so that w(N-1) = M-1 and clamped back to
                  [0.5, 2] with the excess redistributed over the free
                  segments (always feasible for (M-1)/(N-1) in [0.5, 2])
  Y_t = X(w(t)) (linear interpolation between frames) + N(0, 0.01^2 I_d)
        noise, followed by the family's own normalisation.

Every stream is seeded with numpy's PCG64 through
np.random.default_rng([config_id, item_index]) so streams never collide.
Sequences are generated in float64 and cast by the caller.
"""
from __future__ import annotations

import numpy as np
from scipy.signal import lfilter

NOISE_STD = 0.01
WALK_STEP = 0.1
CHROMA_RHO = 0.99


def rng_for(config_id: int, item: int) -> np.random.Generator:
    return np.random.default_rng([int(config_id), int(item) & 0xFFFFFFFF])


def gaussian_walk(rng, M, d, step=WALK_STEP):
    X = rng.standard_normal((M, d)) * step
    X[0] = rng.standard_normal(d)
    return np.cumsum(X, axis=0)


def _normalise_rows(Z):
    n = np.sqrt(np.sum(Z * Z, axis=1, keepdims=True))
    d = Z.shape[1]
    out = np.where(n > 0, Z / np.where(n > 0, n, 1.0), 1.0 / np.sqrt(d))
    return out


def chroma_like(rng, M, d, rho=CHROMA_RHO):
    eps = rng.standard_normal((M, d)) * np.sqrt(1.0 - rho * rho)
    eps[0] = rng.standard_normal(d)
    # Z_0 = eps_0, Z_t = rho Z_{t-1} + eps_t  (first-order recursive filter)
    Z = lfilter([1.0], [1.0, -rho], eps, axis=0)
    return _normalise_rows(np.maximum(Z, 0.0))


def embedding_like(rng, M, d):
    return _normalise_rows(gaussian_walk(rng, M, d))


def warp(rng, M, N):
    """Monotone piecewise-linear w with w(0)=0, w(N-1)=M-1, slopes in [0.5, 2]."""
    if N < 2:
        return np.zeros(N)
    S = max(4, N // 100)
    S = min(S, N - 1)
    L = (N - 1) / S
    target = (M - 1) / L  # required sum of slopes
    lo, hi = 0.5, 2.0
    if not (lo * S - 1e-9 <= target <= hi * S + 1e-9):
        raise ValueError(f"warp infeasible for M={M}, N={N}")
    s = rng.uniform(lo, hi, size=S)
    s *= target / s.sum()
    for _ in range(200):  # water-filling: clamp and redistribute the excess
        s = np.clip(s, lo, hi)
        gap = target - s.sum()
        if abs(gap) < 1e-12 * max(1.0, target):
            break
        free = (s < hi) if gap > 0 else (s > lo)
        if not free.any():
            break
        s[free] += gap / free.sum()
    knots = np.concatenate([[0.0], np.cumsum(s) * L])
    knots[-1] = M - 1
    t = np.arange(N, dtype=np.float64)
    seg = np.minimum((t / L).astype(np.int64), S - 1)
    w = knots[seg] + (t - seg * L) * s[seg]
    w[-1] = M - 1
    return np.clip(w, 0.0, M - 1)


def resample(X, w):
    i0 = np.floor(w).astype(np.int64)
    i1 = np.minimum(i0 + 1, X.shape[0] - 1)
    f = (w - i0)[:, None]
    return X[i0] * (1.0 - f) + X[i1] * f


def make_pair(config_id, item, M, N, d, family):
    """Return (X, Y) float64: Y is a warped noisy copy of X."""
    rng = rng_for(config_id, item)
    if family == "gaussian_walk":
        X = gaussian_walk(rng, M, d)
        Y = resample(X, warp(rng, M, N)) + rng.standard_normal((N, d)) * NOISE_STD
    elif family == "chroma":
        X = chroma_like(rng, M, d)
        Y = resample(X, warp(rng, M, N)) + rng.standard_normal((N, d)) * NOISE_STD
        Y = _normalise_rows(np.maximum(Y, 0.0))
    elif family == "embedding":
        X = embedding_like(rng, M, d)
        Y = resample(X, warp(rng, M, N)) + rng.standard_normal((N, d)) * NOISE_STD
        Y = _normalise_rows(Y)
    else:
        raise ValueError(family)
    return np.ascontiguousarray(X), np.ascontiguousarray(Y)


def random_pair(seed, M, N, d, kind="normal"):
    """Small unstructured inputs for edge-case tests.

    kind: "normal" (continuous, tie-free with probability 1) or "int3"
    (integer values in {0,1,2}, which make exact ties common).
    """
    rng = np.random.default_rng([9, int(seed)])
    if kind == "normal":
        return rng.standard_normal((M, d)), rng.standard_normal((N, d))
    if kind == "int3":
        return (rng.integers(0, 3, (M, d)).astype(np.float64),
                rng.integers(0, 3, (N, d)).astype(np.float64))
    raise ValueError(kind)


# Workload table: (config id, M, N, d, family).
CONFIG_SHAPES = {
    1: dict(M=500, N=400, d=12, family="gaussian_walk"),
    2: dict(M=20000, N=16000, d=12, family="chroma"),
    3: dict(M=200000, N=160000, d=128, family="embedding"),
}


def config_pair(cfg: int, item: int = 0):
    s = CONFIG_SHAPES[cfg]
    return make_pair(cfg, item, s["M"], s["N"], s["d"], s["family"])


def batch_shapes(n_pairs=512, lo=1000, hi=30000, config_id=4):
    """Log-uniform M in [lo, hi], N by rejection so that N/M lies in [0.7, 1.4]."""
    shapes = []
    for p in range(n_pairs):
        rng = np.random.default_rng([config_id, p, 1])
        while True:
            M = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
            N = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
            if 0.7 <= N / M <= 1.4:
                break
        shapes.append((M, N))
    return shapes


# ----------------------------------------------------------------- strings
#
# Byte strings for the edit-distance path: a is uniform over an alphabet of
# `k` letters (bytes 0..k-1); b copies a through a mutation channel -- at
# each position of a, with probability p/3 each, the letter is replaced by
# a uniform letter, deleted, or preceded by an inserted uniform letter --
# and is then cut to N letters or extended by uniform letters.  With p = 0
# and N = M, b == a.  Seeds: np.random.default_rng([7, seed]).

def string_pair(seed, M, N, k=4, p=0.1):
    rng = np.random.default_rng([7, int(seed)])
    a = rng.integers(0, k, M).astype(np.uint8)
    u = rng.random(M)
    kind = np.where(u < p / 3, 1, np.where(u < 2 * p / 3, 2, np.where(u < p, 3, 0)))
    letters = rng.integers(0, k, M).astype(np.uint8)
    extra = rng.integers(0, k, M).astype(np.uint8)
    keep = kind != 2
    sub = np.where(kind == 1, letters, a)
    # an insertion puts `extra` before the position's own letter
    ins = kind == 3
    lens = keep.astype(np.int64) + ins
    out = np.empty(int(lens.sum()), dtype=np.uint8)
    pos = np.cumsum(lens) - lens
    out[pos[ins]] = extra[ins]
    out[(pos + ins)[keep]] = sub[keep]
    if out.size >= N:
        b = out[:N]
    else:
        b = np.concatenate([out, rng.integers(0, k, N - out.size).astype(np.uint8)])
    return np.ascontiguousarray(a), np.ascontiguousarray(b)
