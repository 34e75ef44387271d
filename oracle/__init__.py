"""CPU oracle for exact DTW -- test infrastructure, not part of the product.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  The GPU library never calls it, and it shares no
source with the GPU library (no kernels, headers, helpers or tables).

Contents:
  dtw_oracle.c  plain FP64 C: frame cost, textbook full-table DTW with
                backpointers and backtrace (Sec. 2.1), DiagDTW (Algorithm 1),
                linmdtw (Algorithm 2);
  brute.py      enumeration of every warping path for M, N <= 8 (and of
                every edit-distance lattice path for M, N <= 7);
  edit_oracle.c, edit.py
                the weighted edit distance: textbook table and backtrace,
                and its linear-memory divide and conquer (own library).

This module builds the C file with gcc (floating-point contraction off) and
wraps it with ctypes.  All arrays are numpy float64 / int32 on the host.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dtw_oracle.c")
_LIB = os.path.join(_HERE, "libdtw_oracle.so")

GCC_CMD = [
    "gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
    "-fno-fast-math", "-Wall", "-Wextra", _SRC, "-o", _LIB, "-lm",
]


def build(force: bool = False) -> str:
    """Compile the oracle into oracle/libdtw_oracle.so and return its path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.run(GCC_CMD, check=True)
    return _LIB


_lib = None


def load(path: str):
    """Load a compiled oracle library from ``path`` and declare its signatures."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lp = ctypes.POINTER(ctypes.c_int64)
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    L.dtwo_set_cost.restype = ctypes.c_int
    L.dtwo_set_cost.argtypes = [i32]
    L.dtwo_frame_cost.restype = ctypes.c_double
    L.dtwo_frame_cost.argtypes = [dp, dp, i32]
    L.dtwo_full.restype = ctypes.c_int
    L.dtwo_full.argtypes = [dp, i64, dp, i64, i32, dp, ip, i64, lp, dp]
    for name in ("dtwo_full_f32", "dtwo_full_left_first"):
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = [dp, i64, dp, i64, i32, dp, ip, i64, lp]
    L.dtwo_diag.restype = ctypes.c_int
    L.dtwo_diag.argtypes = [dp, dp, i32, i64, i64, i64, i64, i32, i64, dp]
    L.dtwo_linmdtw.restype = ctypes.c_int
    L.dtwo_linmdtw.argtypes = [dp, i64, dp, i64, i32, i32, dp, ip, i64, lp, dp, lp, ip, i64, lp]
    L.dtwo_path_cost.restype = ctypes.c_double
    L.dtwo_path_cost.argtypes = [dp, i64, dp, i64, i32, ip, i64]
    L.dtwo_tie_pivot.restype = ctypes.c_int
    L.dtwo_tie_pivot.argtypes = [dp, dp, i32, i64, i64, i64, i64, ctypes.c_double, lp, lp, dp]
    L.dtwo_linmdtw_tie.restype = ctypes.c_int
    L.dtwo_linmdtw_tie.argtypes = [dp, i64, dp, i64, i32, i32, dp, ip, i64, lp, lp, ip, i64, lp]
    return L


def build_variant(source_text: str, out_path: str) -> str:
    """Compile an edited copy of the oracle source (used to plant mistakes in
    tests and check that the pins catch them).  Returns the library path."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    cmd = list(GCC_CMD)
    cmd[cmd.index(_SRC)] = src
    cmd[cmd.index(_LIB)] = out_path
    cmd.insert(1, "-I" + _HERE)
    subprocess.run(cmd, check=True)
    return out_path


def source() -> str:
    with open(_SRC) as f:
        return f.read()


def lib():
    global _lib
    if _lib is None:
        _lib = load(build())
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _as2d(X):
    X = _f64(X)
    if X.ndim == 1:
        X = X[:, None]
    return np.ascontiguousarray(X)


# Frame cost kinds of dtwo_set_cost (Sec. 4.1).
COSTS = {"euclidean": 0, "cosine": 1}


class _CostScope:
    """Select a frame cost for the calls inside a `with` block, then restore
    the Euclidean default."""

    def __init__(self, L, cost):
        self.L, self.kind = L, COSTS[cost]

    def __enter__(self):
        if self.L.dtwo_set_cost(self.kind) != 0:
            raise ValueError(f"unknown cost kind {self.kind}")
        return self.L

    def __exit__(self, *exc):
        self.L.dtwo_set_cost(0)
        return False


def frame_cost(x, y, L=None, cost="euclidean") -> float:
    x, y = _f64(x).ravel(), _f64(y).ravel()
    with _CostScope(L or lib(), cost) as lb:
        return lb.dtwo_frame_cost(_dp(x), _dp(y), x.size)


def full(X, Y, return_table: bool = False, L=None, cost="euclidean"):
    """Textbook DTW: returns (cost, path[K,2] int32[, F table M x N])."""
    kind = cost
    X, Y = _as2d(X), _as2d(Y)
    M, d = X.shape
    N = Y.shape[0]
    assert Y.shape[1] == d
    cost = ctypes.c_double()
    path = np.zeros((M + N - 1, 2), dtype=np.int32)
    n = ctypes.c_int64()
    F = np.zeros((M, N), dtype=np.float64) if return_table else None
    with _CostScope(L or lib(), kind) as lb:
        rc = lb.dtwo_full(_dp(X), M, _dp(Y), N, d, ctypes.byref(cost), _ip(path), M + N - 1,
                          ctypes.byref(n), _dp(F) if F is not None else None)
    if rc:
        raise RuntimeError(f"dtwo_full failed: {rc}")
    out = (cost.value, path[: n.value].copy())
    return out + (F,) if return_table else out


def _full_variant(name, X, Y, L, kind="euclidean"):
    X, Y = _as2d(X), _as2d(Y)
    M, d = X.shape
    N = Y.shape[0]
    assert Y.shape[1] == d
    cost = ctypes.c_double()
    path = np.zeros((M + N - 1, 2), dtype=np.int32)
    n = ctypes.c_int64()
    with _CostScope(L or lib(), kind) as lb:
        rc = getattr(lb, name)(_dp(X), M, _dp(Y), N, d, ctypes.byref(cost), _ip(path), M + N - 1,
                               ctypes.byref(n))
    if rc:
        raise RuntimeError(f"{name} failed: {rc}")
    return cost.value, path[: n.value].copy()


def full_f32(X, Y, L=None):
    """Textbook DTW entirely in binary32 (Sec. 4.2's 32-bit CPU reference):
    returns (float optimum as a Python float, path[K,2] int32)."""
    return _full_variant("dtwo_full_f32", X, Y, L)


def full_left_first(X, Y, L=None, cost="euclidean"):
    """Textbook DTW in FP64 with LEFT, then UP, then DIAG winning ties (the
    second tie rule of Sec. 4.2): returns (cost, path[K,2] int32)."""
    return _full_variant("dtwo_full_left_first", X, Y, L, cost)


def diag(X, Y, i0, j0, i1, j1, reverse: bool, kstop: int, L=None, cost="euclidean"):
    """DiagDTW on a block; returns a (3, Mb) array of diagonals kstop-2..kstop by local row."""
    X, Y = _as2d(X), _as2d(Y)
    Mb = i1 - i0 + 1
    out = np.zeros((3, Mb), dtype=np.float64)
    with _CostScope(L or lib(), cost) as lb:
        rc = lb.dtwo_diag(_dp(X), _dp(Y), X.shape[1], i0, j0, i1, j1, int(reverse), kstop, _dp(out))
    if rc:
        raise RuntimeError(f"dtwo_diag failed: {rc}")
    return out


def linmdtw(X, Y, min_block: int = 500, pivots_cap: int = 1 << 16, L=None, cost="euclidean"):
    """linmdtw: returns dict(cost, path, s_min, cells, pivots)."""
    X, Y = _as2d(X), _as2d(Y)
    M, d = X.shape
    N = Y.shape[0]
    kind, cost = cost, ctypes.c_double()
    smin = ctypes.c_double()
    cells = ctypes.c_int64()
    n = ctypes.c_int64()
    npiv = ctypes.c_int64()
    path = np.zeros((M + N - 1, 2), dtype=np.int32)
    piv = np.zeros((pivots_cap, 2), dtype=np.int32)
    with _CostScope(L or lib(), kind) as lb:
        rc = lb.dtwo_linmdtw(_dp(X), M, _dp(Y), N, d, min_block, ctypes.byref(cost), _ip(path),
                             M + N - 1, ctypes.byref(n), ctypes.byref(smin), ctypes.byref(cells),
                             _ip(piv), pivots_cap, ctypes.byref(npiv))
    if rc:
        raise RuntimeError(f"dtwo_linmdtw failed: {rc}")
    return dict(cost=cost.value, path=path[: n.value].copy(), s_min=smin.value,
                cells=cells.value, pivots=piv[: npiv.value].copy())


def tie_pivot(X, Y, i0, j0, i1, j1, f0, L=None, cost="euclidean"):
    """One tie-exact split of a block whose origin holds f0: (row, diagonal,
    accumulated cost) of the pivot, in the block's local coordinates."""
    X, Y = _as2d(X), _as2d(Y)
    a, k, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    with _CostScope(L or lib(), cost) as lb:
        rc = lb.dtwo_tie_pivot(_dp(X), _dp(Y), X.shape[1], i0, j0, i1, j1, float(f0), ctypes.byref(a),
                               ctypes.byref(k), ctypes.byref(f))
    if rc:
        raise RuntimeError(f"dtwo_tie_pivot failed: {rc}")
    return a.value, k.value, f.value


def linmdtw_tie(X, Y, min_block: int = 500, pivots_cap: int = 1 << 16, L=None, cost="euclidean"):
    """Tie-exact divide and conquer: returns dict(cost, path, cells, pivots)."""
    X, Y = _as2d(X), _as2d(Y)
    M, d = X.shape
    N = Y.shape[0]
    c = ctypes.c_double()
    cells, n, npiv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    path = np.zeros((M + N - 1, 2), dtype=np.int32)
    piv = np.zeros((pivots_cap, 2), dtype=np.int32)
    with _CostScope(L or lib(), cost) as lb:
        rc = lb.dtwo_linmdtw_tie(_dp(X), M, _dp(Y), N, d, min_block, ctypes.byref(c), _ip(path), M + N - 1,
                                 ctypes.byref(n), ctypes.byref(cells), _ip(piv), pivots_cap, ctypes.byref(npiv))
    if rc:
        raise RuntimeError(f"dtwo_linmdtw_tie failed: {rc}")
    return dict(cost=c.value, path=path[: n.value].copy(), cells=cells.value, pivots=piv[: npiv.value].copy())


def path_cost(X, Y, path, L=None, cost="euclidean") -> float:
    X, Y = _as2d(X), _as2d(Y)
    p = np.ascontiguousarray(np.asarray(path, dtype=np.int32))
    with _CostScope(L or lib(), cost) as lb:
        return lb.dtwo_path_cost(_dp(X), X.shape[0], _dp(Y), Y.shape[0], X.shape[1], _ip(p), p.shape[0])
