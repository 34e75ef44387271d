"""CPU oracle for the weighted edit distance -- test infrastructure only.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module; the GPU library shares no source with it.

edit_oracle.c (plain C, int64 costs) holds the textbook table with its
backtrace, the row sweep of one block (forward, or on the reversed block),
and the linear-memory divide and conquer with row splits that the GPU path
follows.  Strings are numpy uint8 arrays; paths are (n, 2) int32 node arrays
from (0, 0) to (M, N).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "edit_oracle.c")
_LIB = os.path.join(_HERE, "libedit_oracle.so")

GCC_CMD = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", _SRC, "-o", _LIB]


def build(force: bool = False) -> str:
    """Compile edit_oracle.c into oracle/libedit_oracle.so and return its path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.run(GCC_CMD, check=True)
    return _LIB


def build_variant(source_text: str, out_path: str) -> str:
    """Compile an edited copy of edit_oracle.c (planted mistakes in tests)."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    cmd = list(GCC_CMD)
    cmd[cmd.index(_SRC)] = src
    cmd[cmd.index(_LIB)] = out_path
    subprocess.run(cmd, check=True)
    return out_path


def source() -> str:
    with open(_SRC) as f:
        return f.read()


def load(path: str):
    L = ctypes.CDLL(path)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    ip = ctypes.POINTER(ctypes.c_int32)
    lp = ctypes.POINTER(ctypes.c_int64)
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    L.edo_full.restype = ctypes.c_int
    L.edo_full.argtypes = [u8, i64, u8, i64, i32, i32, lp, ip, lp, lp]
    L.edo_row.restype = ctypes.c_int
    L.edo_row.argtypes = [u8, u8, i64, i64, i64, i64, i32, i32, ctypes.c_int, lp]
    L.edo_levels.restype = i32
    L.edo_levels.argtypes = [i64, i32]
    L.edo_linear.restype = ctypes.c_int
    L.edo_linear.argtypes = [u8, i64, u8, i64, i32, i32, i32, lp, ip, lp, lp, i64, lp]
    L.edo_local_score.restype = ctypes.c_int
    L.edo_local_score.argtypes = [u8, i64, u8, i64, i32, i32, i32, lp, lp, lp]
    L.edo_path_cost.restype = i64
    L.edo_path_cost.argtypes = [u8, i64, u8, i64, i32, i32, ip, i64]
    return L


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load(build())
    return _lib


def _u8(s):
    if isinstance(s, (bytes, bytearray)):
        s = np.frombuffer(bytes(s), dtype=np.uint8)
    elif isinstance(s, str):
        s = np.frombuffer(s.encode("latin-1"), dtype=np.uint8)
    s = np.ascontiguousarray(np.asarray(s, dtype=np.uint8))
    # a zero-length array still needs a valid pointer
    return s if s.size else np.zeros(1, dtype=np.uint8)[:0].copy()


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def full(a, b, sub: int = 1, gap: int = 1, return_table: bool = False, L=None):
    """Textbook table: (distance, path) or (distance, path, table)."""
    L = L or lib()
    a, b = _u8(a), _u8(b)
    M, N = a.size, b.size
    path = np.zeros((M + N + 1, 2), dtype=np.int32)
    n = ctypes.c_int64(0)
    dist = ctypes.c_int64(0)
    table = np.zeros((M + 1, N + 1), dtype=np.int64) if return_table else None
    rc = L.edo_full(_p(a, ctypes.c_uint8), M, _p(b, ctypes.c_uint8), N, sub, gap, ctypes.byref(dist),
                    _p(path, ctypes.c_int32), ctypes.byref(n),
                    _p(table, ctypes.c_int64) if return_table else None)
    if rc:
        raise MemoryError("edo_full")
    out = (int(dist.value), path[: n.value].copy())
    return out + (table,) if return_table else out


def row(a, b, i0, j0, i1, j1, sub=1, gap=1, rev=False, L=None):
    """Least costs from (i0, j0) to node row i1 (rev=False), or from node row
    i0 to (i1, j1) (rev=True), over columns j0..j1."""
    L = L or lib()
    a, b = _u8(a), _u8(b)
    out = np.zeros(j1 - j0 + 1, dtype=np.int64)
    L.edo_row(_p(a, ctypes.c_uint8), _p(b, ctypes.c_uint8), i0, j0, i1, j1, sub, gap, int(rev),
              _p(out, ctypes.c_int64))
    return out


def levels(M: int, leaf_rows: int, L=None) -> int:
    return int((L or lib()).edo_levels(M, leaf_rows))


def linear(a, b, sub: int = 1, gap: int = 1, leaf_rows: int = 64, pivots: bool = False, L=None):
    """Linear-memory divide and conquer: dict(dist, path[, pivots])."""
    L = L or lib()
    a, b = _u8(a), _u8(b)
    M, N = a.size, b.size
    path = np.zeros((M + N + 1, 2), dtype=np.int32)
    n = ctypes.c_int64(0)
    dist = ctypes.c_int64(0)
    n_piv = ctypes.c_int64(0)
    cap = 2 * max(M, 1) + 4
    piv = np.zeros((cap, 4), dtype=np.int64)
    rc = L.edo_linear(_p(a, ctypes.c_uint8), M, _p(b, ctypes.c_uint8), N, sub, gap, leaf_rows,
                      ctypes.byref(dist), _p(path, ctypes.c_int32), ctypes.byref(n),
                      _p(piv, ctypes.c_int64), cap, ctypes.byref(n_piv))
    if rc == -2:
        raise ValueError("leaf_rows must be >= 2")
    if rc:
        raise MemoryError("edo_linear")
    r = {"dist": int(dist.value), "path": path[: n.value].copy()}
    if pivots:
        r["pivots"] = piv[: min(n_piv.value, cap)].copy()
    return r


def path_cost(a, b, path, sub: int = 1, gap: int = 1, L=None) -> int:
    """Cost of a node path under the move costs, or -1 when it is not a path."""
    L = L or lib()
    a, b = _u8(a), _u8(b)
    p = np.ascontiguousarray(np.asarray(path, dtype=np.int32))
    return int(L.edo_path_cost(_p(a, ctypes.c_uint8), a.size, _p(b, ctypes.c_uint8), b.size, sub, gap,
                               _p(p, ctypes.c_int32), p.shape[0]))


def local_score(a, b, match=2, mismatch=1, gap=1, L=None):
    """Smith-Waterman: (best local score, i_end, j_end), the end cell the first
    maximum of the table in row-major order ((0, 0) when the score is 0)."""
    L = L or lib()
    a, b = _u8(a), _u8(b)
    sc, ie, je = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    if L.edo_local_score(_p(a, ctypes.c_uint8), a.size, _p(b, ctypes.c_uint8), b.size, match, mismatch, gap,
                         ctypes.byref(sc), ctypes.byref(ie), ctypes.byref(je)):
        raise MemoryError("edo_local_score")
    return int(sc.value), int(ie.value), int(je.value)
