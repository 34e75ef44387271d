"""Host-side checks of the C-ABI library (no GPU needed): the shared library
loads, exports every function that include/dtw.h declares, and rejects bad
arguments with the documented status codes before touching the device."""
import ctypes

import pytest

from paper_2008_02734_amd import dtw


def test_library_exports_every_header_symbol():
    L = dtw.lib()
    names = dtw.header_functions()
    assert {"dtw_align", "dtw_align_batched", "dtw_workspace_size", "dtw_diag"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = dtw.lib()
    for code, txt in dtw.STATUS.items():
        assert L.dtw_status_string(code).decode() == txt


def test_workspace_is_linear_in_length():
    # O(M+N) working memory (Sec. 3.2 memory discussion): doubling both sides
    # must not quadruple the workspace.
    a = dtw.workspace_size(20000, 16000, 12)
    b = dtw.workspace_size(40000, 32000, 12)
    assert b < 2.3 * a
    assert dtw.workspace_size(200000, 160000, 12) < 200e6


def _align(L, X=1, M=10, Y=1, N=10, d=12, dt=0, opts=None, ws=1, wsb=1 << 40, cost=1, path=1, cap=None, plen=1):
    o = opts if opts is not None else dtw.make_opts()
    cap = (M + N - 1) if cap is None else cap
    vp = ctypes.c_void_p
    return L.dtw_align(vp(X) if X else None, M, vp(Y) if Y else None, N, d, dt, ctypes.byref(o),
                       vp(ws) if ws else None, wsb, vp(cost) if cost else None, vp(path) if path else None,
                       cap, vp(plen) if plen else None, None, None)


def test_argument_errors_before_any_device_work():
    L = dtw.lib()
    assert _align(L, X=0) == -1
    assert _align(L, Y=0) == -1
    assert _align(L, M=0) == -1
    assert _align(L, N=-3) == -1
    assert _align(L, d=0) == -1
    assert _align(L, dt=7) == -1
    assert _align(L, ws=0) == -1
    assert _align(L, cost=0) == -1
    assert _align(L, cap=18) == -2        # M + N - 1 = 19 needed
    assert _align(L, wsb=16) == -3
    assert _align(L, d=129) == -8         # feature dimension not built
    bad = dtw.make_opts(min_block=2)
    assert _align(L, opts=bad) == -1      # recursion would not terminate
    bad = dtw.make_opts(min_block=2000)
    assert _align(L, opts=bad) == -1
    bad = dtw.make_opts()
    bad.reserved[0] = 1
    assert _align(L, opts=bad) == -1
    bad = dtw.make_opts(precision=9)
    assert _align(L, opts=bad) == -1
    bad = dtw.make_opts(cost=5)
    assert _align(L, opts=bad) == -1      # unknown frame cost
    bad = dtw.make_opts()
    bad.tie_exact = 2
    assert _align(L, opts=bad) == -1      # tie_exact is 0 or 1
    n = ctypes.c_size_t()
    for prec in ("fp32", "bf16", "fp16"):  # tie-exact splits: FP64 only
        o = dtw.make_opts(precision=prec, tie_exact=True)
        assert L.dtw_workspace_size(100, 80, 12, 0, ctypes.byref(o), ctypes.byref(n)) == -8
    o = dtw.make_opts(tie_exact=True)
    assert L.dtw_workspace_size(100, 80, 12, 0, ctypes.byref(o), ctypes.byref(n)) == 0 and n.value > 0
    for prec in ("fp64", "fp32", "bf16", "fp16"):  # every precision takes the cosine cost
        o = dtw.make_opts(precision=prec, cost="cosine")
        assert L.dtw_workspace_size(100, 80, 128, 0, ctypes.byref(o), ctypes.byref(n)) == 0 and n.value > 0


def test_workspace_size_errors():
    L = dtw.lib()
    n = ctypes.c_size_t()
    o = dtw.make_opts()
    assert L.dtw_workspace_size(0, 5, 12, 0, ctypes.byref(o), ctypes.byref(n)) == -1
    assert L.dtw_workspace_size(5, 5, 12, 0, ctypes.byref(o), None) == -1
    assert L.dtw_workspace_size(5, 5, 12, 0, None, ctypes.byref(n)) == 0 and n.value > 0


def test_batched_argument_errors():
    L = dtw.lib()
    o = dtw.make_opts()
    arr = lambda v: (ctypes.c_int64 * len(v))(*v)
    vp = ctypes.c_void_p
    # capacity of pair 1 too small (needs 5 + 4 - 1 = 8)
    rc = L.dtw_align_batched(2, vp(1), arr([0, 3, 8]), vp(1), arr([0, 3, 7]), 4, 0, ctypes.byref(o), vp(1),
                             1 << 40, vp(1), vp(1), arr([0, 5, 12]), vp(1), None, None)
    assert rc == -2
    # empty pair
    rc = L.dtw_align_batched(2, vp(1), arr([0, 3, 3]), vp(1), arr([0, 3, 7]), 4, 0, ctypes.byref(o), vp(1),
                             1 << 40, vp(1), vp(1), arr([0, 5, 12]), vp(1), None, None)
    assert rc == -1


def _noalloc(L, M=10, N=10, d=12, opts=None, cap=None):
    o = opts if opts is not None else dtw.make_opts()
    cap = (M + N - 1) if cap is None else cap
    vp = ctypes.c_void_p
    return L.dtw_align_noalloc(vp(1), M, vp(1), N, d, 0, ctypes.byref(o), vp(1), vp(1), cap, vp(1), None, None)


def test_noalloc_rejects_before_any_device_work():
    L = dtw.lib()
    assert dtw.workspace_size(200000, 160000, 12) > dtw.NOALLOC_SCRATCH_BYTES
    assert _noalloc(L, M=200000, N=160000) == -3      # beyond the fixed array
    assert _noalloc(L, M=0) == -1
    assert _noalloc(L, d=129) == -8
    assert _noalloc(L, cap=18) == -2
    assert _noalloc(L, opts=dtw.make_opts(profile=1)) == -1
    assert "#define DTW_NOALLOC_SCRATCH_BYTES (64u << 20)" in open(dtw.HEADER).read()
    assert dtw.NOALLOC_SCRATCH_BYTES == 64 << 20


def test_edit_and_local_argument_checks_before_any_device_work():
    # every check below returns before a HIP call, so host buffers stand in
    L = dtw.lib()
    n = ctypes.c_size_t()
    i64 = ctypes.c_int64
    # workspace sizing: leaf height within 2..64, sizes within 0..2^30, linear in M + N
    assert L.dtw_edit_workspace_size(100, 80, 1, ctypes.byref(n)) == -1
    assert L.dtw_edit_workspace_size(100, 80, 65, ctypes.byref(n)) == -1
    assert L.dtw_edit_workspace_size(-1, 80, 64, ctypes.byref(n)) == -1
    assert L.dtw_edit_workspace_size(100, 80, 64, None) == -1
    sizes = []
    for M in (10000, 20000, 40000):
        assert L.dtw_edit_workspace_size(M, M, 64, ctypes.byref(n)) == 0
        sizes.append(n.value)
    assert sizes[2] - sizes[1] < 2.2 * (sizes[1] - sizes[0])
    assert sizes[2] < 200 * (40000 + 40000) < 40000 * 40000  # bytes: linear in M + N, never the M x N table
    buf = (ctypes.c_uint8 * 4096)()
    a = ctypes.cast(buf, ctypes.c_void_p)
    d, ln = i64(0), i64(0)
    path = (ctypes.c_int32 * 64)()
    assert L.dtw_edit_workspace_size(10, 12, 8, ctypes.byref(n)) == 0
    ws = n.value
    args = lambda **k: dict(dict(M=10, N=12, sub=1, gap=1, h=8, wsb=ws, cap=23), **k)
    def call(**k):
        c = args(**k)
        return L.dtw_edit_align(a, c["M"], a, c["N"], c["sub"], c["gap"], c["h"], a, c["wsb"],
                                ctypes.byref(d), path, c["cap"], ctypes.byref(ln), None, None)
    assert call(cap=22) == -2                # capacity below M + N + 1 nodes
    assert call(wsb=ws - 1) == -3            # workspace below dtw_edit_workspace_size
    assert call(sub=-1) == -1
    assert call(gap=1 << 21) == -1
    assert call(h=1) == -1
    assert call(sub=1 << 20, M=2000, N=2000) == -1  # (M + N + 1) max(sub, gap) reaches 2^30
    assert L.dtw_edit_align(None, 10, a, 12, 1, 1, 8, a, ws, ctypes.byref(d), path, 23, ctypes.byref(ln), None,
                            None) == -1
    # the local score: argument checks, then DTW_ERR_UNSUPPORTED (its device launch is switched off)
    out = (i64 * 3)()
    assert L.dtw_local_workspace_size(10, 12, ctypes.byref(n)) == 0
    lws = n.value
    assert L.dtw_local_score(a, 10, a, 12, 0, 1, 1, a, lws, out, None) == -1
    assert L.dtw_local_score(a, 10, a, 12, 2, -1, 1, a, lws, out, None) == -1
    assert L.dtw_local_score(a, 10, a, 12, 2, 1, 1, a, lws - 1, out, None) == -3
    assert L.dtw_local_score(a, 10, a, 12, 2, 1, 1, a, lws, out, None) == -8
