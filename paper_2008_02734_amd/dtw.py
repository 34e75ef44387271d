"""ctypes binding of libdtw_hip.so (C-ABI in include/dtw.h).

Argument marshalling only: every step of the alignment runs in the HIP
library.  PyTorch supplies device memory (inputs, outputs, workspace) and the
current stream.  There is no CPU fallback: loading fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdtw_hip.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "dtw.h")

DTW_F64, DTW_F32 = 0, 1
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3}
STATUS = {0: "ok", -1: "invalid argument", -2: "path capacity too small", -3: "workspace too small",
          -4: "non-finite input", -5: "HIP runtime error", -6: "not ready", -7: "unknown ticket",
          -8: "unsupported dimension or mode", -9: "device-side consistency check failed"}


class DtwError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({status})")


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("min_block", ctypes.c_int32),
                ("validate_finite", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("wait_limit_us", ctypes.c_int32), ("cost", ctypes.c_int32), ("tie_exact", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 1)]


class Stats(ctypes.Structure):
    _fields_ = [("s_min", ctypes.c_double), ("cost_lowp", ctypes.c_double),
                ("cells_processed", ctypes.c_int64), ("path_len", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("sweep_cells", ctypes.c_int64),
                ("leaf_cells", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("leaves", ctypes.c_int32), ("device_error", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3), ("ms_sweep", ctypes.c_double),
                ("ms_split", ctypes.c_double), ("ms_plan", ctypes.c_double),
                ("ms_leaf", ctypes.c_double), ("ms_other", ctypes.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None


def header_functions():
    """Names of the functions declared in include/dtw.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:dtw_status|void|const char\*|int32_t)\s+(dtw_\w+)\s*\(", txt, re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.dtw_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.dtw_graph_count.restype = i32
        L.dtw_graph_count.argtypes = []
        L.dtw_default_opts.restype = None
        L.dtw_status_string.argtypes = [i32]
        L.dtw_status_string.restype = ctypes.c_char_p
        L.dtw_last_hip_error.restype = i32
        L.dtw_workspace_size.argtypes = [i64, i64, i32, i32, ctypes.POINTER(Opts), ctypes.POINTER(sz)]
        L.dtw_workspace_size.restype = i32
        L.dtw_align.argtypes = [vp, i64, vp, i64, i32, i32, ctypes.POINTER(Opts), vp, sz, vp, vp, i64, vp,
                                ctypes.POINTER(Stats), vp]
        L.dtw_align.restype = i32
        L.dtw_align_noalloc.argtypes = [vp, i64, vp, i64, i32, i32, ctypes.POINTER(Opts), vp, vp, i64, vp,
                                        ctypes.POINTER(Stats), vp]
        L.dtw_align_noalloc.restype = i32
        L.dtw_diag.argtypes = [vp, vp, i32, i32, i64, i64, i64, i64, i32, i64, i32, vp, sz, vp, vp]
        L.dtw_diag.restype = i32
        L.dtw_device_error.argtypes = [vp, ctypes.POINTER(i32), vp]
        L.dtw_device_error.restype = i32
        L.dtw_workspace_size_batched.argtypes = [i32, i64p, i64p, i32, i32, ctypes.POINTER(Opts),
                                                 ctypes.POINTER(sz)]
        L.dtw_workspace_size_batched.restype = i32
        L.dtw_align_batched.argtypes = [i32, vp, i64p, vp, i64p, i32, i32, ctypes.POINTER(Opts), vp, sz, vp,
                                        vp, i64p, vp, ctypes.POINTER(Stats), vp]
        L.dtw_align_batched.restype = i32
        L.dtw_edit_workspace_size.argtypes = [i64, i64, i32, ctypes.POINTER(sz)]
        L.dtw_edit_workspace_size.restype = i32
        L.dtw_edit_align.argtypes = [vp, i64, vp, i64, i32, i32, i32, vp, sz, vp, vp, i64, vp,
                                     ctypes.POINTER(EditStats), vp]
        L.dtw_edit_align.restype = i32
        L.dtw_local_workspace_size.argtypes = [i64, i64, ctypes.POINTER(sz)]
        L.dtw_local_workspace_size.restype = i32
        L.dtw_local_score.argtypes = [vp, i64, vp, i64, i32, i32, i32, vp, sz, vp, vp]
        L.dtw_local_score.restype = i32
        _lib = L
    return _lib


COST = {"euclidean": 0, "cosine": 1}


def make_opts(precision="fp64", min_block=500, validate_finite=False, profile=False, wait_limit_us=0,
              cost="euclidean", tie_exact=False):
    o = Opts()
    lib().dtw_default_opts(ctypes.byref(o))
    o.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    o.min_block = int(min_block)
    o.validate_finite = 1 if validate_finite else 0
    o.profile = int(profile) if not isinstance(profile, bool) else (1 if profile else 0)
    o.wait_limit_us = int(wait_limit_us)
    o.tie_exact = 1 if tie_exact else 0
    if isinstance(cost, str):
        o.cost = COST[cost]
    elif isinstance(cost, int):
        o.cost = cost
    else:
        raise TypeError(f"cost must be a name or a dtw_cost value, not {type(cost).__name__}")
    return o


def _check(rc, what):
    if rc != 0:
        raise DtwError(rc, what)


class DeviceError(DtwError):
    """A call's kernels recorded a device-side error (dtw_device_error)."""

    def __init__(self, code, what=""):
        self.code = code
        super().__init__(-9, f"{what}: device error {code}")


def graph_count():
    """Graphs the library keeps for replaying repeated dtw_align calls."""
    return int(lib().dtw_graph_count())


def device_error(ws, stream=None):
    """Device error code of the latest call that ran in workspace `ws` (a device
    tensor); synchronises the stream."""
    code = ctypes.c_int32()
    _check(lib().dtw_device_error(ctypes.c_void_p(ws.data_ptr()), ctypes.byref(code), _stream_ptr(stream)),
           "dtw_device_error")
    return code.value


def _dtype_code(t):
    if t.dtype == torch.float64:
        return DTW_F64
    if t.dtype == torch.float32:
        return DTW_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("inputs must be contiguous device tensors")
    return ctypes.c_void_p(t.data_ptr())


def workspace_size(M, N, d, dtype=torch.float64, precision="fp64", min_block=500, cost="euclidean",
                   tie_exact=False):
    o = make_opts(precision, min_block, cost=cost, tie_exact=tie_exact)
    n = ctypes.c_size_t()
    code = DTW_F64 if dtype == torch.float64 else DTW_F32
    _check(lib().dtw_workspace_size(M, N, d, code, ctypes.byref(o), ctypes.byref(n)), "dtw_workspace_size")
    return n.value


class Aligner:
    """Reusable buffers for repeated alignments of one problem shape."""

    def __init__(self, M, N, d, dtype=torch.float64, precision="fp64", min_block=500, device="cuda",
                 wait_limit_us=0, cost="euclidean", tie_exact=False):
        self.M, self.N, self.d, self.dtype = M, N, d, dtype
        self.opts = make_opts(precision, min_block, wait_limit_us=wait_limit_us, cost=cost, tie_exact=tie_exact)
        self.ws_bytes = workspace_size(M, N, d, dtype, precision, min_block, cost, tie_exact)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.cost = torch.empty(1, dtype=torch.float64, device=device)
        self.cap = M + N - 1
        self.path = torch.empty((self.cap, 2), dtype=torch.int32, device=device)
        self.plen = torch.empty(1, dtype=torch.int64, device=device)

    def run(self, X, Y, stats=False, stream=None, check=True):
        """One alignment into self.cost / self.path / self.plen.  With stats the
        call synchronises and returns the stats dict; otherwise it is
        asynchronous unless `check` is set, which waits for the call and
        raises DeviceError if its kernels recorded a device-side error."""
        st = Stats()
        rc = lib().dtw_align(_dev(X), self.M, _dev(Y), self.N, self.d, _dtype_code(X), ctypes.byref(self.opts),
                             ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                             ctypes.c_void_p(self.cost.data_ptr()), ctypes.c_void_p(self.path.data_ptr()),
                             self.cap, ctypes.c_void_p(self.plen.data_ptr()),
                             ctypes.byref(st) if stats else None, _stream_ptr(stream))
        if rc == -9 and stats and st.device_error:
            raise DeviceError(st.device_error, "dtw_align")
        _check(rc, "dtw_align")
        if not stats and check:
            code = device_error(self.ws, stream)
            if code:
                raise DeviceError(code, "dtw_align")
        return st.to_dict() if stats else None


def align(X, Y, precision="fp64", min_block=500, validate_finite=False, stream=None, wait_limit_us=0,
          cost="euclidean", tie_exact=False):
    """Optimal warping path of X (M x d) and Y (N x d), device tensors.

    Returns (cost: float, path: int32 tensor [K, 2] on the device, stats: dict).
    Raises DeviceError when the call's kernels recorded a device-side error.
    """
    if X.dtype != Y.dtype or X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
        raise ValueError("X and Y must be 2-D with equal dtype and feature dimension")
    M, d = X.shape
    N = Y.shape[0]
    al = Aligner(M, N, d, X.dtype, precision, min_block, device=X.device, wait_limit_us=wait_limit_us, cost=cost,
                 tie_exact=tie_exact)
    al.opts.validate_finite = 1 if validate_finite else 0
    st = al.run(X, Y, stats=True, stream=stream)
    n = int(st["path_len"])
    return float(al.cost.item()), al.path[:n], st


NOALLOC_SCRATCH_BYTES = 64 << 20  # DTW_NOALLOC_SCRATCH_BYTES of include/dtw.h


def align_noalloc(X, Y, cost, path, plen, precision="fp64", min_block=500, stats=False, stream=None):
    """dtw_align_noalloc: the alignment of X and Y into the caller's device
    tensors cost (1 float64), path ([>= M+N-1, 2] int32) and plen (1 int64),
    with the library's own fixed device array as the workspace.  Returns the
    stats dict when `stats` is set (the call then synchronises), else None."""
    if X.dtype != Y.dtype or X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
        raise ValueError("X and Y must be 2-D with equal dtype and feature dimension")
    M, d = X.shape
    N = Y.shape[0]
    o = make_opts(precision, min_block)
    st = Stats()
    rc = lib().dtw_align_noalloc(_dev(X), M, _dev(Y), N, d, _dtype_code(X), ctypes.byref(o), _dev(cost),
                                 _dev(path), path.shape[0], _dev(plen), ctypes.byref(st) if stats else None,
                                 _stream_ptr(stream))
    if rc == -9 and stats and st.device_error:
        raise DeviceError(st.device_error, "dtw_align_noalloc")
    _check(rc, "dtw_align_noalloc")
    return st.to_dict() if stats else None


class BatchAligner:
    """Reusable packed inputs and buffers for repeated batched alignments of
    one fixed set of pairs (dtw_align_batched)."""

    def __init__(self, Xs, Ys, precision="fp64", min_block=500, profile=False, cost="euclidean", tie_exact=False):
        self.B = len(Xs)
        dev = Xs[0].device
        self.d = Xs[0].shape[1]
        xo, yo, po = [0], [0], [0]
        for X, Y in zip(Xs, Ys):
            xo.append(xo[-1] + X.shape[0])
            yo.append(yo[-1] + Y.shape[0])
            po.append(po[-1] + X.shape[0] + Y.shape[0] - 1)
        self.po = po
        self.Xp = torch.cat(list(Xs)).contiguous()
        self.Yp = torch.cat(list(Ys)).contiguous()
        arr = lambda v: (ctypes.c_int64 * len(v))(*v)
        self.xo_a, self.yo_a, self.po_a = arr(xo), arr(yo), arr(po)
        self.opts = make_opts(precision, min_block, profile=profile, cost=cost, tie_exact=tie_exact)
        n = ctypes.c_size_t()
        _check(lib().dtw_workspace_size_batched(self.B, self.xo_a, self.yo_a, self.d, _dtype_code(self.Xp),
                                                ctypes.byref(self.opts), ctypes.byref(n)),
               "dtw_workspace_size_batched")
        self.ws_bytes = n.value
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=dev)
        self.costs = torch.empty(self.B, dtype=torch.float64, device=dev)
        self.paths = torch.empty((po[-1], 2), dtype=torch.int32, device=dev)
        self.lens = torch.empty(self.B, dtype=torch.int64, device=dev)

    def run(self, stream=None):
        st = Stats()
        rc = lib().dtw_align_batched(self.B, _dev(self.Xp), self.xo_a, _dev(self.Yp), self.yo_a, self.d,
                                     _dtype_code(self.Xp), ctypes.byref(self.opts),
                                     ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                     ctypes.c_void_p(self.costs.data_ptr()), ctypes.c_void_p(self.paths.data_ptr()),
                                     self.po_a, ctypes.c_void_p(self.lens.data_ptr()), ctypes.byref(st),
                                     _stream_ptr(stream))
        _check(rc, "dtw_align_batched")
        return st.to_dict()

    def path_list(self):
        lens_h = self.lens.tolist()
        return [self.paths[self.po[b]:self.po[b] + lens_h[b]] for b in range(self.B)]


def align_batched(Xs, Ys, precision="fp64", min_block=500, stream=None, cost="euclidean", tie_exact=False):
    """Align B independent pairs in one call.  Returns (costs [B] float64 tensor,
    list of path tensors, stats dict)."""
    ba = BatchAligner(Xs, Ys, precision, min_block, cost=cost, tie_exact=tie_exact)
    st = ba.run(stream)
    return ba.costs, ba.path_list(), st


def diag(X, Y, i0, j0, i1, j1, reverse, kstop, precision="fp64", stream=None):
    """DiagDTW sweep (Algorithm 1) on a block: (3, Mb) float64 device tensor of
    diagonals kstop-2..kstop by local row, NaN outside the block."""
    d = X.shape[1]
    o = make_opts(precision)
    n = ctypes.c_size_t()
    _check(lib().dtw_workspace_size(i1 + 1, j1 + 1, d, _dtype_code(X), ctypes.byref(o), ctypes.byref(n)),
           "dtw_workspace_size")
    ws = torch.empty(n.value, dtype=torch.uint8, device=X.device)
    Mb = i1 - i0 + 1
    out = torch.empty((3, Mb), dtype=torch.float64, device=X.device)
    rc = lib().dtw_diag(_dev(X), _dev(Y), d, _dtype_code(X), i0, j0, i1, j1, int(bool(reverse)), kstop,
                        o.precision, ctypes.c_void_p(ws.data_ptr()), n.value, ctypes.c_void_p(out.data_ptr()),
                        _stream_ptr(stream))
    _check(rc, "dtw_diag")
    code = device_error(ws, stream)
    if code:
        raise DeviceError(code, "dtw_diag")
    return out


# ------------------------------------------------------------------ serving form

class ServerOpts(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("device", ctypes.c_int32), ("reserved", ctypes.c_int32 * 5)]


class Request(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("M", ctypes.c_int64), ("Y", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("d", ctypes.c_int32), ("in_dtype", ctypes.c_int32), ("opts", Opts),
                ("cost_out", ctypes.c_void_p), ("path_out", ctypes.c_void_p), ("path_cap", ctypes.c_int64),
                ("path_len_out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("device_error", ctypes.c_int32), ("batch_size", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


def _server_lib():
    L = lib()
    if not getattr(L, "_server_bound", False):
        vp = ctypes.c_void_p
        L.dtw_server_default_opts.argtypes = [ctypes.POINTER(ServerOpts)]
        L.dtw_server_default_opts.restype = None
        L.dtw_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
        L.dtw_server_create.restype = ctypes.c_int32
        L.dtw_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
        L.dtw_server_submit.restype = ctypes.c_int32
        for name in ("dtw_server_poll", "dtw_server_wait"):
            f = getattr(L, name)
            f.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Result)]
            f.restype = ctypes.c_int32
        L.dtw_server_destroy.argtypes = [vp]
        L.dtw_server_destroy.restype = ctypes.c_int32
        L._server_bound = True
    return L


class Server:
    """Continuous-batching request loop of the library (dtw_server_* in
    include/dtw.h).  Inputs must be fully written before submit; outputs are
    device tensors owned here until the result is collected."""

    BUSY = -6

    def __init__(self, pool_bytes=8 << 30, max_slots=4, max_batch=64, device=0):
        L = _server_lib()
        o = ServerOpts()
        L.dtw_server_default_opts(ctypes.byref(o))
        o.pool_bytes, o.max_slots, o.max_batch, o.device = int(pool_bytes), int(max_slots), int(max_batch), int(device)
        h = ctypes.c_void_p()
        _check(L.dtw_server_create(ctypes.byref(o), ctypes.byref(h)), "dtw_server_create")
        self._h = h
        self._live = {}

    def submit(self, X, Y, precision="fp64", min_block=500, cost="euclidean", tie_exact=False):
        if X.dtype != Y.dtype or X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
            raise ValueError("X and Y must be 2-D with equal dtype and feature dimension")
        torch.cuda.current_stream(X.device).synchronize()  # inputs written before the server's stream reads them
        M, d = X.shape
        N = Y.shape[0]
        out_cost = torch.empty(1, dtype=torch.float64, device=X.device)
        path = torch.empty((M + N - 1, 2), dtype=torch.int32, device=X.device)
        plen = torch.empty(1, dtype=torch.int64, device=X.device)
        r = Request(_dev(X).value, M, _dev(Y).value, N, d, _dtype_code(X), make_opts(precision, min_block, cost=cost,
                                                                                 tie_exact=tie_exact),
                    out_cost.data_ptr(), path.data_ptr(), M + N - 1, plen.data_ptr())
        tk = ctypes.c_uint64()
        _check(_server_lib().dtw_server_submit(self._h, ctypes.byref(r), ctypes.byref(tk)), "dtw_server_submit")
        self._live[tk.value] = (X, Y, out_cost, path, plen)
        return tk.value

    def _collect(self, ticket, block):
        res = Result()
        f = _server_lib().dtw_server_wait if block else _server_lib().dtw_server_poll
        rc = f(self._h, ticket, ctypes.byref(res))
        if rc == self.BUSY:
            return None
        _check(rc, "dtw_server_poll")
        X, Y, cost, path, plen = self._live.pop(ticket)
        out = res.to_dict()
        if res.status == 0:
            n = int(plen.item())
            out.update(cost=float(cost.item()), path=path[:n])
        return out

    def poll(self, ticket):
        """None while the request is queued or running, else its result dict."""
        return self._collect(ticket, False)

    def wait(self, ticket):
        return self._collect(ticket, True)

    def close(self):
        if self._h:
            _check(_server_lib().dtw_server_destroy(self._h), "dtw_server_destroy")
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- edit distance

def edit_workspace_size(M, N, leaf_rows=64):
    n = ctypes.c_size_t()
    _check(lib().dtw_edit_workspace_size(int(M), int(N), int(leaf_rows), ctypes.byref(n)), "dtw_edit_workspace_size")
    return n.value


class EditStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("device_error", ctypes.c_int32), ("sweep_cells", ctypes.c_int64),
                ("leaf_cells", ctypes.c_int64), ("sweep_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EditAligner:
    """Reusable workspace and outputs for edit-distance alignments of strings
    of at most M and N bytes (dtw_edit_align)."""

    def __init__(self, M, N, leaf_rows=64, device="cuda"):
        self.M, self.N, self.leaf_rows = int(M), int(N), int(leaf_rows)
        self.ws_bytes = edit_workspace_size(M, N, leaf_rows)
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        self.dist = torch.empty(1, dtype=torch.int64, device=device)
        self.path = torch.empty((self.M + self.N + 1, 2), dtype=torch.int32, device=device)
        self.plen = torch.empty(1, dtype=torch.int64, device=device)

    def run(self, a, b, sub=1, gap=1, stream=None, stats=False):
        """Enqueue one alignment of device uint8 tensors a (M) and b (N).  With
        stats=True the call synchronises and returns the stats dict."""
        for t in (a, b):
            if t.dtype != torch.uint8 or t.dim() != 1 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("a and b must be contiguous 1-D uint8 device tensors")
        M, N = a.shape[0], b.shape[0]
        st = EditStats()
        if (M, N) != (self.M, self.N):
            raise ValueError(f"sized for {self.M} x {self.N}, got {M} x {N}")
        _check(lib().dtw_edit_align(ctypes.c_void_p(a.data_ptr() if M else 0), M,
                                    ctypes.c_void_p(b.data_ptr() if N else 0), N, int(sub), int(gap),
                                    self.leaf_rows, ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                    ctypes.c_void_p(self.dist.data_ptr()), ctypes.c_void_p(self.path.data_ptr()),
                                    self.path.shape[0], ctypes.c_void_p(self.plen.data_ptr()),
                                    ctypes.byref(st) if stats else None, _stream_ptr(stream)),
               "dtw_edit_align")
        return st.to_dict() if stats else None


def edit_align(a, b, sub=1, gap=1, leaf_rows=64, stream=None):
    """Edit distance and an optimal alignment of device uint8 tensors a and b.

    Returns (distance: int, path: int32 tensor [n, 2] of nodes (i, j) on the
    device).  Synchronises the stream.  Raises DeviceError when the call's
    kernels recorded a device-side error."""
    al = EditAligner(a.shape[0], b.shape[0], leaf_rows, device=a.device)
    al.run(a, b, sub, gap, stream)
    d = int(al.dist.item())
    n = int(al.plen.item())
    if d < 0:
        raise DeviceError(-d, "dtw_edit_align")
    return d, al.path[:n]


# ----------------------------------------------------------------- local alignment score

class LocalScorer:
    """Reusable workspace and output for Smith-Waterman scores of strings of M
    and N bytes (dtw_local_score)."""

    def __init__(self, M, N, device="cuda"):
        self.M, self.N = int(M), int(N)
        n = ctypes.c_size_t()
        _check(lib().dtw_local_workspace_size(self.M, self.N, ctypes.byref(n)), "dtw_local_workspace_size")
        self.ws_bytes = n.value
        self.ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=device)
        self.out = torch.empty(3, dtype=torch.int64, device=device)

    def run(self, a, b, match=2, mismatch=1, gap=1, stream=None):
        for t in (a, b):
            if t.dtype != torch.uint8 or t.dim() != 1 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("a and b must be contiguous 1-D uint8 device tensors")
        if (a.shape[0], b.shape[0]) != (self.M, self.N):
            raise ValueError(f"sized for {self.M} x {self.N}, got {a.shape[0]} x {b.shape[0]}")
        _check(lib().dtw_local_score(ctypes.c_void_p(a.data_ptr() if self.M else 0), self.M,
                                     ctypes.c_void_p(b.data_ptr() if self.N else 0), self.N, int(match),
                                     int(mismatch), int(gap), ctypes.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                     ctypes.c_void_p(self.out.data_ptr()), _stream_ptr(stream)), "dtw_local_score")


def local_score(a, b, match=2, mismatch=1, gap=1, stream=None):
    """Smith-Waterman score of device uint8 tensors a and b and the end cell of
    a best local alignment: (score, i_end, j_end).  Synchronises the stream."""
    sc = LocalScorer(a.shape[0], b.shape[0], device=a.device)
    sc.run(a, b, match, mismatch, gap, stream)
    s, i, j = (int(v) for v in sc.out.cpu().tolist())
    if s < 0:
        raise DeviceError(-s, "dtw_local_score")
    return s, i, j
