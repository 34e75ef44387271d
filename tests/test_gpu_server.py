"""Serving form: continuous batching over one device pool (dtw_server_*).

Each request's result must be the same alone (dtw_align) and in the mix, and
requests submitted while others run must be admitted and run concurrently.
Every served result is also checked against the CPU oracle: FP64 requests
return the textbook path, reduced-precision requests a valid path within
their tolerance of the exact optimum, and every reported cost is the FP64
cost of the returned path.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2008_02734_amd import synth

# relative cost error against the exact optimum, per form
TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp16": 1e-5, "bf16": 1e-2}

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dtw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_02734_amd import dtw as mod
    mod.lib()
    return mod


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def mixed_requests(n, seed=5, host=False):
    """Uneven lengths and the four precision forms, from the generators.  With
    `host`, each entry also carries the FP64 host frames the device frames were
    made from (as the device sees them: rounded to FP32 for the FP32 inputs)."""
    rng = np.random.default_rng([5, 999, seed])
    reqs = []
    for r in range(n):
        M = int(np.exp(rng.uniform(np.log(200), np.log(4000))))
        N = int(M * rng.uniform(0.75, 1.3))
        kind = r % 4
        if kind == 0:
            X, Y = synth.make_pair(5, r, M, N, 12, "chroma")
            item = (dev(X, torch.float64), dev(Y, torch.float64), "fp64")
        elif kind == 1:
            X, Y = synth.make_pair(5, r, M, N, 12, "chroma")
            item = (dev(X, torch.float32), dev(Y, torch.float32), "fp32")
        else:
            X, Y = synth.make_pair(5, r, M, N, 128, "embedding")
            item = (dev(X, torch.float32), dev(Y, torch.float32), "bf16" if kind == 2 else "fp16")
        if host:
            item = item + (item[0].double().cpu().numpy(), item[1].double().cpu().numpy())
        reqs.append(item)
    return reqs


def check_against_oracle(Xh, Yh, prec, cost, path):
    """A served result against the oracle: textbook path and cost for FP64, a
    valid path within the form's tolerance of the exact optimum otherwise, and
    the reported cost equal to the FP64 cost of the returned path."""
    p = path.cpu().numpy()
    M, N = Xh.shape[0], Yh.shape[0]
    assert tuple(p[0]) == (0, 0) and tuple(p[-1]) == (M - 1, N - 1)
    assert {tuple(v) for v in np.diff(p, axis=0).tolist()} <= {(0, 1), (1, 0), (1, 1)}
    c_ref, p_ref = oracle.full(Xh, Yh)
    if prec == "fp64":
        assert p.tolist() == p_ref.tolist()
    assert -1e-12 <= (cost - c_ref) / c_ref <= TOL[prec], (prec, cost, c_ref)
    assert abs(cost - oracle.path_cost(Xh, Yh, p)) <= 1e-12 * c_ref


def test_results_same_alone_and_in_the_mix(dtw):
    reqs = mixed_requests(20, host=True)
    srv = dtw.Server(pool_bytes=256 << 20, max_slots=3, max_batch=4)
    try:
        tickets = [srv.submit(X, Y, precision=p, min_block=128) for X, Y, p, _, _ in reqs]
        results = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for (X, Y, p, Xh, Yh), res in zip(reqs, results):
        assert res["status"] == 0 and res["device_error"] == 0, res
        cost, path, _ = dtw.align(X, Y, precision=p, min_block=128)
        assert res["cost"] == cost
        assert torch.equal(res["path"], path)
        check_against_oracle(Xh, Yh, p, res["cost"], res["path"])
    # several requests per batch, and batches of different requests overlapped in time
    assert max(r["batch_size"] for r in results) > 1
    spans = sorted((r["t_admit_ns"], r["t_done_ns"]) for r in results)
    overlap = any(spans[i + 1][0] < spans[i][1] and (spans[i + 1][0], spans[i + 1][1]) != spans[i]
                  for i in range(len(spans) - 1))
    assert overlap


def test_requests_arriving_while_others_run(dtw):
    # a long request first, then short ones: the short ones are admitted into
    # other slots and finish before the long one
    X, Y = synth.make_pair(5, 100, 16000, 14000, 12, "chroma")
    long_req = (dev(X, torch.float64), dev(Y, torch.float64))
    shorts = mixed_requests(6, seed=9)
    srv = dtw.Server(pool_bytes=2 << 30, max_slots=4, max_batch=2)
    try:
        t_long = srv.submit(*long_req, precision="fp64")
        time.sleep(0.001)
        t_short = [srv.submit(X, Y, precision=p) for X, Y, p in shorts]
        res_short = [srv.wait(t) for t in t_short]
        res_long = srv.wait(t_long)
    finally:
        srv.close()
    assert res_long["status"] == 0
    assert all(r["status"] == 0 for r in res_short)
    assert min(r["t_admit_ns"] for r in res_short) < res_long["t_done_ns"]
    assert sum(r["t_done_ns"] < res_long["t_done_ns"] for r in res_short) >= 3
    cost, path, _ = dtw.align(*long_req)
    assert res_long["cost"] == cost and torch.equal(res_long["path"], path)
    check_against_oracle(X, Y, "fp64", res_long["cost"], res_long["path"])


def test_long_request_in_the_mix(dtw):
    # one request of 120000 x 100000 frames (FP32, d = 12) served beside
    # shorter ones: its cost is within 1e-5 of the GPU's exact FP64 path on the
    # same frames (whose path equals the oracle's by the parity tests), and the
    # reported cost is the FP64 cost of the returned path
    X, Y = synth.make_pair(5, 300, 120000, 100000, 12, "chroma")
    X32, Y32 = dev(X, torch.float32), dev(Y, torch.float32)
    Xh, Yh = X32.double().cpu().numpy(), Y32.double().cpu().numpy()
    shorts = mixed_requests(4, seed=11)
    srv = dtw.Server(pool_bytes=2 << 30, max_slots=4, max_batch=4)
    try:
        t_long = srv.submit(X32, Y32, precision="fp32")
        t_short = [srv.submit(Xs, Ys, precision=p) for Xs, Ys, p in shorts]
        res = srv.wait(t_long)
        res_short = [srv.wait(t) for t in t_short]
    finally:
        srv.close()
    assert res["status"] == 0 and res["device_error"] == 0, res
    assert all(r["status"] == 0 for r in res_short)
    c64, p64, st = dtw.align(X32.double(), Y32.double())
    assert st["device_error"] == 0
    assert -1e-12 <= (res["cost"] - c64) / c64 <= 1e-5
    p = res["path"].cpu().numpy()
    assert tuple(p[0]) == (0, 0) and tuple(p[-1]) == (X.shape[0] - 1, Y.shape[0] - 1)
    assert {tuple(v) for v in np.diff(p, axis=0).tolist()} <= {(0, 1), (1, 0), (1, 1)}
    assert abs(res["cost"] - oracle.path_cost(Xh, Yh, p)) <= 1e-12 * c64


def test_poll_busy_then_done_and_errors(dtw):
    X, Y = synth.make_pair(5, 200, 3000, 2800, 12, "chroma")
    Xd, Yd = dev(X, torch.float64), dev(Y, torch.float64)
    srv = dtw.Server(pool_bytes=16 << 20, max_slots=1, max_batch=1)
    try:
        tk = srv.submit(Xd, Yd)
        first = srv.poll(tk)  # None while queued or running (the request may also be done already)
        res = first if first is not None else srv.wait(tk)
        assert res["status"] == 0
        with pytest.raises(dtw.DtwError) as e:  # collected tickets are released
            srv.poll(tk)
        assert e.value.status == -7
        # a request that cannot fit in the pool even alone
        big = synth.make_pair(5, 201, 60000, 50000, 12, "chroma")
        with pytest.raises(dtw.DtwError) as e:
            srv.submit(dev(big[0], torch.float64), dev(big[1], torch.float64))
        assert e.value.status == -3
        # d beyond the widest frame form
        Z = torch.zeros((10, 129), dtype=torch.float64, device="cuda")
        with pytest.raises(dtw.DtwError) as e:
            srv.submit(Z, Z)
        assert e.value.status == -8
    finally:
        srv.close()
