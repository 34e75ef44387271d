"""Serving form: continuous batching over one device pool (dtw_server_*).

Each request's result must be the same alone (dtw_align) and in the mix, and
requests submitted while others run must be admitted and run concurrently.
"""
import time

import numpy as np
import pytest
import torch

from paper_2008_02734_amd import synth

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


def mixed_requests(n, seed=5):
    """Uneven lengths and the four precision forms, from the generators."""
    rng = np.random.default_rng([5, 999, seed])
    reqs = []
    for r in range(n):
        M = int(np.exp(rng.uniform(np.log(200), np.log(4000))))
        N = int(M * rng.uniform(0.75, 1.3))
        kind = r % 4
        if kind == 0:
            X, Y = synth.make_pair(5, r, M, N, 12, "chroma")
            reqs.append((dev(X, torch.float64), dev(Y, torch.float64), "fp64"))
        elif kind == 1:
            X, Y = synth.make_pair(5, r, M, N, 12, "chroma")
            reqs.append((dev(X, torch.float32), dev(Y, torch.float32), "fp32"))
        else:
            X, Y = synth.make_pair(5, r, M, N, 128, "embedding")
            reqs.append((dev(X, torch.float32), dev(Y, torch.float32), "bf16" if kind == 2 else "fp16"))
    return reqs


def test_results_same_alone_and_in_the_mix(dtw):
    reqs = mixed_requests(20)
    srv = dtw.Server(pool_bytes=256 << 20, max_slots=3, max_batch=4)
    try:
        tickets = [srv.submit(X, Y, precision=p, min_block=128) for X, Y, p in reqs]
        results = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for (X, Y, p), res in zip(reqs, results):
        assert res["status"] == 0 and res["device_error"] == 0, res
        cost, path, _ = dtw.align(X, Y, precision=p, min_block=128)
        assert res["cost"] == cost
        assert torch.equal(res["path"], path)
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
