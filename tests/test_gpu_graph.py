"""Replay of repeated dtw_align calls from a recorded HIP graph: every replay
gives the launch-by-launch result bit for bit, reads the inputs as they are
when it runs, and survives eager work between replays."""
import os

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


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def result(al):
    n = int(al.plen.item())
    return float(al.cost.item()), al.path[:n].cpu().numpy().copy()


def eager(dtw, X, Y, dtype=torch.float64, **kw):
    os.environ["DTW_GRAPHS"] = "0"
    try:
        al = dtw.Aligner(X.shape[0], Y.shape[0], X.shape[1], dtype, device="cuda", **kw)
        al.run(dev(X, dtype), dev(Y, dtype))
        return result(al)
    finally:
        del os.environ["DTW_GRAPHS"]


@pytest.mark.parametrize("kw", [dict(), dict(tie_exact=True), dict(precision="fp32"), dict(precision="bf16")])
def test_replays_equal_the_eager_sequence(dtw, kw):
    M, N, d = (3000, 2400, 12) if kw.get("precision") != "bf16" else (3000, 2400, 64)
    dtype = torch.float32 if kw.get("precision") in ("fp32", "bf16") else torch.float64
    X, Y = synth.make_pair(2, 7, M, N, d, "chroma" if d == 12 else "embedding")
    ref_c, ref_p = eager(dtw, X, Y, dtype, **kw)
    al = dtw.Aligner(M, N, d, dtype, device="cuda", **kw)
    Xd, Yd = dev(X, dtype), dev(Y, dtype)
    before = dtw.graph_count()
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(6):
        st = al.run(Xd, Yd, stats=True)
        assert st["device_error"] == 0
        c, p = result(al)
        assert c == ref_c and p.tolist() == ref_p.tolist(), rep
        junk.mul_(1.0001).add_(0.5)  # the program's own eager work between replays
        torch.cuda.synchronize()
    assert dtw.graph_count() > before or dtw.graph_count() == 16  # recorded on the second call


def test_replay_reads_the_inputs_when_it_runs(dtw):
    # the same buffers refilled between calls: each replay aligns what they
    # hold then (graph recorded on the second call, replayed after)
    pairs = [synth.make_pair(2, 20 + k, 1500, 1300, 12, "chroma") for k in range(3)]
    al = dtw.Aligner(1500, 1300, 12, device="cuda")
    Xd, Yd = dev(pairs[0][0]), dev(pairs[0][1])
    for rep in range(7):
        X, Y = pairs[rep % 3]
        Xd.copy_(dev(X))
        Yd.copy_(dev(Y))
        al.run(Xd, Yd)
        c, p = result(al)
        c_ref, p_ref = oracle.full(X, Y)
        assert p.tolist() == p_ref.tolist(), rep
        assert abs(c - c_ref) <= 1e-12 * c_ref


def test_alternating_calls_each_replay_their_own_graph(dtw):
    shapes = [(900, 700), (1200, 1500)]
    cases = []
    for k, (M, N) in enumerate(shapes):
        X, Y = synth.make_pair(2, 40 + k, M, N, 12, "chroma")
        cases.append((dtw.Aligner(M, N, 12, device="cuda"), dev(X), dev(Y), eager(dtw, X, Y)))
    for rep in range(4):
        for al, Xd, Yd, (rc, rp) in cases:
            al.run(Xd, Yd)
            c, p = result(al)
            assert c == rc and p.tolist() == rp.tolist()
