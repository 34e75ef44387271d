"""The no-allocation entry point (dtw_align_noalloc) against dtw_align.

dtw_align_noalloc runs the same kernels as dtw_align with the library's own
fixed device array as the workspace, so its results must equal dtw_align's
bit for bit: the same path and the same FP64 cost.  Two calls in a row, the
second on a smaller problem, check that nothing the first call left in the
shared array leaks into the second.  The textbook oracle pins the FP64 paths.
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


def _outputs(M, N, dev="cuda"):
    cost = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    path = torch.full((M + N - 1, 2), -1, dtype=torch.int32, device=dev)
    plen = torch.zeros(1, dtype=torch.int64, device=dev)
    return cost, path, plen


def _case(dtw, M, N, d, seed, precision, min_block, dtype=torch.float64):
    X, Y = synth.make_pair(9, seed, M, N, d, "chroma")
    Xd = torch.from_numpy(X).to("cuda", dtype)
    Yd = torch.from_numpy(Y).to("cuda", dtype)
    al = dtw.Aligner(M, N, d, dtype, precision, min_block)
    st_ref = al.run(Xd, Yd, stats=True)
    n_ref = int(st_ref["path_len"])
    cost, path, plen = _outputs(M, N)
    st = dtw.align_noalloc(Xd, Yd, cost, path, plen, precision, min_block, stats=True)
    n = int(plen.item())
    assert st["device_error"] == 0 and n == n_ref == int(st["path_len"])
    assert torch.equal(path[:n].cpu(), al.path[:n_ref].cpu())
    c, c_ref = float(cost.item()), float(al.cost.item())
    assert np.float64(c).view(np.int64) == np.float64(c_ref).view(np.int64), (c, c_ref)
    assert st["cells_processed"] == st_ref["cells_processed"]
    if precision == "fp64":
        c_o, p_o = oracle.full(X, Y)
        assert path[:n].cpu().numpy().tolist() == p_o.tolist()
        assert abs(c - c_o) <= 1e-12 * c_o
    # the asynchronous form (no stats) gives the same result
    cost2, path2, plen2 = _outputs(M, N)
    dtw.align_noalloc(Xd, Yd, cost2, path2, plen2, precision, min_block)
    torch.cuda.synchronize()
    assert int(plen2.item()) == n and torch.equal(path2[:n], path[:n]) and torch.equal(cost2, cost)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_equals_align_twice_second_smaller(dtw, precision):
    _case(dtw, 1500, 1300, 12, 0, precision, 64)   # several levels, stripes and leaves
    _case(dtw, 333, 210, 12, 1, precision, 32)     # smaller, right after, same array


def test_noalloc_large_then_small(dtw):
    # the 20000 x 16000 FP64 workload (about 10 MiB of the 64 MiB array), then a tiny one
    X, Y = synth.make_pair(2, 0, 20000, 16000, 12, "chroma")
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    al = dtw.Aligner(20000, 16000, 12)
    al.run(Xd, Yd, stats=True)
    cost, path, plen = _outputs(20000, 16000)
    st = dtw.align_noalloc(Xd, Yd, cost, path, plen, stats=True)
    n = int(plen.item())
    assert st["device_error"] == 0
    assert torch.equal(path[:n], al.path[:n]) and torch.equal(cost, al.cost)
    _case(dtw, 70, 50, 3, 2, "fp64", 3)


def test_noalloc_rejects_oversize(dtw):
    cost, path, plen = _outputs(200000, 160000)
    X = torch.zeros((200000, 12), dtype=torch.float64, device="cuda")
    Y = torch.zeros((160000, 12), dtype=torch.float64, device="cuda")
    with pytest.raises(dtw.DtwError) as e:
        dtw.align_noalloc(X, Y, cost, path, plen)
    assert e.value.status == -3
