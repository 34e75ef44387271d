"""The numerical precision / tie-breaking experiment of Sec. 4.2, with the
discrepancy distributions of Sec. 4.4, on synthetic stand-ins for the paper's
audio features.

The paper checks (i) its 32-bit GPU alignment against a brute-force 32-bit CPU
textbook solve and (ii) two 64-bit CPU textbook solves that differ only in
whether DIAG or LEFT wins a tie, and reports, for each comparison, the
fraction of path correspondences whose discrepancy is within 23 ms, 47 ms,
510 ms and 1 s (1, 2, 22 and 43 frames at 43 frames per second).  Here:

  GPU FP32 form      vs  CPU binary32 textbook (oracle.full_f32)
  GPU exact FP64     vs  CPU FP64 textbook (oracle.full, DIAG first)
  CPU FP64, DIAG first  vs  CPU FP64, LEFT first (oracle.full_left_first)

on a tie-free Gaussian walk, a chroma-like pair, and a chroma-like pair
quantised to steps of 1/8, whose frame costs repeat and tie often.  The
distributions are printed; the assertions are the parts that are fixed: both
tie rules reach the same optimum, the exact GPU path is the CPU FP64 path on
tie-free inputs and has the optimal cost on every input, and the 32-bit
answers differ from the 64-bit ones by a rounding-size amount.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2008_02734_amd import metrics, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dtw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_02734_amd import dtw as mod
    mod.lib()
    return mod


def quantised_chroma(item, M, N, step=0.125):
    X, Y = synth.make_pair(6, item, M, N, 12, "chroma")
    return np.round(X / step) * step, np.round(Y / step) * step


CASES = {
    "gaussian walk 500x400 d=12": lambda: synth.make_pair(1, 0, 500, 400, 12, "gaussian_walk"),
    "chroma 1500x1200 d=12": lambda: synth.make_pair(6, 1, 1500, 1200, 12, "chroma"),
    "quantised chroma 900x800 d=12": lambda: quantised_chroma(2, 900, 800),
}


def row(name, s):
    return (f"  {name:<34} " + " ".join(f"{s[f'frac_le_{t}']:.4f}" for t in metrics.THRESHOLDS_FRAMES)
            + f"   mean {s['mean_frames']:.3f}  max {s['max_frames']}")


@pytest.mark.parametrize("case", sorted(CASES))
def test_precision_and_tie_rule_discrepancies(dtw, case):
    X, Y = CASES[case]()
    M, N = X.shape[0], Y.shape[0]
    tie_free = not case.startswith("quantised")
    c64, p64 = oracle.full(X, Y)
    cL, pL = oracle.full_left_first(X, Y)
    c32, p32 = oracle.full_f32(X, Y)
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.from_numpy(Y).cuda()
    g64, gp64, st = dtw.align(Xd, Yd)
    g32, gp32, st32 = dtw.align(Xd, Yd, precision="fp32")
    gp64, gp32 = gp64.cpu().numpy(), gp32.cpu().numpy()
    rows = {
        "GPU FP32 vs CPU binary32": metrics.summary(gp32, p32),
        "GPU FP64 vs CPU FP64": metrics.summary(gp64, p64),
        "CPU FP64 DIAG vs LEFT first": metrics.summary(p64, pL),
        "CPU binary32 vs CPU FP64": metrics.summary(p32, p64),
    }
    print(f"\n{case}: fraction of correspondences within 1 / 2 / 22 / 43 frames")
    for k, v in rows.items():
        print(row(k, v))
    print(f"  costs: FP64 {c64:.12g}  LEFT-first {cL:.12g}  binary32 {c32:.9g}  GPU FP64 {g64:.12g}  "
          f"GPU FP32 form {g32:.12g}")
    # both tie rules are optimal: same cost, both valid paths
    assert cL == c64
    assert oracle.path_cost(X, Y, pL) == pytest.approx(c64, rel=1e-12)
    # the exact GPU path: the textbook path on tie-free inputs, optimal always
    assert abs(g64 - c64) <= 1e-12 * c64
    if tie_free:
        assert gp64.tolist() == p64.tolist()
        assert rows["CPU FP64 DIAG vs LEFT first"]["max_frames"] == 0
    # 32-bit answers: a rounding-size cost difference, and the GPU FP32 form's
    # path is within its 1e-5 bound of the optimum
    K = M + N - 1
    assert abs(c32 - c64) <= 2 * (K + 15) * 2.0 ** -24 * c64
    assert -1e-12 <= (g32 - c64) / c64 <= 1e-5
    # every comparison keeps all of its correspondences within one second
    for k, v in rows.items():
        assert v["frac_le_43"] == 1.0, (k, v)
