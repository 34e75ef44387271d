"""CPU model of the edit-distance kernels: the real dtw_edit.hip source (its
kernels and host entry points) compiled for the host with AddressSanitizer
and UndefinedBehaviorSanitizer against the thread-based HIP stand-in of
tests/cpu_model, one OS thread per lane.  Blocks of a launch run one after
another, so the persistent sweep's first workgroup takes every stripe in
ticket order.  Results are compared with the oracle (edit distance of the
textbook table, path of the linear-memory recursion), bit for bit."""
import os
import struct
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import edit
from paper_2008_02734_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL = os.path.join(ROOT, "tests", "cpu_model")
CSRC = os.path.join(ROOT, "paper_2008_02734_amd", "csrc")


def _build(d, extra=()):
    exe = str(d / "edit_model")
    subprocess.run(["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-Wno-unknown-pragmas", "-pthread", *extra, "-I", MODEL,
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "c++",
                    os.path.join(MODEL, "edit_driver.cpp"), "-o", exe], check=True)
    return exe


@pytest.fixture(scope="module")
def edit_model(tmp_path_factory):
    # problems up to 65536 rows take 128-row stripes (two rows per lane); the
    # local score's launch, switched off in the library, is switched on here
    return _build(tmp_path_factory.mktemp("edit_model"), ["-DDTW_LOCAL_SCORE_ENABLED=1"])


@pytest.fixture(scope="module")
def edit_model_r4(tmp_path_factory):
    # the 256-row stripes (four rows per lane) of taller problems, forced here
    # for small ones by lowering the threshold
    return _build(tmp_path_factory.mktemp("edit_model_r4"), ["-DED_SMALL_M=0"])


def run_edit_model(exe, a, b, sub, gap, leaf_rows):
    with tempfile.TemporaryDirectory() as td:
        fi, fo = os.path.join(td, "in"), os.path.join(td, "out")
        with open(fi, "wb") as f:
            f.write(struct.pack("2q4i", a.size, b.size, sub, gap, leaf_rows, 0))
            f.write(a.tobytes())
            f.write(b.tobytes())
        r = subprocess.run([exe, fi, fo], capture_output=True, timeout=600,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
        assert r.returncode == 0, r.stderr.decode()[-3000:]
        buf = open(fo, "rb").read()
    rc, levels = struct.unpack_from("2i", buf, 0)
    dist, n, sweep_cells, leaf_cells = struct.unpack_from("4q", buf, 8)
    path = np.frombuffer(buf[40:40 + 8 * n], dtype=np.int32).reshape(-1, 2) if rc == 0 else None
    run_edit_model.cells = (sweep_cells, leaf_cells)
    return rc, levels, dist, path


def oracle_cells(M, N, h, pivots):
    """Sweep and leaf cells implied by the oracle's splits: block k of level L
    spans rows floor(k M / 2^L) .. floor((k+1) M / 2^L); its half sweeps cover
    all its rows times its columns, and the blocks of the last level are leaves."""
    levels = edit.levels(M, h)
    cols = {(0, 0): (0, N)}
    sweep = 0
    for L, k, mid, j in pivots.tolist():
        j0, j1 = cols[(L, k)]
        sweep += (((k + 1) * M >> L) - (k * M >> L)) * (j1 - j0)
        cols[(L + 1, 2 * k)] = (j0, j)
        cols[(L + 1, 2 * k + 1)] = (j, j1)
    leaf = sum((((k + 1) * M >> levels) - (k * M >> levels)) * (cols[(levels, k)][1] - cols[(levels, k)][0])
               for k in range(1 << levels))
    return sweep, leaf


# (M, N, sub, gap, leaf_rows): empty strings, one leaf, leaves of two rows,
# several levels, and half sweeps of three 128-row stripes whose later stripes
# read the previous one's last row through the ring
CASES = [(0, 5, 1, 1, 2), (5, 0, 1, 1, 2), (1, 1, 1, 1, 2), (7, 9, 1, 1, 2), (40, 33, 1, 1, 3),
         (600, 90, 3, 2, 64)]


@pytest.mark.parametrize("M,N,sub,gap,h", CASES)
def test_edit_model_equals_oracle(edit_model, M, N, sub, gap, h):
    a, b = synth.string_pair(8000 + M + N, M, N, k=4, p=0.2)
    rc, levels, dist, path = run_edit_model(edit_model, a, b, sub, gap, h)
    assert rc == 0
    assert levels == edit.levels(M, h)
    assert dist == edit.full(a, b, sub, gap)[0]
    r = edit.linear(a, b, sub, gap, leaf_rows=h, pivots=True)
    assert path.tolist() == r["path"].tolist()
    assert run_edit_model.cells == oracle_cells(M, N, h, r["pivots"])


@pytest.mark.parametrize("M,N,sub,gap,h", [(7, 9, 1, 1, 2), (600, 90, 3, 2, 64)])
def test_edit_model_four_rows_per_lane(edit_model_r4, M, N, sub, gap, h):
    a, b = synth.string_pair(8100 + M + N, M, N, k=4, p=0.2)
    rc, levels, dist, path = run_edit_model(edit_model_r4, a, b, sub, gap, h)
    assert rc == 0
    assert dist == edit.full(a, b, sub, gap)[0]
    assert path.tolist() == edit.linear(a, b, sub, gap, leaf_rows=h)["path"].tolist()


def test_edit_model_rejects_bad_arguments(edit_model):
    a, b = synth.string_pair(1, 10, 10)
    assert run_edit_model(edit_model, a, b, 1, 1, 1)[0] == -1    # leaf_rows below 2
    assert run_edit_model(edit_model, a, b, 1, 1, 65)[0] == -1   # above one wave
    assert run_edit_model(edit_model, a, b, -1, 1, 8)[0] == -1   # negative cost
    assert run_edit_model(edit_model, a, b, 1 << 21, 1, 8)[0] == -1


def run_local_model(exe, a, b, match, mismatch, gap):
    with tempfile.TemporaryDirectory() as td:
        fi, fo = os.path.join(td, "in"), os.path.join(td, "out")
        with open(fi, "wb") as f:
            f.write(struct.pack("2q4i", a.size, b.size, match, mismatch, gap, 1))
            f.write(a.tobytes())
            f.write(b.tobytes())
        r = subprocess.run([exe, fi, fo], capture_output=True, timeout=600,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
        assert r.returncode == 0, r.stderr.decode()[-3000:]
        buf = open(fo, "rb").read()
    (rc,) = struct.unpack_from("i", buf, 0)
    return rc, struct.unpack_from("3q", buf, 4)


# the local alignment score kernels (dtw_local.hip): empty strings, one
# stripe, and two stripes with the maximum in the second
@pytest.mark.parametrize("M,N,p", [(0, 5, 0.3), (5, 0, 0.3), (7, 9, 0.3), (300, 280, 0.3)])
def test_local_model_equals_oracle(edit_model, M, N, p):
    a, b = synth.string_pair(8300 + M + N, M, N, k=4, p=p)
    for match, mismatch, gap in ((2, 1, 1), (3, 2, 2)):
        rc, out = run_local_model(edit_model, a, b, match, mismatch, gap)
        assert rc == 0
        assert tuple(out) == edit.local_score(a, b, match, mismatch, gap)
