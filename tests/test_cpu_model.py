"""CPU model of the device orchestration, built from the real sources.

The orchestration kernels (paper_2008_02734_amd/csrc/dtw_plan.hip, without
its launcher section) and the real host runtime (dtw_api.hip) are compiled
for the host with g++ and AddressSanitizer against a thread-based stand-in
for the HIP runtime (tests/cpu_model/hip/hip_runtime.h).  The two wave
kernels are replaced by plain loops that write the same outputs and check
the stripe queue and every buffer index (tests/cpu_model/harness.cpp).
Every result is compared with the CPU oracle.
"""
import os
import struct
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_2008_02734_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2008_02734_amd", "csrc")
MODEL = os.path.join(ROOT, "tests", "cpu_model")
MARK = "// ----------------------------------------------------------------- launchers"


# The textual edits the wave kernels need to compile for the host: each
# inline-asm statement becomes its C++ meaning (minimum, register move,
# workgroup barrier, completion of outstanding memory operations), and the
# dynamic LDS array becomes a static buffer.
WAVE_EDITS = [
    # v_min in IEEE mode returns the other operand of a quiet NaN
    ('asm volatile("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));',
     "r = (a != a) ? b : ((b != b) ? a : ((b < a) ? b : a));"),
    ('asm volatile("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));',
     "r = (a != a) ? b : ((b != b) ? a : ((b < a) ? b : a));"),
    ('asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));', "r = x;"),
    ('asm volatile("v_min_f64 %0, %1, %2\\n\\tv_min_f64 %0, %0, %3\\n\\tv_add_f64 %0, %0, %4"\n'
     '               : "=&v"(r) : "v"(diag), "v"(left), "v"(up), "v"(c));',
     "{ const double m1 = (diag != diag) ? left : ((left != left) ? diag : ((left < diag) ? left : diag));"
     " const double m2 = (m1 != m1) ? up : ((up != up) ? m1 : ((up < m1) ? up : m1)); r = m2 + c; }"),
    ('asm volatile("v_min_f32 %0, %1, %2\\n\\tv_min_f32 %0, %0, %3\\n\\tv_add_f32 %0, %0, %4"\n'
     '               : "=&v"(r) : "v"(diag), "v"(left), "v"(up), "v"(c));',
     "{ const float m1 = (diag != diag) ? left : ((left != left) ? diag : ((left < diag) ? left : diag));"
     " const float m2 = (m1 != m1) ? up : ((up != up) ? m1 : ((up < m1) ? up : m1)); r = m2 + c; }"),
    ('asm volatile("s_waitcnt lgkmcnt(0)\\n\\ts_barrier" ::: "memory");', "__syncthreads();"),
    ('asm volatile("s_waitcnt vmcnt(0)" ::: "memory");', "std::atomic_thread_fence(std::memory_order_seq_cst);"),
    ("extern __shared__ __align__(16) unsigned char lds_raw[];", "unsigned char* lds_raw = cpu_dynamic_lds;"),
    # instrumentation: count every read of a boundary-ring cell, i.e. every
    # place where a stripe depends on another stripe's published values
    ("__device__ __forceinline__ uint64_t poll_word(const uint64_t* p, uint32_t tag, const Work& w) {\n",
     "__device__ __forceinline__ uint64_t poll_word(const uint64_t* p, uint32_t tag, const Work& w) {\n"
     "  cpu_poll_calls.fetch_add(1);\n"),
]


def _build_model(d, wave):
    src = open(os.path.join(CSRC, "dtw_plan.hip")).read()
    assert MARK in src
    with open(d / "dtw_plan_kernels.inc", "w") as f:
        f.write(src[: src.index(MARK)] + "}  // namespace dtw\n")
    wsrc = open(os.path.join(CSRC, "dtw_wave.hip")).read()
    body = wsrc[: wsrc.index(MARK)] + "}  // namespace dtw\n"
    for old, new in WAVE_EDITS:
        assert old in body, old
        body = body.replace(old, new)
    body = body.replace('#include "dtw_common.h"', "")
    with open(d / "dtw_wave_kernels.inc", "w") as f:
        f.write(body)
    exe = d / ("cpu_model_wave" if wave else "cpu_model")
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-Wno-unknown-pragmas", "-pthread",
           "-I", MODEL, "-I", str(d), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(MODEL, "harness.cpp"), os.path.join(MODEL, "driver.cpp"),
           "-x", "c++", os.path.join(CSRC, "dtw_api.hip"), "-o", str(exe)]
    if wave:
        cmd.insert(1, "-DMODEL_WAVE")
    subprocess.run(cmd, check=True)
    return str(exe)


@pytest.fixture(scope="module")
def model_exe(tmp_path_factory):
    return _build_model(tmp_path_factory.mktemp("cpu_model"), wave=False)


@pytest.fixture(scope="module")
def wave_exe(tmp_path_factory):
    return _build_model(tmp_path_factory.mktemp("cpu_model_wave"), wave=True)


def run_model(exe, pairs, m, precision=0, env=None, cost=0, tie=0):
    d = pairs[0][0].shape[1]
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        with open(fin, "wb") as f:
            f.write(struct.pack("4i", len(pairs), d, m, precision | (cost << 8) | (tie << 16)))
            for X, Y in pairs:
                f.write(struct.pack("2q", X.shape[0], Y.shape[0]))
            for X, _ in pairs:
                f.write(np.ascontiguousarray(X, dtype=np.float64).tobytes())
            for _, Y in pairs:
                f.write(np.ascontiguousarray(Y, dtype=np.float64).tobytes())
        r = subprocess.run([exe, fin, fout], capture_output=True, timeout=300,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0", **(env or {})))
        assert r.returncode == 0, r.stderr.decode()[-3000:]
        buf = open(fout, "rb").read()
        polls = int(r.stdout.decode().split("poll_calls=")[1].split()[0])
    rc, derr, levels, leaves = struct.unpack_from("4i", buf, 0)
    (cells,) = struct.unpack_from("q", buf, 16)
    off = 24
    out = []
    for _ in pairs:
        cost, n = struct.unpack_from("dq", buf, off)
        off += 16
        path = np.frombuffer(buf, dtype=np.int32, count=2 * n, offset=off).reshape(-1, 2) if rc == 0 else None
        off += 8 * n if rc == 0 else 0
        out.append((cost, path))
    return dict(rc=rc, device_error=derr, levels=levels, leaves=leaves, cells=cells, results=out, polls=polls)


def run_model_diag(exe, X, Y, i0, j0, i1, j1, reverse, kstop, precision=0):
    """DiagDTW (dtw_diag) in the model: (status, device error, (3, Mb) array)."""
    d = X.shape[1]
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        with open(fin, "wb") as f:
            f.write(struct.pack("4i", -1, d, 0, precision))
            f.write(struct.pack("8q", X.shape[0], Y.shape[0], i0, j0, i1, j1, reverse, kstop))
            f.write(np.ascontiguousarray(X, dtype=np.float64).tobytes())
            f.write(np.ascontiguousarray(Y, dtype=np.float64).tobytes())
        r = subprocess.run([exe, fin, fout], capture_output=True, timeout=300,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
        assert r.returncode == 0, r.stderr.decode()[-3000:]
        buf = open(fout, "rb").read()
    rc, derr = struct.unpack_from("2i", buf, 0)
    Mb = i1 - i0 + 1
    return rc, derr, np.frombuffer(buf, dtype=np.float64, count=3 * Mb, offset=8).reshape(3, Mb)


CASES = [(37, 29, 3, 3), (100, 80, 12, 3), (129, 257, 5, 16), (300, 240, 12, 16), (70, 70, 4, 64),
         (2, 300, 4, 3), (300, 1, 4, 3), (1, 1, 2, 3), (200, 130, 1, 5), (64, 65, 32, 3),
         (2200, 300, 2, 100),  # several scan chunks, > 16 stripes per top-level sweep
         (5000, 300, 2, 200)]  # few passes with many stripes: tickets spread over the threads


@pytest.mark.parametrize("M,N,d,m", CASES)
def test_model_matches_oracle(model_exe, M, N, d, m):
    X, Y = synth.random_pair(8000 + M + N, M, N, d, "normal")
    r = run_model(model_exe, [(X, Y)], m)
    assert r["rc"] == 0 and r["device_error"] == 0, r
    cost, path = r["results"][0]
    c_ref, p_ref = oracle.full(X, Y)
    assert path.tolist() == p_ref.tolist()
    assert abs(cost - c_ref) <= 1e-12 * c_ref
    assert r["cells"] == oracle.linmdtw(X, Y, min_block=m)["cells"]


@pytest.mark.parametrize("seed", range(6))
def test_model_ties_equal_linmdtw(model_exe, seed):
    rng = np.random.default_rng(seed)
    M, N = int(rng.integers(3, 90)), int(rng.integers(3, 90))
    X, Y = synth.random_pair(9000 + seed, M, N, 1, "int3")
    r = run_model(model_exe, [(X, Y)], 3)
    assert r["rc"] == 0 and r["device_error"] == 0
    assert r["results"][0][1].tolist() == oracle.linmdtw(X, Y, min_block=3)["path"].tolist()


def test_model_batched(model_exe):
    shapes = [(40, 33), (7, 90), (120, 100), (1, 1), (64, 64)]
    pairs = [synth.random_pair(500 + i, M, N, 6, "normal") for i, (M, N) in enumerate(shapes)]
    r = run_model(model_exe, pairs, 5)
    assert r["rc"] == 0 and r["device_error"] == 0
    for (X, Y), (cost, path) in zip(pairs, r["results"]):
        c_ref, p_ref = oracle.full(X, Y)
        assert path.tolist() == p_ref.tolist()
        assert abs(cost - c_ref) <= 1e-12 * c_ref


WAVE_CASES = [(37, 29, 3, 3), (70, 50, 12, 16), (130, 90, 5, 8), (20, 300, 4, 16), (9, 9, 2, 500),
              (90, 75, 64, 16), (70, 100, 100, 500), (80, 60, 128, 16)]


@pytest.mark.parametrize("M,N,d,m", WAVE_CASES)
def test_wave_model_matches_oracle(wave_exe, M, N, d, m):
    # the real sweep and leaf kernels, emulated lane by lane
    X, Y = synth.random_pair(8000 + M + N, M, N, d, "normal")
    r = run_model(wave_exe, [(X, Y)], m)
    assert r["rc"] == 0 and r["device_error"] == 0, r
    cost, path = r["results"][0]
    c_ref, p_ref = oracle.full(X, Y)
    assert path.tolist() == p_ref.tolist()
    assert abs(cost - c_ref) <= 1e-12 * c_ref


def test_wave_model_single_stripe_case_has_no_wait(wave_exe):
    # 37 x 29 at m = 3: every sweep has at most 34 rows (one stripe) and every
    # leaf at most 2 rows, so no kernel of this alignment ever reads a
    # boundary row from another stripe; a taller pair at the same cutoff does
    X, Y = synth.random_pair(8000, 37, 29, 3, "normal")
    r = run_model(wave_exe, [(X, Y)], 3)
    assert r["rc"] == 0 and r["device_error"] == 0, r
    assert r["polls"] == 0
    assert r["results"][0][1].tolist() == oracle.full(X, Y)[1].tolist()
    X2, Y2 = synth.random_pair(8001, 90, 60, 5, "normal")  # forward sweep to diagonal 75: two stripes
    r2 = run_model(wave_exe, [(X2, Y2)], 3)
    assert r2["rc"] == 0 and r2["polls"] > 0


def test_launch_check_refuses_launch_beyond_lds(model_exe):
    # the host-side launch check: with a per-workgroup LDS limit below the
    # sweep kernel's static LDS the call returns DTW_ERR_INTERNAL (-9) before
    # anything runs, instead of enqueueing a launch the device cannot place
    X, Y = synth.random_pair(8100, 100, 80, 12, "normal")
    r = run_model(model_exe, [(X, Y)], 16, env={"CPU_MODEL_LDS_MAX": "65536"})
    assert r["rc"] == -9
    # the same problem under the device's real limit runs
    r_ok = run_model(model_exe, [(X, Y)], 16)
    assert r_ok["rc"] == 0 and r_ok["device_error"] == 0


@pytest.mark.parametrize("M,N", [(130, 90), (90, 130)])
def test_wave_model_leaf_ties(wave_exe, M, N):
    # one leaf of two stripes (transposed or not) on integer frames with many
    # exact ties: the leaf's walk gives the textbook path and exact cost
    X, Y = synth.random_pair(9200 + M + N, M, N, 1, "int3")
    r = run_model(wave_exe, [(X, Y)], 500)
    assert r["rc"] == 0 and r["device_error"] == 0, r
    cost, path = r["results"][0]
    c_ref, p_ref = oracle.full(X, Y)
    assert path.tolist() == p_ref.tolist()
    assert cost == c_ref


@pytest.mark.parametrize("M,N,d,m", [(70, 50, 12, 16), (90, 75, 24, 500), (80, 60, 4, 8), (60, 70, 100, 16)])
def test_wave_model_fp32_form(model_exe, wave_exe, M, N, d, m):
    # the real kernels in FP32 (staged Y frames for d <= 32, wide frames
    # above): the same path as the plain model, which evaluates the same FP32
    # costs and recurrence cell by cell
    X, Y = synth.random_pair(8100 + M + N + d, M, N, d, "normal")
    r_wave = run_model(wave_exe, [(X, Y)], m, precision=1)
    r_plain = run_model(model_exe, [(X, Y)], m, precision=1)
    assert r_wave["rc"] == 0 and r_wave["device_error"] == 0, r_wave
    assert r_wave["results"][0][1].tolist() == r_plain["results"][0][1].tolist()
    assert abs(r_wave["results"][0][0] - r_plain["results"][0][0]) <= 1e-12 * r_plain["results"][0][0]


# ------------------------------------------------------------ BF16 Gram form

BF16_REL_TOL = 1e-2


def _gram_case(M, N, d, seed):
    X, Y = synth.make_pair(3, seed, M, N, d, "embedding")
    return X, Y


@pytest.mark.parametrize("M,N,d,m", [(150, 120, 64, 16), (90, 140, 128, 500), (70, 70, 20, 3)])
def test_model_gram_form(model_exe, M, N, d, m):
    # orchestration with the Gram-form costs: a valid path whose FP64 cost is
    # within the BF16 tolerance of the oracle's optimum
    X, Y = _gram_case(M, N, d, M + N)
    r = run_model(model_exe, [(X, Y)], m, precision=2)
    assert r["rc"] == 0 and r["device_error"] == 0, r
    cost, path = r["results"][0]
    c_ref, _ = oracle.full(X, Y)
    assert abs(cost - oracle.path_cost(X, Y, path)) <= 1e-12 * c_ref
    assert -1e-12 <= (cost - c_ref) / c_ref <= BF16_REL_TOL


@pytest.mark.parametrize("M,N,d,m", [(120, 100, 128, 16), (60, 90, 40, 500)])
def test_model_fp16_gram_form(model_exe, M, N, d, m):
    # the FP16 frames: a valid path within 1e-5 of the oracle's optimum
    X, Y = _gram_case(M, N, d, 3 * M + N)
    r = run_model(model_exe, [(X, Y)], m, precision=3)
    assert r["rc"] == 0 and r["device_error"] == 0, r
    cost, path = r["results"][0]
    c_ref, _ = oracle.full(X, Y)
    assert abs(cost - oracle.path_cost(X, Y, path)) <= 1e-12 * c_ref
    assert -1e-12 <= (cost - c_ref) / c_ref <= 1e-5


@pytest.mark.parametrize("M,N,d,m,prec", [(90, 70, 64, 16, 2), (100, 60, 128, 500, 2), (80, 75, 128, 16, 3)])
def test_wave_model_gram_form(model_exe, wave_exe, M, N, d, m, prec):
    # the real kernels with the matrix-core operation emulated in the device's
    # lane layout: same path as the plain model (both sum the bf16 products
    # in k order in FP32)
    X, Y = _gram_case(M, N, d, 7 * M + N)
    r_wave = run_model(wave_exe, [(X, Y)], m, precision=prec)
    r_plain = run_model(model_exe, [(X, Y)], m, precision=prec)
    assert r_wave["rc"] == 0 and r_wave["device_error"] == 0, r_wave
    assert r_wave["results"][0][1].tolist() == r_plain["results"][0][1].tolist()
    # the FP64 path cost: compensated per-leaf sums on the device, a plain sum in the model
    assert abs(r_wave["results"][0][0] - r_plain["results"][0][0]) <= 1e-12 * r_plain["results"][0][0]


@pytest.mark.parametrize("M,N,d,block,rev,ks", [
    (70, 50, 12, (0, 0, 69, 49), 0, 60),      # one stripe: full phase, then the band tail
    (200, 150, 12, (0, 0, 199, 149), 0, 175),  # four stripes chained through the boundary ring
    (200, 150, 12, (0, 0, 199, 149), 1, 176),  # the same on the reversed series
    (260, 90, 5, (3, 7, 250, 80), 0, 200),     # sub-block, stripes past the triangle, ragged tail
    (150, 140, 64, (0, 0, 149, 139), 1, 150),  # wide frames staged in LDS
])
def test_wave_model_diag_bitwise(wave_exe, M, N, d, block, rev, ks):
    # the real sweep kernel (Algorithm 1) lane by lane: every band value equals
    # the oracle's DiagDTW bit for bit
    X, Y = synth.random_pair(8200 + M + d, M, N, d, "normal")
    rc, derr, out = run_model_diag(wave_exe, X, Y, *block, rev, ks)
    assert rc == 0 and derr == 0
    ref = oracle.diag(X, Y, *block, rev, ks)
    assert np.array_equal(np.isnan(out), np.isnan(ref))
    ok = ~np.isnan(ref)
    assert np.array_equal(out[ok].view(np.int64), ref[ok].view(np.int64))


@pytest.mark.parametrize("M,N,d,m,prec", [(90, 110, 5, 8, 0), (100, 80, 12, 16, 1)])
def test_wave_model_cosine(model_exe, wave_exe, M, N, d, m, prec):
    # the cosine frame cost (Sec. 4.1): the real kernels lane by lane give the
    # oracle's textbook path under the cosine cost in FP64, and the FP32 form
    # lies within 1e-5 of its optimum; the plain-loop model agrees
    X, Y = synth.make_pair(8300, M + d, M, N, d, "chroma")
    for exe in (model_exe, wave_exe):
        r = run_model(exe, [(X, Y)], m, precision=prec, cost=1)
        assert r["rc"] == 0 and r["device_error"] == 0, r
        cost, path = r["results"][0]
        c_ref, p_ref = oracle.full(X, Y, cost="cosine")
        assert oracle.path_cost(X, Y, path, cost="cosine") == pytest.approx(cost, rel=1e-12)
        if prec == 0:
            assert path.tolist() == p_ref.tolist()
            assert abs(cost - c_ref) <= 1e-12 * c_ref
        else:
            assert (cost - c_ref) / c_ref <= 1e-5 and cost >= c_ref * (1 - 1e-12)


@pytest.mark.parametrize("M,N,d,m,prec", [(90, 70, 64, 16, 2), (80, 75, 128, 16, 3)])
def test_wave_model_gram_cosine(model_exe, wave_exe, M, N, d, m, prec):
    # the cosine cost on the matrix-core tile: frames normalised in FP64 at
    # staging, rounded to bf16/fp16, cost max(0, 1 - dot).  The real kernels
    # (matrix-core operation emulated in its lane layout) and the plain model
    # take the same path, whose FP64 cosine cost is reported exactly
    X, Y = synth.make_pair(8400, M + d, M, N, d, "embedding")
    r_wave = run_model(wave_exe, [(X, Y)], m, precision=prec, cost=1)
    r_plain = run_model(model_exe, [(X, Y)], m, precision=prec, cost=1)
    assert r_wave["rc"] == 0 and r_wave["device_error"] == 0, r_wave
    cost, path = r_wave["results"][0]
    assert path.tolist() == r_plain["results"][0][1].tolist()
    assert abs(cost - r_plain["results"][0][0]) <= 1e-12 * cost
    c_ref, _ = oracle.full(X, Y, cost="cosine")
    assert oracle.path_cost(X, Y, path, cost="cosine") == pytest.approx(cost, rel=1e-12)
    print("rel", (cost - c_ref) / c_ref)
    assert -1e-12 <= (cost - c_ref) / c_ref <= (BF16_REL_TOL if prec == 2 else 1e-5)


@pytest.mark.parametrize("M,N,d,fam", [(200, 230, 4, "normal"), (3100, 90, 1, "int3")])
def test_wave_model_leaf_on_several_workgroups(wave_exe, M, N, d, fam):
    # one leaf (m = 500) whose stripes run on the model's two workgroups,
    # chained through the leaf ring: four stripes (ring rows reused, walk
    # through pointer blocks copied into LDS two at a time), and a leaf so
    # wide that two pointer blocks do not fit the LDS (walk from global
    # scratch); continuous and tie-heavy integer frames
    X, Y = synth.random_pair(9300 + M + N, M, N, d, fam)
    r = run_model(wave_exe, [(X, Y)], 500)
    assert r["rc"] == 0 and r["device_error"] == 0, r
    assert r["polls"] > 0
    cost, path = r["results"][0]
    c_ref, p_ref = oracle.full(X, Y)
    assert path.tolist() == p_ref.tolist()
    assert abs(cost - c_ref) <= 1e-12 * c_ref


@pytest.mark.parametrize("M,N,d,fam,m", [(150, 120, 1, "int3", 16), (70, 60, 2, "int3", 3), (260, 90, 1, "int3", 32)])
def test_wave_model_tie_exact(wave_exe, M, N, d, fam, m):
    # tie-exact mode: the real kernels (labelled forward sweeps chained over
    # several stripes, leaves from their origin's value) give the oracle's
    # textbook path bit for bit, also on tie-heavy integer frames where the
    # split of Algorithm 2 leaves it
    X, Y = synth.random_pair(9400 + M + N, M, N, d, fam)
    r = run_model(wave_exe, [(X, Y)], m, tie=1)
    assert r["rc"] == 0 and r["device_error"] == 0, r
    cost, path = r["results"][0]
    c_ref, p_ref = oracle.full(X, Y)
    assert path.tolist() == p_ref.tolist()
    assert abs(cost - c_ref) <= 1e-12 * max(c_ref, 1.0)
    assert oracle.linmdtw_tie(X, Y, min_block=m)["path"].tolist() == p_ref.tolist()


def test_wave_model_batch_keeps_leaves_on_one_workgroup(wave_exe):
    # 18 pairs (more than a call splits leaves for): every leaf, two stripes
    # tall, runs on one workgroup stripe after stripe; each pair's path is the
    # oracle's textbook path
    pairs = [synth.random_pair(9800 + b, 70 + 3 * b, 90 - 2 * b, 3, "normal") for b in range(18)]
    r = run_model(wave_exe, pairs, 500)
    assert r["rc"] == 0 and r["device_error"] == 0, r
    for (X, Y), (cost, path) in zip(pairs, r["results"]):
        c_ref, p_ref = oracle.full(X, Y)
        assert path.tolist() == p_ref.tolist()
        assert abs(cost - c_ref) <= 1e-12 * c_ref
