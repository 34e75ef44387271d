// Host runtime of libdtw_hip.so: argument checks, workspace planning and the
// launch sequence of one alignment (Algorithm 2 of arXiv 2008.02734 run
// level-synchronously, every level's work lists resident on the device).
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "dtw.h"
#include "dtw_internal.h"

namespace dtw {
hipError_t launch_pass(const Work& w, int level, int grid, hipStream_t st);
hipError_t launch_leaf(const Work& w, int grid, int64_t lds_leaf_bytes, const void* Xo, const void* Yo, int in_f64,
                       hipStream_t st);
hipError_t leaf_lds_setup(int64_t lds_max, int64_t* dyn_f64, int64_t* dyn_f32);
hipError_t launch_init(const Work& w, hipStream_t st);
hipError_t launch_store_pair(PairDesc* dst, const PairDesc& v, hipStream_t st);
hipError_t launch_plan(const Work& w, int level, int final_level, int64_t lds_leaf_bytes, hipStream_t st);
hipError_t launch_combine(const Work& w, int grid, hipStream_t st);
hipError_t launch_assemble(const Work& w, int32_t* poff, int32_t* lidx, double* costs, int64_t* lens,
                           int32_t* paths, int grid, hipStream_t st);
hipError_t launch_pad_convert(const void* in, int in_f64, void* out, int out_f64, int64_t rows, int d, int D,
                              hipStream_t st);
hipError_t launch_normalize(const void* in, int in_f64, void* out, int out_f64, int64_t rows, int d, int D,
                            hipStream_t st);
hipError_t launch_gram_stage(const void* in, int in_f64, int64_t rows, int d, int D, int bf16, int cos, uint16_t* out,
                             float* norms,
                             hipStream_t st);
hipError_t launch_nonfinite(const void* in, int in_f64, int64_t n, int32_t* flag, hipStream_t st);
hipError_t launch_diag(const Work& w, int32_t i0, int32_t j0, int32_t i1, int32_t j1, int32_t dir,
                       int32_t kstop, int grid, double* out, hipStream_t st);
int pick_dmax(int d);
int pick_dgram(int d);
}  // namespace dtw

using namespace dtw;

namespace {

thread_local int32_t g_last_hip = 0;

struct DevInfo {
  int cus = 0;
  int lds_max = 0;
  int64_t wall_khz = 0;
  bool attr_set = false;
  int64_t leaf_dyn[2] = {0, 0};  // dynamic LDS of the leaf kernels: FP64, FP32 compute
};

DevInfo& dev_info() {
  static DevInfo info[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  DevInfo& I = info[dev];
  if (I.cus == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) I.cus = v;
    else I.cus = 256;
    v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      I.lds_max = std::min(v, 160 * 1024);
    else
      I.lds_max = 64 * 1024;
    v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) == hipSuccess && v > 0) I.wall_khz = v;
    else I.wall_khz = 100000;
  }
  return I;
}

thread_local bool g_launch_rejected = false;

int env_int(const char* name, int dflt) {
  const char* s = getenv(name);
  if (!s || !*s) return dflt;
  return atoi(s);
}

// Device wall-clock ticks of one boundary wait: `us` microseconds, or 20 s.
uint64_t wait_ticks(const DevInfo& I, int32_t us) {
  const uint64_t lim_us = us > 0 ? (uint64_t)us : 20000000ull;
  return std::max<uint64_t>(1, (uint64_t)I.wall_khz * lim_us / 1000);
}

// Split levels that can occur: a block that is split has both sides >= m, so
// K = Mb + Nb - 1 >= 2m - 1, and each child has K' <= min(K - 1, floor(K/2) + 3)
// (the pivot lies on diagonals kf-2..kf with kf = ceil(K/2)).
int level_bound(int64_t K0, int m) {
  int L = 0;
  int64_t K = K0;
  while (K >= 2 * (int64_t)m - 1) {
    ++L;
    K = std::min(K - 1, K / 2 + 3);
  }
  return L;
}

struct Region {
  size_t off = 0, bytes = 0;
};

struct Layout {
  Caps caps{};
  int lmax = 0;
  int n_pairs = 0;
  bool conv = false;
  int cbytes = 8;  // bytes of the compute type
  int D = 0;       // padded frame stride of the compute copies
  Region ctl, pairs, subs0, subs1, piv_key, piv_pos, smin, passes, tickets, hist, chunk_sub, bandF, bandC,
      bandB, ring, lring, leaves, leaf_scratch, tpath, cnt, poff, lidx, leaf_cost, leaf_tk, leaf_ring, leaf_done, xconv,
      yconv, xnorm, ynorm, nonfinite;
  size_t total = 0;
};

void put(Layout& L, Region& r, size_t bytes) {
  r.off = (L.total + 255) & ~(size_t)255;
  r.bytes = bytes;
  L.total = r.off + bytes;
}

bool valid_precision(int p) { return p == DTW_PREC_FP64 || p == DTW_PREC_FP32 || is_gram_precision(p); }

// Padded frame width of the compute copies for a precision, 0 if unsupported.
int frame_width(int d, int precision) {
  if (d < 1) return 0;
  return is_gram_precision(precision) ? pick_dgram(d) : pick_dmax(d);
}

// Xrows / Yrows: frames of X / Y that the compute copies must cover.
Layout plan_layout(int n_pairs, const std::vector<int64_t>& Ms, const std::vector<int64_t>& Ns, int d,
                   int in_dtype, int precision, int m, int64_t Xrows, int64_t Yrows, int cost, int tie) {
  Layout L;
  L.n_pairs = n_pairs;
  int64_t K0sum = 0, Msum = 0, Nsum = 0, Mmax = 0, sub = 0, leaf = 0;
  for (int b = 0; b < n_pairs; ++b) {
    const int64_t K0 = Ms[b] + Ns[b] - 1;
    K0sum += K0;
    Msum += Ms[b];
    Nsum += Ns[b];
    Mmax = std::max(Mmax, std::max(Ms[b], Ns[b]));
    sub += K0 / (2 * (int64_t)m - 2) + 1;
    leaf += K0 / ((int64_t)m - 2) + 2;
    L.lmax = std::max(L.lmax, level_bound(K0, m));
  }
  Caps& c = L.caps;
  c.sub = sub + 1;
  c.cand = std::max<int64_t>(2 * c.sub, n_pairs);
  c.leaf = leaf + 1;
  c.band = (3 * K0sum) / 2 + (3 + kBandChunk) * c.sub + 3 * Mmax + kBandChunk;
  c.chunk = c.band / kBandChunk + c.sub + 1;
  c.ring = 2 * kRing * (Nsum + c.sub) + kRing * Mmax;
  c.ticket = 2 * ((Msum + kWave - 1) / kWave + 2 * c.sub) + Mmax / kWave + 2;
  c.hist = Mmax / kWave + 3;
  // per leaf: ceil(R/64)*64 <= R+63 rows of ceil((Cc+63)/16) <= Cc/16+5 words, R < m,
  // sum of Cc over leaves <= K0sum + leaves; then 2 words per bottom-row column
  c.leaf_words = (((int64_t)m + kWave) * (K0sum + c.leaf)) / 16 + ((int64_t)m + kWave) * 6 * c.leaf +
                 2 * (K0sum + c.leaf) + 64;
  c.pslots = K0sum;
  // leaf stripes: a leaf's shorter side is below m, so at most ceil((m-1)/64)
  // stripes; a leaf of several stripes has min(stripes - 1, kRing) boundary
  // rows of Cc cells, and the Cc of all leaves sum to at most K0sum + leaves
  c.leaf_tk = c.leaf * (((int64_t)m - 1 + kWave - 1) / kWave) + 1;
  c.leaf_ring = kRing * (K0sum + c.leaf) + 1;
  const bool gram = is_gram_precision(precision);
  const bool f32 = precision == DTW_PREC_FP32 || gram;  // compute type of the recurrence
  L.cbytes = f32 ? 4 : 8;
  L.D = frame_width(d, precision);
  L.conv = gram || (f32 && in_dtype == DTW_F64) || (!f32 && in_dtype == DTW_F32) || (L.D != d) ||
           cost == DTW_COST_COSINE;  // the cosine cost reads normalised copies
  put(L, L.ctl, sizeof(Ctl));  // first, at offset 0: dtw_device_error reads it there
  put(L, L.pairs, sizeof(PairDesc) * n_pairs);
  put(L, L.subs0, sizeof(Block) * c.sub);
  put(L, L.subs1, sizeof(Block) * c.sub);
  put(L, L.piv_key, 8 * c.sub);
  put(L, L.piv_pos, 8 * c.sub);
  put(L, L.smin, 8 * (size_t)n_pairs);
  put(L, L.passes, sizeof(PassDesc) * 2 * c.sub);
  put(L, L.tickets, sizeof(int2) * c.ticket);
  put(L, L.hist, 4 * 4 * c.hist);
  put(L, L.chunk_sub, 4 * c.chunk);
  put(L, L.bandF, 8 * c.band);
  put(L, L.bandC, 8 * c.band);
  put(L, L.bandB, 8 * c.band);
  put(L, L.ring, (size_t)L.cbytes * 2 * c.ring);  // cells of 2 (FP64) or 1 (FP32) 8-byte words
  if (tie) put(L, L.lring, 8 * (size_t)c.ring);     // tie-exact mode: a label word per cell
  put(L, L.leaves, sizeof(LeafDesc) * c.leaf);
  put(L, L.leaf_scratch, 4 * c.leaf_words);
  put(L, L.tpath, 8 * c.pslots);
  put(L, L.cnt, 4 * c.pslots);
  put(L, L.poff, 4 * c.pslots);
  put(L, L.lidx, 4 * c.pslots);
  put(L, L.leaf_cost, 16 * c.leaf);
  put(L, L.leaf_tk, sizeof(int2) * c.leaf_tk);
  put(L, L.leaf_ring, (size_t)L.cbytes * 2 * c.leaf_ring);  // cells as in the sweep ring
  put(L, L.leaf_done, 4 * c.leaf);
  if (L.conv) {
    const size_t eb = gram ? 2 : (size_t)L.cbytes;  // bf16 frames in the Gram form
    put(L, L.xconv, eb * Xrows * L.D);
    put(L, L.yconv, eb * Yrows * L.D);
  }
  if (gram) {
    put(L, L.xnorm, 4 * (size_t)Xrows);
    put(L, L.ynorm, 4 * (size_t)Yrows);
  }
  put(L, L.nonfinite, 4);
  return L;
}

template <typename T>
T* at(void* base, const Region& r) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + r.off);
}

Work make_work(const Layout& L, void* ws, int d, int m, int precision, int cost, int tie) {
  Work w{};
  w.cost = cost;
  w.tie = tie;
  w.leaf_split = L.n_pairs <= kLeafSplitPairs ? 1 : 0;
  w.ctl = at<Ctl>(ws, L.ctl);
  w.pairs = at<PairDesc>(ws, L.pairs);
  w.n_pairs = L.n_pairs;
  w.min_block = m;
  w.d = d;
  w.precision = precision;
  w.subs[0] = at<Block>(ws, L.subs0);
  w.subs[1] = at<Block>(ws, L.subs1);
  w.piv_key = at<uint64_t>(ws, L.piv_key);
  w.piv_pos = at<uint64_t>(ws, L.piv_pos);
  w.smin = at<double>(ws, L.smin);
  w.passes = at<PassDesc>(ws, L.passes);
  w.tickets = at<int2>(ws, L.tickets);
  w.hist = at<int32_t>(ws, L.hist);
  w.chunk_sub = at<int32_t>(ws, L.chunk_sub);
  w.bandF = at<double>(ws, L.bandF);
  w.bandC = at<double>(ws, L.bandC);
  w.bandB = at<double>(ws, L.bandB);
  w.ring = at<uint64_t>(ws, L.ring);
  w.lring = tie ? at<uint64_t>(ws, L.lring) : nullptr;
  w.ring_words = L.cbytes / 4;
  w.leaves = at<LeafDesc>(ws, L.leaves);
  w.leaf_scratch = at<uint32_t>(ws, L.leaf_scratch);
  w.tpath = at<int2>(ws, L.tpath);
  w.cnt = at<int32_t>(ws, L.cnt);
  w.leaf_cost = at<double2>(ws, L.leaf_cost);
  w.leaf_tk = at<int2>(ws, L.leaf_tk);
  w.leaf_ring = at<uint64_t>(ws, L.leaf_ring);
  w.leaf_done = at<int32_t>(ws, L.leaf_done);
  w.caps = L.caps;
  return w;
}

// A failed HIP call returns DTW_ERR_HIP; a launch that check_launch refused
// (it could not run on the device) returns DTW_ERR_INTERNAL.
#define HIP_TRY(expr)                                         \
  do {                                                        \
    g_launch_rejected = false;                                \
    hipError_t e_ = (expr);                                   \
    if (e_ != hipSuccess) {                                   \
      g_last_hip = (int32_t)e_;                               \
      return g_launch_rejected ? DTW_ERR_INTERNAL : DTW_ERR_HIP; \
    }                                                         \
  } while (0)

dtw_status read_opts(const dtw_opts* o, dtw_opts* out) {
  dtw_default_opts(out);
  if (o) *out = *o;
  if (!valid_precision(out->precision)) return DTW_ERR_INVALID_ARG;
  if (out->min_block < 3 || out->min_block > kMaxMinBlock) return DTW_ERR_INVALID_ARG;
  if (out->wait_limit_us < 0) return DTW_ERR_INVALID_ARG;
  if (out->cost != DTW_COST_EUCLIDEAN && out->cost != DTW_COST_COSINE) return DTW_ERR_INVALID_ARG;
  if (out->tie_exact != 0 && out->tie_exact != 1) return DTW_ERR_INVALID_ARG;
  if (out->tie_exact && out->precision != DTW_PREC_FP64) return DTW_ERR_UNSUPPORTED;
  for (int i = 0; i < 1; ++i)
    if (out->reserved[i] != 0) return DTW_ERR_INVALID_ARG;
  return DTW_OK;
}

// Kernel-class timing with HIP events recorded on the caller's stream.
enum ProfClass { kProfSweep = 0, kProfSplit, kProfPlan, kProfLeaf, kProfOther, kProfClasses };
constexpr int kProfEvents = 1024;

struct Profiler {
  bool on = false;
  bool sweep_only = false;  // profile = 2: the sweep launches only (fewer events in the stream)
  bool rec = false;         // the current launch is being timed
  hipStream_t st = nullptr;
  hipEvent_t* ev = nullptr;
  int used = 0;
  int cls[kProfEvents / 2];

  hipError_t init(bool enable, bool sweeps, hipStream_t s) {
    on = enable;
    sweep_only = sweeps;
    st = s;
    if (!on) return hipSuccess;
    static hipEvent_t pools[64][kProfEvents];
    static bool made[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (!made[dev]) {
      for (int i = 0; i < kProfEvents; ++i) {
        hipError_t e = hipEventCreate(&pools[dev][i]);
        if (e != hipSuccess) return e;
      }
      made[dev] = true;
    }
    ev = pools[dev];
    return hipSuccess;
  }
  hipError_t begin(int c) {
    rec = on && used + 2 <= kProfEvents && (!sweep_only || c == kProfSweep);
    if (!rec) return hipSuccess;
    cls[used / 2] = c;
    return hipEventRecord(ev[used], st);
  }
  hipError_t end() {
    if (!rec) return hipSuccess;
    rec = false;
    hipError_t e = hipEventRecord(ev[used + 1], st);
    used += 2;
    return e;
  }
  // after the stream has completed
  hipError_t sums(double* ms) {
    for (int c = 0; c < kProfClasses; ++c) ms[c] = 0.0;
    for (int i = 0; i < used; i += 2) {
      float t = 0.f;
      hipError_t e = hipEventElapsedTime(&t, ev[i], ev[i + 1]);
      if (e != hipSuccess) return e;
      ms[cls[i / 2]] += t;
    }
    return hipSuccess;
  }
};

#define PROF_TRY(P, CLS, expr)     \
  do {                             \
    HIP_TRY((P).begin(CLS));       \
    HIP_TRY(expr);                 \
    HIP_TRY((P).end());            \
  } while (0)

// Compute copies of the inputs when the layout asks for them: padded /
// converted frames for the Euclidean forms, bf16 frames and their FP32
// squared norms for the Gram form.  Points w.X / w.Y (and w.Xn / w.Yn) at
// what the kernels read.
hipError_t stage_inputs(const Layout& L, void* ws, const void* X, const void* Y, int in_f64, int64_t xrows,
                        int64_t yrows, int d, int precision, int cost, Work& w, hipStream_t st) {
  w.X = X;
  w.Y = Y;
  w.Xn = nullptr;
  w.Yn = nullptr;
  if (!L.conv) return hipSuccess;
  void* xc = at<void>(ws, L.xconv);
  void* yc = at<void>(ws, L.yconv);
  hipError_t e;
  if (is_gram_precision(precision)) {
    float* xn = at<float>(ws, L.xnorm);
    float* yn = at<float>(ws, L.ynorm);
    const int bf16 = precision == DTW_PREC_BF16_COST ? 1 : 0;
    const int cos = cost == DTW_COST_COSINE ? 1 : 0;
    e = launch_gram_stage(X, in_f64, xrows, d, L.D, bf16, cos, static_cast<uint16_t*>(xc), xn, st);
    if (e == hipSuccess) e = launch_gram_stage(Y, in_f64, yrows, d, L.D, bf16, cos, static_cast<uint16_t*>(yc), yn, st);
    w.Xn = xn;
    w.Yn = yn;
  } else if (cost == DTW_COST_COSINE) {
    const int out_f64 = precision == DTW_PREC_FP64 ? 1 : 0;
    e = launch_normalize(X, in_f64, xc, out_f64, xrows, d, L.D, st);
    if (e == hipSuccess) e = launch_normalize(Y, in_f64, yc, out_f64, yrows, d, L.D, st);
  } else {
    const int out_f64 = precision == DTW_PREC_FP64 ? 1 : 0;
    e = launch_pad_convert(X, in_f64, xc, out_f64, xrows, d, L.D, st);
    if (e == hipSuccess) e = launch_pad_convert(Y, in_f64, yc, out_f64, yrows, d, L.D, st);
  }
  w.X = xc;
  w.Y = yc;
  return e;
}

// ----------------------------------------------------------------- graphs
//
// The launch sequence of a one-pair call is fixed by its arguments (the
// recursion depth bound lmax, the kernels and their parameters follow from
// the shapes and options; every decision inside is made on the device).  A
// call whose every kernel argument (pointers, sizes, options, device) was
// seen before is recorded once into a graph on a library stream (recording
// runs nothing) and from then on replayed with one launch on the caller's
// stream.  A first sighting runs eagerly, so one-off calls never pay the
// recording.  DTW_GRAPHS=0 in the environment turns replay off.
struct GraphKey {
  int dev;
  const void *X, *Y, *ws;
  size_t ws_bytes;
  double* costs;
  int32_t* paths;
  int64_t* lens;
  int64_t path_cap, M, N;
  int32_t d, in_dtype;
  dtw_opts opts;
  bool same(const GraphKey& o) const {
    return dev == o.dev && X == o.X && Y == o.Y && ws == o.ws && ws_bytes == o.ws_bytes && costs == o.costs &&
           paths == o.paths && lens == o.lens && path_cap == o.path_cap && M == o.M && N == o.N && d == o.d &&
           in_dtype == o.in_dtype && memcmp(&opts, &o.opts, sizeof(dtw_opts)) == 0;
  }
};

struct GraphCache {
  struct Entry {
    GraphKey key;
    hipGraphExec_t exec;
    uint64_t used;
  };
  static constexpr size_t kMaxGraphs = 16, kMaxSeen = 64;
  std::mutex mu;
  std::vector<Entry> graphs;
  std::vector<GraphKey> seen;
  uint64_t clock = 0;
  hipStream_t rec[64] = {};  // per device: the stream calls are recorded on
};
GraphCache& graph_cache() {
  static GraphCache c;
  return c;
}

// The replayable graph of `key`, recording it with `enqueue` when the key
// was seen before; *exec stays null when the call should run eagerly.
template <typename F>
dtw_status graph_for(const GraphKey& key, F&& enqueue, hipGraphExec_t* exec) {
  *exec = nullptr;
  GraphCache& c = graph_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  ++c.clock;
  for (auto& e : c.graphs)
    if (e.key.same(key)) {
      e.used = c.clock;
      *exec = e.exec;
      return DTW_OK;
    }
  bool seen = false;
  for (auto& k : c.seen) seen = seen || k.same(key);
  if (!seen) {
    if (c.seen.size() >= GraphCache::kMaxSeen) c.seen.erase(c.seen.begin());
    c.seen.push_back(key);
    return DTW_OK;
  }
  if (key.dev < 0 || key.dev >= 64) return DTW_OK;
  if (!c.rec[key.dev]) HIP_TRY(hipStreamCreateWithFlags(&c.rec[key.dev], hipStreamNonBlocking));
  hipStream_t rs = c.rec[key.dev];
  if (hipStreamBeginCapture(rs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return DTW_OK;  // no recording on this device: the call runs eagerly
  }
  const dtw_status rc = enqueue(rs);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(rs, &g);
  if (rc != DTW_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  HIP_TRY(ee);
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIP_TRY(ei);
  if (c.graphs.size() >= GraphCache::kMaxGraphs) {
    size_t lru = 0;
    for (size_t i = 1; i < c.graphs.size(); ++i)
      if (c.graphs[i].used < c.graphs[lru].used) lru = i;
    HIP_TRY(hipDeviceSynchronize());  // the evicted graph may still be running
    HIP_TRY(hipGraphExecDestroy(c.graphs[lru].exec));
    c.graphs.erase(c.graphs.begin() + (ptrdiff_t)lru);
  }
  c.graphs.push_back({key, x, c.clock});
  *exec = x;
  return DTW_OK;
}

// Core of dtw_align and dtw_align_batched.
dtw_status run(int n_pairs, const void* X, const void* Y, const int64_t* xo, const int64_t* yo, int d,
               int in_dtype, const dtw_opts* opts_in, void* ws, size_t ws_bytes, double* costs,
               int32_t* paths, const int64_t* path_offsets, int64_t path_cap_single, int64_t* lens,
               dtw_stats* stats, hipStream_t st, int32_t** device_error_word = nullptr,
               bool allow_graph = false) {
  dtw_opts opts;
  dtw_status rc = read_opts(opts_in, &opts);
  if (rc != DTW_OK) return rc;
  if (n_pairs < 1 || !X || !Y || !xo || !yo || !ws || !costs || !paths || !lens) return DTW_ERR_INVALID_ARG;
  if (in_dtype != DTW_F64 && in_dtype != DTW_F32) return DTW_ERR_INVALID_ARG;
  if (d < 1) return DTW_ERR_INVALID_ARG;
  if (frame_width(d, opts.precision) == 0) return DTW_ERR_UNSUPPORTED;
  std::vector<int64_t> Ms(n_pairs), Ns(n_pairs);
  std::vector<PairDesc> pd(n_pairs);
  int64_t pbase = 0, Mtot = 0, Ntot = 0;
  for (int b = 0; b < n_pairs; ++b) {
    Ms[b] = xo[b + 1] - xo[b];
    Ns[b] = yo[b + 1] - yo[b];
    if (Ms[b] < 1 || Ns[b] < 1 || xo[b] < 0 || yo[b] < 0) return DTW_ERR_INVALID_ARG;
    if (xo[b + 1] > INT32_MAX || yo[b + 1] > INT32_MAX) return DTW_ERR_INVALID_ARG;
    const int64_t need = Ms[b] + Ns[b] - 1;
    int64_t out_off = 0;
    if (path_offsets) {
      if (path_offsets[b + 1] - path_offsets[b] < need || path_offsets[b] < 0) return DTW_ERR_CAPACITY;
      out_off = path_offsets[b];
    } else if (path_cap_single < need) {
      return DTW_ERR_CAPACITY;
    }
    pd[b] = PairDesc{xo[b], yo[b], Ms[b], Ns[b], pbase, out_off};
    pbase += need;
    Mtot = std::max(Mtot, xo[b + 1]);
    Ntot = std::max(Ntot, yo[b + 1]);
  }
  const int m = opts.min_block;
  Layout L = plan_layout(n_pairs, Ms, Ns, d, in_dtype, opts.precision, m, Mtot, Ntot, opts.cost, opts.tie_exact);
  if (ws_bytes < L.total) return DTW_ERR_WORKSPACE;
  const bool f32 = opts.precision != DTW_PREC_FP64;  // FP32 recurrence (FP32 and Gram forms)
  const int in_f64 = in_dtype == DTW_F64;
  DevInfo& I = dev_info();
  if (!I.attr_set) {
    HIP_TRY(leaf_lds_setup(I.lds_max, &I.leaf_dyn[0], &I.leaf_dyn[1]));
    I.attr_set = true;
  }

  if (opts.validate_finite) {
    int32_t* flag = at<int32_t>(ws, L.nonfinite);
    HIP_TRY(hipMemsetAsync(flag, 0, 4, st));
    HIP_TRY(launch_nonfinite(X, in_f64, Mtot * d, flag, st));
    HIP_TRY(launch_nonfinite(Y, in_f64, Ntot * d, flag, st));
    int32_t h = 0;
    HIP_TRY(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h) return DTW_ERR_NONFINITE;
  }

  Profiler prof;
  HIP_TRY(prof.init(opts.profile != 0 && stats != nullptr, opts.profile == 2, st));
  Work w = make_work(L, ws, d, m, opts.precision, opts.cost, opts.tie_exact);
  if (device_error_word) *device_error_word = &w.ctl->error;
  w.X = X;
  w.Y = Y;
  w.spin_ticks = wait_ticks(I, opts.wait_limit_us);
  // resident sweep workgroups per CU: two of 10 waves, or four of the Gram form's 4
  const int pass_grid = I.cus * std::max(1, env_int("DTW_PASS_WG_PER_CU", is_gram_precision(opts.precision) ? 4 : 2));
  const int comb_grid = I.cus * 4;
  const int64_t lds_leaf_bytes = I.leaf_dyn[f32 ? 1 : 0];
  PairDesc* pairs_dev = at<PairDesc>(ws, L.pairs);
  auto enqueue = [&](hipStream_t q, Profiler& pr) -> dtw_status {
    PROF_TRY(pr, kProfOther, stage_inputs(L, ws, X, Y, in_f64, Mtot, Ntot, d, opts.precision, opts.cost, w, q));
    if (n_pairs == 1) HIP_TRY(launch_store_pair(pairs_dev, pd[0], q));
    else HIP_TRY(hipMemcpyAsync(pairs_dev, pd.data(), sizeof(PairDesc) * n_pairs, hipMemcpyHostToDevice, q));
    PROF_TRY(pr, kProfOther, launch_init(w, q));
    for (int lvl = 0; lvl <= L.lmax; ++lvl) {
      const int final_level = (lvl == L.lmax) ? 1 : 0;
      PROF_TRY(pr, kProfPlan, launch_plan(w, lvl, final_level, lds_leaf_bytes, q));
      if (final_level) break;
      PROF_TRY(pr, kProfSweep, launch_pass(w, lvl, pass_grid, q));
      if (!opts.tie_exact) PROF_TRY(pr, kProfSplit, launch_combine(w, comb_grid, q));  // tie-exact: the sweep names the split
    }
    PROF_TRY(pr, kProfLeaf, launch_leaf(w, I.cus, lds_leaf_bytes, X, Y, in_f64, q));
    PROF_TRY(pr, kProfOther,
             launch_assemble(w, at<int32_t>(ws, L.poff), at<int32_t>(ws, L.lidx), costs, lens, paths, I.cus * 2, q));
    return DTW_OK;
  };
  hipGraphExec_t exec = nullptr;
  if (allow_graph && n_pairs == 1 && !prof.on && env_int("DTW_GRAPHS", 1) != 0) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const GraphKey key{dev, X, Y, ws, ws_bytes, costs, paths, lens, path_cap_single, Ms[0], Ns[0], d, in_dtype, opts};
    Profiler off;
    rc = graph_for(key, [&](hipStream_t rs) { return enqueue(rs, off); }, &exec);
    if (rc != DTW_OK) return rc;
  }
  if (exec) {
    HIP_TRY(hipGraphLaunch(exec, st));
  } else {
    rc = enqueue(st, prof);
    if (rc != DTW_OK) return rc;
  }

  if (stats) {
    Ctl c{};
    double smin = 0.0;
    int64_t len = 0;
    HIP_TRY(hipMemcpyAsync(&c, w.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&smin, w.smin, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&len, lens, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    memset(stats, 0, sizeof(*stats));
    if (prof.on) {
      double ms[kProfClasses];
      HIP_TRY(prof.sums(ms));
      stats->ms_sweep = ms[kProfSweep];
      stats->ms_split = ms[kProfSplit];
      stats->ms_plan = ms[kProfPlan];
      stats->ms_leaf = ms[kProfLeaf];
      stats->ms_other = ms[kProfOther];
    }
    stats->s_min = smin;
    stats->cost_lowp = (opts.precision == DTW_PREC_FP64) ? 0.0 : smin;
    stats->cells_processed = c.cells + c.leaf_cells;
    stats->sweep_cells = c.cells;
    stats->leaf_cells = c.leaf_cells;
    stats->path_len = len;
    stats->workspace_bytes = (int64_t)L.total;
    stats->levels = c.levels_run;
    stats->leaves = c.n_leaf;
    stats->device_error = c.error;
    if (c.error) return DTW_ERR_INTERNAL;
  }
  return DTW_OK;
}

// ------------------------------------------------------------ no-allocation form
//
// Workspace of dtw_align_noalloc: a fixed array in device memory, one copy per
// GPU, held from the library's load until the process ends.  Host code never
// passes `scratch` itself to a kernel or a copy (in host code the name is a
// host-side stand-in, not a device address): it passes the address that
// hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) unsigned char scratch[DTW_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_dev[64] = {};

// Device address of the current device's `scratch`, looked up once per device
// with that device current.
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

namespace dtw {

void note_hip_error(hipError_t e) { g_last_hip = (int32_t)e; }
int64_t wall_ticks_per_ms() { return dev_info().wall_khz; }
int device_cus() { return dev_info().cus; }

// Compiled resources of each kernel, read once per device; the dynamic LDS
// limit of the leaf kernels is set before their first launch (leaf_lds_setup)
// and the cache entry is taken after that.
hipError_t check_launch(const void* fn, int grid, int threads, size_t dyn_lds) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, hipFuncAttributes> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  hipFuncAttributes a{};
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({dev, fn});
    if (it == cache.end()) {
      const hipError_t e = hipFuncGetAttributes(&a, fn);
      if (e != hipSuccess) return e;
      cache.emplace(std::make_pair(dev, fn), a);
    } else {
      a = it->second;
    }
  }
  const int64_t lds_max = dev_info().lds_max;
  const bool ok = grid >= 1 && threads >= 1 && threads <= a.maxThreadsPerBlock &&
                  (int64_t)a.sharedSizeBytes + (int64_t)dyn_lds <= lds_max &&
                  (dyn_lds == 0 || (int64_t)dyn_lds <= (int64_t)a.maxDynamicSharedSizeBytes);
  if (!ok) {
    g_launch_rejected = true;
    return hipErrorInvalidConfiguration;
  }
  return hipSuccess;
}

bool launch_rejected() { return g_launch_rejected; }

// Entry points of the serving loop (dtw_server.hip): workspace of a batch,
// and the batch enqueued on a stream without any host synchronisation; the
// device error word of the batch is returned for a later asynchronous read.
dtw_status batch_workspace(int32_t B, const int64_t* x_offsets, const int64_t* y_offsets, int32_t d,
                           int32_t in_dtype, const dtw_opts* opts, size_t* bytes) {
  return dtw_workspace_size_batched(B, x_offsets, y_offsets, d, in_dtype, opts, bytes);
}
dtw_status enqueue_batch(int32_t B, const void* X, const int64_t* xo, const void* Y, const int64_t* yo, int32_t d,
                         int32_t in_dtype, const dtw_opts* opts, void* ws, size_t ws_bytes, double* costs,
                         int32_t* paths, const int64_t* path_offsets, int64_t* lens, hipStream_t st,
                         int32_t** device_error_word) {
  dtw_opts o;
  dtw_status rc = read_opts(opts, &o);
  if (rc != DTW_OK) return rc;
  o.validate_finite = 0;  // the serving loop never synchronises
  o.profile = 0;
  return run(B, X, Y, xo, yo, d, in_dtype, &o, ws, ws_bytes, costs, paths, path_offsets, 0, lens, nullptr, st,
             device_error_word);
}
}  // namespace dtw

extern "C" {

void dtw_default_opts(dtw_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->precision = DTW_PREC_FP64;
  o->min_block = 500;
  o->validate_finite = 0;
  o->profile = 0;
}

const char* dtw_status_string(int32_t s) {
  switch (s) {
    case DTW_OK: return "ok";
    case DTW_ERR_INVALID_ARG: return "invalid argument";
    case DTW_ERR_CAPACITY: return "path capacity too small";
    case DTW_ERR_WORKSPACE: return "workspace too small";
    case DTW_ERR_NONFINITE: return "non-finite input";
    case DTW_ERR_HIP: return "HIP runtime error";
    case DTW_ERR_BUSY: return "not ready";
    case DTW_ERR_NOT_FOUND: return "unknown ticket";
    case DTW_ERR_UNSUPPORTED: return "unsupported dimension or mode";
    case DTW_ERR_INTERNAL: return "device-side consistency check failed";
    default: return "unknown status";
  }
}

int32_t dtw_last_hip_error(void) { return g_last_hip; }

dtw_status dtw_workspace_size(int64_t M, int64_t N, int32_t d, int32_t in_dtype, const dtw_opts* opts_in,
                              size_t* bytes) {
  dtw_opts opts;
  dtw_status rc = read_opts(opts_in, &opts);
  if (rc != DTW_OK) return rc;
  if (!bytes || M < 1 || N < 1 || d < 1 || M > INT32_MAX || N > INT32_MAX) return DTW_ERR_INVALID_ARG;
  if (in_dtype != DTW_F64 && in_dtype != DTW_F32) return DTW_ERR_INVALID_ARG;
  if (frame_width(d, opts.precision) == 0) return DTW_ERR_UNSUPPORTED;
  std::vector<int64_t> Ms{M}, Ns{N};
  *bytes = plan_layout(1, Ms, Ns, d, in_dtype, opts.precision, opts.min_block, M, N, opts.cost, opts.tie_exact).total;
  return DTW_OK;
}

dtw_status dtw_align(const void* X, int64_t M, const void* Y, int64_t N, int32_t d, int32_t in_dtype,
                     const dtw_opts* opts, void* workspace, size_t ws_bytes, double* cost_out,
                     int32_t* path_out, int64_t path_cap, int64_t* path_len_out, dtw_stats* stats,
                     void* stream) {
  if (M < 1 || N < 1) return DTW_ERR_INVALID_ARG;
  const int64_t xo[2] = {0, M}, yo[2] = {0, N};
  return run(1, X, Y, xo, yo, d, in_dtype, opts, workspace, ws_bytes, cost_out, path_out, nullptr, path_cap,
             path_len_out, stats, (hipStream_t)stream, nullptr, /*allow_graph=*/true);
}

dtw_status dtw_align_noalloc(const void* X, int64_t M, const void* Y, int64_t N, int32_t d, int32_t in_dtype,
                             const dtw_opts* opts, double* cost_out, int32_t* path_out, int64_t path_cap,
                             int64_t* path_len_out, dtw_stats* stats, void* stream) {
  if (M < 1 || N < 1 || !X || !Y || !cost_out || !path_out || !path_len_out) return DTW_ERR_INVALID_ARG;
  if (opts && opts->profile != 0) return DTW_ERR_INVALID_ARG;  // the profiler creates events
  if (path_cap < M + N - 1) return DTW_ERR_CAPACITY;
  size_t need = 0;
  dtw_status rc = dtw_workspace_size(M, N, d, in_dtype, opts, &need);
  if (rc != DTW_OK) return rc;
  if (need > (size_t)DTW_NOALLOC_SCRATCH_BYTES) return DTW_ERR_WORKSPACE;
  void* ws = nullptr;
  HIP_TRY(scratch_address(&ws));
  const int64_t xo[2] = {0, M}, yo[2] = {0, N};
  return run(1, X, Y, xo, yo, d, in_dtype, opts, ws, (size_t)DTW_NOALLOC_SCRATCH_BYTES, cost_out, path_out,
             nullptr, path_cap, path_len_out, stats, (hipStream_t)stream);
}

int32_t dtw_graph_count(void) {
  GraphCache& c = graph_cache();
  std::lock_guard<std::mutex> lock(c.mu);
  return (int32_t)c.graphs.size();
}

dtw_status dtw_device_error(const void* workspace, int32_t* code, void* stream) {
  if (!workspace || !code) return DTW_ERR_INVALID_ARG;
  // the control block is the first region of every workspace (plan_layout)
  int32_t v = 0;
  HIP_TRY(hipMemcpyAsync(&v, static_cast<const char*>(workspace) + offsetof(Ctl, error), sizeof(v),
                         hipMemcpyDeviceToHost, (hipStream_t)stream));
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  *code = v;
  return DTW_OK;
}

dtw_status dtw_workspace_size_batched(int32_t B, const int64_t* x_offsets, const int64_t* y_offsets, int32_t d,
                                      int32_t in_dtype, const dtw_opts* opts_in, size_t* bytes) {
  dtw_opts opts;
  dtw_status rc = read_opts(opts_in, &opts);
  if (rc != DTW_OK) return rc;
  if (!bytes || B < 1 || !x_offsets || !y_offsets || d < 1) return DTW_ERR_INVALID_ARG;
  if (in_dtype != DTW_F64 && in_dtype != DTW_F32) return DTW_ERR_INVALID_ARG;
  if (frame_width(d, opts.precision) == 0) return DTW_ERR_UNSUPPORTED;
  std::vector<int64_t> Ms(B), Ns(B);
  int64_t Xrows = 0, Yrows = 0;
  for (int b = 0; b < B; ++b) {
    Ms[b] = x_offsets[b + 1] - x_offsets[b];
    Ns[b] = y_offsets[b + 1] - y_offsets[b];
    if (Ms[b] < 1 || Ns[b] < 1 || x_offsets[b] < 0 || y_offsets[b] < 0) return DTW_ERR_INVALID_ARG;
    Xrows = std::max(Xrows, x_offsets[b + 1]);
    Yrows = std::max(Yrows, y_offsets[b + 1]);
  }
  *bytes = plan_layout(B, Ms, Ns, d, in_dtype, opts.precision, opts.min_block, Xrows, Yrows, opts.cost, opts.tie_exact).total;
  return DTW_OK;
}

dtw_status dtw_align_batched(int32_t B, const void* X_packed, const int64_t* x_offsets, const void* Y_packed,
                             const int64_t* y_offsets, int32_t d, int32_t in_dtype, const dtw_opts* opts,
                             void* workspace, size_t ws_bytes, double* costs_out, int32_t* paths_out,
                             const int64_t* path_offsets, int64_t* path_lens_out, dtw_stats* stats,
                             void* stream) {
  if (B < 1 || !x_offsets || !y_offsets || !path_offsets) return DTW_ERR_INVALID_ARG;
  return run(B, X_packed, Y_packed, x_offsets, y_offsets, d, in_dtype, opts, workspace, ws_bytes, costs_out,
             paths_out, path_offsets, 0, path_lens_out, stats, (hipStream_t)stream);
}

dtw_status dtw_diag(const void* X, const void* Y, int32_t d, int32_t in_dtype, int64_t i0, int64_t j0, int64_t i1,
                    int64_t j1, int32_t reverse, int64_t kstop, int32_t precision, void* workspace,
                    size_t ws_bytes, double* out, void* stream) {
  if (!X || !Y || !workspace || !out || d < 1 || i0 < 0 || j0 < 0 || i1 < i0 || j1 < j0) return DTW_ERR_INVALID_ARG;
  if (i1 > INT32_MAX || j1 > INT32_MAX) return DTW_ERR_INVALID_ARG;
  if (in_dtype != DTW_F64 && in_dtype != DTW_F32) return DTW_ERR_INVALID_ARG;
  if (!valid_precision(precision)) return DTW_ERR_UNSUPPORTED;
  if (frame_width(d, precision) == 0) return DTW_ERR_UNSUPPORTED;
  const int64_t Mb = i1 - i0 + 1, Nb = j1 - j0 + 1;
  if (kstop < 2 || kstop > Mb + Nb - 2) return DTW_ERR_INVALID_ARG;
  const int in_f64 = in_dtype == DTW_F64;
  std::vector<int64_t> Ms{Mb}, Ns{Nb};
  // same layout as dtw_workspace_size(i1+1, j1+1, d, in_dtype, opts with this precision)
  Layout L = plan_layout(1, Ms, Ns, d, in_dtype, precision, 500, i1 + 1, j1 + 1, DTW_COST_EUCLIDEAN, 0);
  {
    std::vector<int64_t> Mf{i1 + 1}, Nf{j1 + 1};
    Layout Lf = plan_layout(1, Mf, Nf, d, in_dtype, precision, 500, i1 + 1, j1 + 1, DTW_COST_EUCLIDEAN, 0);
    if (Lf.total > L.total) L = Lf;
  }
  if (ws_bytes < L.total) return DTW_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  Work w = make_work(L, workspace, d, 500, precision, DTW_COST_EUCLIDEAN, 0);
  HIP_TRY(stage_inputs(L, workspace, X, Y, in_f64, i1 + 1, j1 + 1, d, precision, DTW_COST_EUCLIDEAN, w, st));
  w.bandC = nullptr;
  DevInfo& I = dev_info();
  w.spin_ticks = wait_ticks(I, 0);
  HIP_TRY(launch_diag(w, (int32_t)i0, (int32_t)j0, (int32_t)i1, (int32_t)j1, reverse ? 1 : 0, (int32_t)kstop,
                      I.cus * (is_gram_precision(precision) ? 4 : 2), out, st));
  return DTW_OK;
}

}  // extern "C"
