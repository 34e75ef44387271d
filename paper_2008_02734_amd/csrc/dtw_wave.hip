// HIP wave kernels for gfx950: the anti-diagonal wavefront sweep (DiagDTW,
// Algorithm 1 of arXiv 2008.02734) and the leaf solve (textbook DTW with
// backpointers and backtrace, Sec. 2.1).  One wavefront owns 64 DP rows; the
// wave-level primitives (DPP lane shift, readfirstlane, scalar frame loads)
// live only in this file.
#include "dtw_common.h"

#pragma clang fp contract(off)

namespace dtw {

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// FP64: the correctly rounded square root (LLVM's f64 sqrt expansion for gfx9).
__device__ __forceinline__ double sqrt_t(double s) { return __builtin_sqrt(s); }
// FP32 precision mode: the hardware square root.
__device__ __forceinline__ float sqrt_t(float s) { return __builtin_amdgcn_sqrtf(s); }
// Exact minimum of two non-NaN values: one v_min instruction (the builtin
// would canonicalise both inputs first under IEEE mode).
__device__ __forceinline__ double min_t(double a, double b) {
  double r;
  asm volatile("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float min_t(float a, float b) {
  float r;
  asm volatile("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

template <typename T> __device__ __forceinline__ T inf_t();
template <> __device__ __forceinline__ double inf_t<double>() { return __builtin_inf(); }
template <> __device__ __forceinline__ float inf_t<float>() { return __builtin_inff(); }

// DPP wave_shr:1 -- lane l receives lane l-1's value; lane 0 (no source
// lane) keeps `old`, which carries the boundary value of the stripe above.
constexpr int kDppWaveShr1 = 0x138;
__device__ __forceinline__ double wave_shr1(double old, double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), kDppWaveShr1, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), kDppWaveShr1, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float wave_shr1(float old, float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), kDppWaveShr1, 0xf, 0xf, false));
}

// Euclidean frame cost (Sec. 4.1): sum over t of fma(e, e, s), e = x_t - y_t,
// in dimension order, then the square root.  Frames are zero-padded to D
// dimensions; a padded dimension contributes fma(0, 0, s) = s exactly.  x is
// the lane's own frame in registers; y is a wave-uniform frame (scalar loads).
template <typename T, int D>
__device__ __forceinline__ T frame_cost(const T (&x)[D], const T* __restrict__ y) {
  T s = T(0);
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const T e = x[k] - y[k];
    s = fma_t(e, e, s);
  }
  return sqrt_t(s);
}

// ----------------------------------------------------------------- pass kernel
//
// One wave owns a stripe of 64 consecutive local rows of one sweep; lane r is
// row a = 64*s + r.  At step t lane r evaluates column b = t - r, so the wave
// advances along anti-diagonals exactly as Algorithm 1 does.  Each step:
//   (A) the frame cost of column t for all 64 rows (the column's Y frame is
//       wave-uniform and arrives through scalar loads), written to an LDS
//       ring indexed by column;
//   (B) the recurrence for cell (a, t - r): UP from lane r-1 by a DPP lane
//       shift, DIAG = the UP value of the previous step, LEFT = own last value.
// Row 64*s - 1 (the stripe above) arrives through a boundary row in HBM that
// the previous stripe publishes kChunkCols columns at a time behind a flag.
// Stripes are dequeued from a queue ordered stripe-major across all sweeps of
// the level, so a stripe only ever waits on a stripe that was dequeued before
// it by a running wave: the persistent grid cannot deadlock.

// Boundary row of the stripe above, kChunkCols columns starting at `col`:
// wait for the chunk's flag, then copy it into the LDS ring `bring` that lane
// 0 reads one value per step.  The wait is bounded by the device wall clock
// (w.spin_ticks); on expiry the wave records an error and carries on, so a
// broken protocol ends the kernel instead of hanging it.
template <typename T>
__device__ __forceinline__ void fetch_chunk(const T* ring_in, const uint32_t* flag_in, uint32_t tag, int col,
                                            int Nb, T* bring, int lane, const Work& w) {
  const int ch = col / kChunkCols;
  if (__hip_atomic_load(flag_in + ch, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != tag) {
    const uint64_t t0 = wall_clock64();
    for (uint32_t it = 0;; ++it) {
      if (__hip_atomic_load(flag_in + ch, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == tag) break;
      __builtin_amdgcn_s_sleep(2);
      if (wall_clock64() - t0 > w.spin_ticks || it > kSpinIterCap) {
        set_error(w.ctl, kErrSpinTimeout);
        break;
      }
    }
  }
  const int c = col + lane;
  if (lane < kChunkCols && c < Nb) bring[c & (kWave - 1)] = ring_in[c];
}

template <typename T, int D>
__global__ __launch_bounds__(kWave) void pass_kernel(const T* __restrict__ X, const T* __restrict__ Y, Work w,
                                                     int level) {
  __shared__ T cring[kWave * kWave];  // frame cost, [column & 63][lane]
  __shared__ T bring[kWave];          // boundary row, [column & 63]
  const int lane = threadIdx.x;
  Ctl* ctl = w.ctl;
  const int n_tickets = clamp_count(ctl, ctl->n_tickets, w.caps.ticket);
  const int n_pass = clamp_count(ctl, ctl->n_pass, 2 * w.caps.sub);
  const T INF = inf_t<T>();

  for (int iter = 0; iter <= n_tickets; ++iter) {  // each iteration consumes one ticket
    int tk = 0;
    if (lane == 0) tk = atomicAdd(&ctl->ticket, 1);
    tk = __builtin_amdgcn_readfirstlane(__shfl(tk, 0));
    if (tk >= n_tickets || tk < 0) break;
    const int2 tv = w.tickets[tk];
    const int p = __builtin_amdgcn_readfirstlane(tv.x);
    const int s = __builtin_amdgcn_readfirstlane(tv.y);
    if (p < 0 || p >= n_pass) {
      if (lane == 0) set_error(ctl, kErrBadPass);
      continue;
    }
    const PassDesc P = w.passes[p];
    if (P.Mb != P.i1 - P.i0 + 1 || P.Nb != P.j1 - P.j0 + 1 || P.Mb < 1 || P.Nb < 1 || P.kstop < 0 ||
        P.kstop > P.Mb + P.Nb - 2 || P.n_rows != min(P.Mb - 1, P.kstop) + 1 || s < 0 || s >= P.n_stripes ||
        P.n_stripes != (P.n_rows + kWave - 1) / kWave) {
      if (lane == 0) set_error(ctl, kErrBadPass);
      continue;
    }

    const int a0 = s * kWave;
    const int a = a0 + lane;
    const int last_row = min(a0 + kWave - 1, P.n_rows - 1);
    const bool row_ok = a <= last_row;
    const int Lr = last_row - a0;
    const int bmax_first = min(P.Nb - 1, P.kstop - a0);
    const int bmax = row_ok ? min(P.Nb - 1, P.kstop - a) : -1;
    const int n_steps = min(P.Nb - 1 + Lr, P.kstop - a0) + 1;
    const int K = P.Mb + P.Nb - 1;
    const int jbase = P.dir ? P.j1 : P.j0;
    const int jstep = P.dir ? -1 : 1;

    T x[D];
    {
      const int gi = P.dir ? P.i1 - (row_ok ? a : 0) : P.i0 + (row_ok ? a : 0);
      const T* xr = X + (int64_t)gi * D;
#pragma unroll
      for (int k = 0; k < D; ++k) x[k] = xr[k];
    }

    const bool has_pred = s > 0;
    const bool has_succ = s + 1 < P.n_stripes;
    const uint32_t my_tag = ((uint32_t)(level + 1) << 20) | (uint32_t)(s + 1);
    const uint32_t pred_tag = my_tag - 1u;
    const int nch = (P.Nb + kChunkCols - 1) / kChunkCols;
    T* ring = static_cast<T*>(w.ring) + P.ring_off;
    T* ring_out = ring + (int64_t)(s % kRing) * P.Nb;
    const T* ring_in = ring + (int64_t)((s + kRing - 1) % kRing) * P.Nb;
    uint32_t* flag_out = w.flags + P.flag_off + (int64_t)(s % kRing) * nch;
    const uint32_t* flag_in = w.flags + P.flag_off + (int64_t)((s + kRing - 1) % kRing) * nch;

    // prologue: column 0 costs and the first boundary chunk
    {
      const int gj = __builtin_amdgcn_readfirstlane(jbase);
      cring[lane] = frame_cost<T, D>(x, Y + (int64_t)gj * D);
      if (has_pred) fetch_chunk(ring_in, flag_in, pred_tag, 0, P.Nb, bring, lane, w);
    }

    T f = T(0);       // own F(a, b-1)
    T up_prev = INF;  // F(a-1, b-1)
    for (int t = 0; t < n_steps; ++t) {
      const int b = t - lane;
      // reads for this step, before the writes below reuse their slots
      const T c = cring[(b & (kWave - 1)) * kWave + lane];
      const T bv = has_pred ? bring[t & (kWave - 1)] : INF;
      // frame cost of the next column, all 64 rows
      if (t + 1 <= bmax_first) {
        const int gj = __builtin_amdgcn_readfirstlane(jbase + jstep * (t + 1));
        cring[((t + 1) & (kWave - 1)) * kWave + lane] = frame_cost<T, D>(x, Y + (int64_t)gj * D);
        if (has_pred && ((t + 1) % kChunkCols) == 0)
          fetch_chunk(ring_in, flag_in, pred_tag, t + 1, P.Nb, bring, lane, w);
      }
      // recurrence on the skewed diagonal: UP from lane-1 (lane 0: the row above)
      const T up = wave_shr1(bv, f);
      if (row_ok && b >= 0 && b <= bmax) {
        const T diag = (b == 0) ? INF : up_prev;
        const T left = (b == 0) ? INF : f;
        const T m = min_t(min_t(diag, up), left);
        f = (a == 0 && b == 0) ? c : m + c;
        const int k = a + b;
        if (k >= P.kstop - 2) {
          if (P.dir == 0 || P.raw) {
            const int q = k - (P.kstop - 2);
            const int lo = max(0, k - (P.Nb - 1));
            const int64_t idx = P.band_off + (int64_t)q * P.L + (a - lo);
            w.bandF[idx] = (double)f;
            if (w.bandC) w.bandC[idx] = (double)c;
          } else {
            const int kfw = K - 1 - k;
            const int q = kfw - (P.kf - 2);
            const int af = P.Mb - 1 - a;
            const int lo = max(0, kfw - (P.Nb - 1));
            w.bandB[P.band_off + (int64_t)q * P.L + (af - lo)] = (double)f;
          }
        }
        if (has_succ && lane == kWave - 1) {
          ring_out[b] = f;
          if ((b % kChunkCols) == kChunkCols - 1 || b == bmax)
            __hip_atomic_store(flag_out + b / kChunkCols, my_tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      up_prev = up;
    }
  }
}

// ----------------------------------------------------------------- leaf

// Textbook DTW on one leaf block by one wave: the shorter side is the row
// dimension (so one wave sweeps it in ceil(R/64) passes of 64 rows), the
// longer side the column dimension.  When the block is transposed (rows = Y
// frames), the UP/LEFT roles swap; the stored 2-bit codes always use the
// original meaning: 0 DIAG (i-1,j-1), 1 UP (i-1,j), 2 LEFT (i,j-1), chosen
// DIAG, then UP, then LEFT on ties.  Row 0 of X moves LEFT, column 0 of Y UP.
template <typename T, int D>
__global__ __launch_bounds__(kLeafThreads) void leaf_kernel(const T* __restrict__ X, const T* __restrict__ Y,
                                                           Work w, int64_t lds_leaf_bytes, const void* Xorig,
                                                           const void* Yorig, int in_f64, int d) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* cring = reinterpret_cast<T*>(lds_raw);
  T* bring = cring + kWave * kWave;
  uint32_t* lds_free = reinterpret_cast<uint32_t*>(bring + kWave);
  const int lane = threadIdx.x;
  Ctl* ctl = w.ctl;
  const int n_leaf = clamp_count(ctl, ctl->n_leaf, w.caps.leaf);
  const T INF = inf_t<T>();

  for (int iter = 0; iter <= n_leaf; ++iter) {  // each iteration consumes one ticket
    int tk = 0;
    if (lane == 0) tk = atomicAdd(&ctl->leaf_ticket, 1);
    tk = __builtin_amdgcn_readfirstlane(__shfl(tk, 0));
    if (tk >= n_leaf || tk < 0) break;
    const LeafDesc Lf = w.leaves[tk];
    if (Lf.pair < 0 || Lf.pair >= w.n_pairs) {
      if (lane == 0) set_error(ctl, kErrBadLeaf);
      continue;
    }
    const PairDesc pd = w.pairs[Lf.pair];
    const int Mb = Lf.i1 - Lf.i0 + 1, Nb = Lf.j1 - Lf.j0 + 1;
    // a leaf lies inside its pair and is non-empty; refuse anything else
    if (Mb < 1 || Nb < 1 || Lf.i0 < pd.x_off || Lf.j0 < pd.y_off || Lf.i1 >= pd.x_off + pd.M ||
        Lf.j1 >= pd.y_off + pd.N) {
      if (lane == 0) set_error(ctl, kErrBadLeaf);
      continue;
    }
    const bool tr = Mb > Nb;
    const int R = tr ? Nb : Mb, Cc = tr ? Mb : Nb;
    const T* __restrict__ RowSrc = tr ? Y : X;
    const T* __restrict__ ColSrc = tr ? X : Y;
    const int r0 = tr ? Lf.j0 : Lf.i0, c0 = tr ? Lf.i0 : Lf.j0;
    const int stride = (Cc + 15) / 16;
    const int64_t bpw = (((int64_t)R * stride) + 1) & ~(int64_t)1;
    uint32_t* bp = (Lf.scratch_off < 0) ? lds_free : (w.leaf_scratch + Lf.scratch_off);
    T* brow = reinterpret_cast<T*>(bp + bpw);
    T fend = T(0);

    for (int sw = 0; sw < R; sw += kWave) {
      const int a = sw + lane;
      const bool row_ok = a < R;
      const int Lr = min(kWave - 1, R - 1 - sw);
      const int n_steps = Cc + Lr;
      const bool has_pred = sw > 0;
      const bool has_succ = sw + kWave < R;
      T x[D];
      {
        const T* xr = RowSrc + (int64_t)(r0 + (row_ok ? a : 0)) * D;
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = xr[k];
      }
      {
        const int gj = __builtin_amdgcn_readfirstlane(c0);
        cring[lane] = frame_cost<T, D>(x, ColSrc + (int64_t)gj * D);
        if (has_pred && lane < kChunkCols && lane < Cc) bring[lane] = brow[lane];
      }
      T f = T(0), up_prev = INF;
      uint32_t word = 0;
      for (int t = 0; t < n_steps; ++t) {
        const int b = t - lane;
        const T c = cring[(b & (kWave - 1)) * kWave + lane];
        const T bv = has_pred ? bring[t & (kWave - 1)] : INF;
        if (t + 1 < Cc) {
          const int gj = __builtin_amdgcn_readfirstlane(c0 + t + 1);
          cring[((t + 1) & (kWave - 1)) * kWave + lane] = frame_cost<T, D>(x, ColSrc + (int64_t)gj * D);
          if (has_pred && ((t + 1) % kChunkCols) == 0) {
            const int col = t + 1 + lane;
            if (lane < kChunkCols && col < Cc) bring[col & (kWave - 1)] = brow[col];
          }
        }
        const T up = wave_shr1(bv, f);
        if (row_ok && b >= 0 && b < Cc) {
          const T diag = (b == 0) ? INF : up_prev;
          const T left = (b == 0) ? INF : f;
          uint32_t code;
          if (diag <= up && diag <= left) code = 0u;
          else if (tr ? (left <= up) : (up <= left)) code = 1u;
          else code = 2u;
          const T m = min_t(min_t(diag, up), left);
          f = (a == 0 && b == 0) ? c : m + c;
          word |= code << (2 * (b & 15));
          if ((b & 15) == 15 || b == Cc - 1) {
            bp[(int64_t)a * stride + (b >> 4)] = word;
            word = 0u;
          }
          if (has_succ && lane == kWave - 1) brow[b] = f;
          if (a == R - 1 && b == Cc - 1) fend = f;
        }
        up_prev = up;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_s_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }

    // backtrace from the block's last cell, writing cells backwards into the
    // diagonal-indexed path scratch (the end cell sits on diagonal e)
    const int64_t e = (int64_t)(Lf.i1 - pd.x_off) + (Lf.j1 - pd.y_off);
    const int64_t slot_end = pd.pbase + e;
    int cnt_written = 0;
    fend = __shfl(fend, (R - 1) % kWave);
    if (lane == 0) {
      int ri = R - 1, cj = Cc - 1;
      for (int guard = 0; guard < R + Cc; ++guard) {  // every step decrements ri or cj
        const bool at_start = (ri == 0 && cj == 0);
        if (!at_start || Lf.first) {
          const int gi = tr ? (Lf.i0 + cj) : (Lf.i0 + ri);
          const int gj = tr ? (Lf.j0 + ri) : (Lf.j0 + cj);
          w.tpath[slot_end - cnt_written] = make_int2((int)(gi - pd.x_off), (int)(gj - pd.y_off));
          ++cnt_written;
        }
        if (at_start) break;
        if (ri == 0) { --cj; continue; }  // first row / column: the only move
        if (cj == 0) { --ri; continue; }
        const uint32_t code = (bp[(int64_t)ri * stride + (cj >> 4)] >> (2 * (cj & 15))) & 3u;
        if (code == 0u) { --ri; --cj; }
        else if (code == 1u) { if (tr) --cj; else --ri; }
        else { if (tr) --ri; else --cj; }
      }
      w.cnt[slot_end] = cnt_written;
      atomicAdd((unsigned long long*)&ctl->leaf_cells, (unsigned long long)((int64_t)R * Cc));
      if (Lf.first && Lf.i1 == pd.x_off + pd.M - 1 && Lf.j1 == pd.y_off + pd.N - 1)
        w.smin[Lf.pair] = (double)fend;
    }
    // FP64 cost of the cells this leaf wrote, from the caller's inputs
    cnt_written = __shfl(cnt_written, 0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    double2 acc = make_double2(0.0, 0.0);
    for (int q = lane; q < cnt_written; q += kWave) {
      const int2 cell = w.tpath[slot_end - cnt_written + 1 + q];
      const int64_t gi = pd.x_off + cell.x, gj = pd.y_off + cell.y;
      double ss = 0.0;
      if (in_f64) {
        const double* xr = static_cast<const double*>(Xorig) + gi * d;
        const double* yr = static_cast<const double*>(Yorig) + gj * d;
        for (int k = 0; k < d; ++k) { const double ee = xr[k] - yr[k]; ss = __builtin_fma(ee, ee, ss); }
      } else {
        const float* xr = static_cast<const float*>(Xorig) + gi * d;
        const float* yr = static_cast<const float*>(Yorig) + gj * d;
        for (int k = 0; k < d; ++k) { const double ee = (double)xr[k] - (double)yr[k]; ss = __builtin_fma(ee, ee, ss); }
      }
      acc = two_sum_acc(acc, __builtin_sqrt(ss));
    }
    // fixed-order tree reduction over the wave
    for (int off = 1; off < kWave; off <<= 1) {
      const double2 other = make_double2(__shfl_xor(acc.x, off), __shfl_xor(acc.y, off));
      acc = ((lane & off) == 0) ? dd_add(acc, other) : dd_add(other, acc);
    }
    if (lane == 0) w.leaf_cost[tk] = acc;
  }
}

// ----------------------------------------------------------------- launchers

int pick_dmax(int d) {
  if (d <= 4) return 4;
  if (d <= 8) return 8;
  if (d <= 12) return 12;
  if (d <= 16) return 16;
  if (d <= 24) return 24;
  if (d <= 32) return 32;
  return 0;
}

#define DTW_DISPATCH_DMAX(DM, CALL) \
  switch (DM) {                     \
    case 4: { constexpr int D_ = 4; CALL; } break;   \
    case 8: { constexpr int D_ = 8; CALL; } break;   \
    case 12: { constexpr int D_ = 12; CALL; } break; \
    case 16: { constexpr int D_ = 16; CALL; } break; \
    case 24: { constexpr int D_ = 24; CALL; } break; \
    case 32: { constexpr int D_ = 32; CALL; } break; \
    default: return hipErrorInvalidValue;            \
  }

hipError_t launch_pass(const Work& w, int level, bool f32, int grid, hipStream_t st) {
  const int dm = pick_dmax(w.d);
  if (f32) {
    DTW_DISPATCH_DMAX(dm, (pass_kernel<float, D_><<<grid, kWave, 0, st>>>(
                              static_cast<const float*>(w.X), static_cast<const float*>(w.Y), w, level)))
  } else {
    DTW_DISPATCH_DMAX(dm, (pass_kernel<double, D_><<<grid, kWave, 0, st>>>(
                              static_cast<const double*>(w.X), static_cast<const double*>(w.Y), w, level)))
  }
  return hipGetLastError();
}

hipError_t launch_leaf(const Work& w, bool f32, int grid, size_t lds_bytes, int64_t lds_leaf_bytes,
                       const void* Xo, const void* Yo, int in_f64, hipStream_t st) {
  const int dm = pick_dmax(w.d);
  if (f32) {
    DTW_DISPATCH_DMAX(dm, (leaf_kernel<float, D_><<<grid, kLeafThreads, lds_bytes, st>>>(
                              static_cast<const float*>(w.X), static_cast<const float*>(w.Y), w, lds_leaf_bytes,
                              Xo, Yo, in_f64, w.d)))
  } else {
    DTW_DISPATCH_DMAX(dm, (leaf_kernel<double, D_><<<grid, kLeafThreads, lds_bytes, st>>>(
                              static_cast<const double*>(w.X), static_cast<const double*>(w.Y), w, lds_leaf_bytes,
                              Xo, Yo, in_f64, w.d)))
  }
  return hipGetLastError();
}

hipError_t set_leaf_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
#define DTW_SET_ATTR(T_, D_)                                                                        \
  {                                                                                                 \
    hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void*>(&leaf_kernel<T_, D_>),         \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);     \
    if (r != hipSuccess) e = r;                                                                     \
  }
  DTW_SET_ATTR(double, 4) DTW_SET_ATTR(double, 8) DTW_SET_ATTR(double, 12) DTW_SET_ATTR(double, 16)
  DTW_SET_ATTR(double, 24) DTW_SET_ATTR(double, 32) DTW_SET_ATTR(float, 4) DTW_SET_ATTR(float, 8)
  DTW_SET_ATTR(float, 12) DTW_SET_ATTR(float, 16) DTW_SET_ATTR(float, 24) DTW_SET_ATTR(float, 32)
#undef DTW_SET_ATTR
  return e;
}

}  // namespace dtw
