// Device helpers shared by the wave kernels (dtw_wave.hip) and the
// orchestration kernels (dtw_plan.hip).
#pragma once

#include "dtw_internal.h"

#pragma clang fp contract(off)

namespace dtw {

// Number of cells (a,b) of an Mb x Nb block with a + b <= k.
__device__ __forceinline__ int64_t cells_upto(int64_t Mb, int64_t Nb, int64_t k) {
  const int64_t A = min(Mb - 1, k);
  if (A < 0) return 0;
  const int64_t t = k - (Nb - 1);
  const int64_t nfull = max((int64_t)0, min(A, t) + 1);
  int64_t cells = nfull * Nb;
  const int64_t lo = nfull, hi = A;
  if (hi >= lo) cells += (hi - lo + 1) * (2 * k - lo - hi + 2) / 2;
  return cells;
}

__device__ __forceinline__ void set_error(Ctl* ctl, int32_t code) { atomicCAS(&ctl->error, 0, code); }

// A work count read from the control block, clamped to the capacity the host
// planned for it: every device loop takes its trip count from such a value,
// so no corrupted count can make a kernel run away.
__device__ __forceinline__ int clamp_count(Ctl* ctl, int32_t v, int64_t cap) {
  if (v < 0 || v > cap) {
    set_error(ctl, kErrBadCount);
    return v < 0 ? 0 : (int)cap;
  }
  return v;
}

// Error-free transformation a + b = s + e (Knuth's TwoSum).
__device__ __forceinline__ double2 two_sum_acc(double2 acc, double v) {
  const double s = acc.x + v;
  const double bp = s - acc.x;
  const double e = (acc.x - (s - bp)) + (v - bp);
  return make_double2(s, acc.y + e);
}
__device__ __forceinline__ double2 dd_add(double2 a, double2 b) {
  double2 r = two_sum_acc(a, b.x);
  r.y += b.y;
  return r;
}

// ----------------------------------------------------------------- block scan

// Exclusive prefix sum over the workgroup in thread order; *total = the sum.
// Inclusive scan inside each wave by lane shuffles, wave totals through
// tmp[0 .. waves-1], two workgroup barriers. Every thread of the workgroup
// must call it; tmp may be reused as soon as it returns.
__device__ int64_t block_excl_scan(int64_t v, int64_t* tmp, int64_t* total) {
  const int t = threadIdx.x, n = blockDim.x;
  const int lane = t & (kWave - 1), wv = t / kWave, nw = (n + kWave - 1) / kWave;
  int64_t x = v;
  for (int off = 1; off < kWave; off <<= 1) {
    const int64_t u = __shfl(x, lane >= off ? lane - off : lane);
    if (lane >= off) x += u;
  }
  if (lane == kWave - 1 || t == n - 1) tmp[wv] = x;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int k = 0; k < nw; ++k) {
    const int64_t s = tmp[k];
    if (k < wv) before += s;
    all += s;
  }
  *total = all;
  __syncthreads();
  return before + x - v;
}

}  // namespace dtw
