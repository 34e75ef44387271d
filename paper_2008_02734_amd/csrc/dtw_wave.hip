// HIP wave kernels for gfx950: the anti-diagonal wavefront sweep (DiagDTW,
// Algorithm 1 of arXiv 2008.02734) and the leaf solve (textbook DTW with
// backpointers and backtrace, Sec. 2.1).  One wavefront owns 64 DP rows; the
// wave-level primitives (DPP lane shift, readfirstlane, scalar frame loads)
// live only in this file.
#include "dtw_common.h"
#include "dtw_gram.h"

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

// One unpredicated recurrence step, min(min(diag, left), up) + c, as a single
// assembly group: v_min keeps its IEEE-mode NaN rule (the other operand), and
// the compiler pads around one inline-assembly statement instead of three.
__device__ __forceinline__ double step_t(double diag, double left, double up, double c) {
  double r;
  asm volatile("v_min_f64 %0, %1, %2\n\tv_min_f64 %0, %0, %3\n\tv_add_f64 %0, %0, %4"
               : "=&v"(r) : "v"(diag), "v"(left), "v"(up), "v"(c));
  return r;
}
__device__ __forceinline__ float step_t(float diag, float left, float up, float c) {
  float r;
  asm volatile("v_min_f32 %0, %1, %2\n\tv_min_f32 %0, %0, %3\n\tv_add_f32 %0, %0, %4"
               : "=&v"(r) : "v"(diag), "v"(left), "v"(up), "v"(c));
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

// One dimension of a frame cost, and its final form.  Euclidean cost
// (Sec. 4.1): s = fma(e, e, s) with e = x_t - y_t, then the square root.
// Cosine cost (frames normalised at staging): s = fma(x_t, y_t, s), then
// 1 - s, raised to 0 where rounding takes it below.
template <bool kCos, typename T>
__device__ __forceinline__ T cost_acc(T x, T y, T s) {
  if constexpr (kCos) {
    return fma_t(x, y, s);
  } else {
    const T e = x - y;
    return fma_t(e, e, s);
  }
}
template <bool kCos, typename T>
__device__ __forceinline__ T cost_fin(T s) {
  if constexpr (kCos) {
    const T c = T(1) - s;
    return c < T(0) ? T(0) : c;
  } else {
    return sqrt_t(s);
  }
}

// Euclidean frame cost (Sec. 4.1): sum over t of fma(e, e, s), e = x_t - y_t,
// in dimension order, then the square root (the cosine form likewise with
// cost_acc / cost_fin).  Frames are zero-padded to D
// dimensions; a padded dimension contributes fma(0, 0, s) = s exactly.  x is
// the lane's own frame in registers; y0 and y1 are wave-uniform frames (the
// leaf reads them with scalar loads).  Two Y frames at once give two
// independent fma chains.
template <typename T, int D, bool kCos = false>
__device__ __forceinline__ void frame_cost2(const T (&x)[D], const T* __restrict__ y0, const T* __restrict__ y1,
                                            T& c0, T& c1) {
  T s0 = T(0), s1 = T(0);
#pragma unroll
  for (int k = 0; k < D; ++k) {
    s0 = cost_acc<kCos>(x[k], y0[k], s0);
    s1 = cost_acc<kCos>(x[k], y1[k], s1);
  }
  c0 = cost_fin<kCos>(s0);
  c1 = cost_fin<kCos>(s1);
}

// The same two costs with the Y frames in LDS (broadcast reads), KC
// dimensions at a time: the scheduling barrier keeps the compiler from
// hoisting every read ahead of the arithmetic, which would hold 2D values in
// registers; the other producer waves on the SIMD cover the read latency.
template <typename T, int D, bool kCos = false>
__device__ __forceinline__ void frame_cost2_lds(const T (&x)[D], const T* __restrict__ y0, const T* __restrict__ y1,
                                                T& c0, T& c1) {
  constexpr int KC = (sizeof(T) == 8 && D >= 24) ? 2 : 4;
  static_assert(D % KC == 0, "narrow frame widths are multiples of 4");
  T s0 = T(0), s1 = T(0);
#pragma unroll
  for (int k0 = 0; k0 < D; k0 += KC) {
    T a[KC], b[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      a[q] = y0[k0 + q];
      b[q] = y1[k0 + q];
    }
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      s0 = cost_acc<kCos>(x[k0 + q], a[q], s0);
      s1 = cost_acc<kCos>(x[k0 + q], b[q], s1);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  c0 = cost_fin<kCos>(s0);
  c1 = cost_fin<kCos>(s1);
}

// Frame widths of 64 and more: the lane's frame xl is read in chunks of 16
// dimensions (from LDS in the sweep, where the stripe's frames are staged, or
// from HBM in the leaf) and each chunk serves four wave-uniform Y frames, so
// register use stays bounded and every cost keeps the dimension order of
// frame_cost2.  kUnroll chunks are unrolled (the leaf, with more live state,
// takes 1 to stay within its registers).
template <typename T, int D, int kUnroll, bool kCos = false>
__device__ __forceinline__ void frame_cost4_wide(const T* __restrict__ xl, const T* __restrict__ y0,
                                                 const T* __restrict__ y1, const T* __restrict__ y2,
                                                 const T* __restrict__ y3, T (&c)[4]) {
  constexpr int KC = 16;
  static_assert(D % KC == 0, "wide frame widths are multiples of 16");
  T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll kUnroll
  for (int kc = 0; kc < D; kc += KC) {
    T xc[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) xc[q] = xl[kc + q];
#pragma unroll
    for (int q = 0; q < KC; ++q) {
      s0 = cost_acc<kCos>(xc[q], y0[kc + q], s0);
      s1 = cost_acc<kCos>(xc[q], y1[kc + q], s1);
      s2 = cost_acc<kCos>(xc[q], y2[kc + q], s2);
      s3 = cost_acc<kCos>(xc[q], y3[kc + q], s3);
    }
  }
  c[0] = cost_fin<kCos>(s0);
  c[1] = cost_fin<kCos>(s1);
  c[2] = cost_fin<kCos>(s2);
  c[3] = cost_fin<kCos>(s3);
}

// ----------------------------------------------------------------- pass kernel
//
// One workgroup owns a stripe of 64 consecutive local rows of one sweep and
// splits the work of Algorithm 1 over three roles:
//   wave 0      the recurrence.  Lane r is row a = a0 + r; at step t it
//               evaluates column b = t - r, so every lane of step t lies on
//               the diagonal k = a0 + t and the wave advances one diagonal
//               per step.  UP comes from lane r-1 through a DPP lane shift
//               (lane 0: the bottom row of the stripe above), DIAG is the
//               previous step's UP and LEFT the lane's own previous value.
//   producers   waves 1..pass_producers(CM): frame costs (Sec. 4.1) of whole
//               columns, one phase ahead of the recurrence, into an LDS ring
//               (Euclidean forms: eight waves, Y frames staged in LDS or read
//               wave-uniformly, X frames in registers or LDS; Gram form: two
//               waves with matrix-core tiles).
//   last wave   boundary input: the bottom row of the stripe above, read from
//               HBM one phase ahead into LDS.
// Phases of kPhase steps are separated by workgroup barriers.  The
// recurrence also writes its value of step t into slot t of the cost ring
// once it has read that slot's cost; the bottom row is published from there.
//
// Cost ring: lane r's cost for column j sits in slot (j + r) mod kCostRing,
// so the recurrence reads slot t at step t (one address per step for the
// whole wave).  At phase k the recurrence reads slots [32k, 32k+31] and the
// producers write columns [32k+32, 32k+63], i.e. slots [32k+32, 32k+126]:
// the two ranges never meet modulo 128.
//
// Bottom row hand-off between stripes: a per-sweep HBM ring of kRing rows of
// cells.  A cell carries one value and the id of the stripe that wrote it,
// ring_tag(level, s), in 8-byte words that are each stored and loaded as one
// relaxed device-scope atomic: a 32-bit half of the value and the id (FP32:
// one word, FP64: two).  Stripe s publishes its bottom row (lane 63's
// values, column c at step c + 63) into row s % kRing every kPubGroup
// steps; the input wave of stripe s+1 polls each word it needs until it
// carries stripe s's id, one phase ahead, into the LDS row `bring`.  No cell
// is ever reset and no fence is needed:
//  - an id is never reused within a call (the ring is cleared to id 0 when
//    the call starts), so an earlier writer's value or a half-written FP64
//    value (one word old, one new) never passes for the expected one;
//  - stripe s + kRing overwrites column c of the row only after computing
//    its own column c, which needs column c of stripe s + kRing - 1, ...,
//    which stripe s+1 computed after its input wave's load of column c from
//    the row had returned: no value is overwritten before it was read.
// Stripes are dequeued stripe-major across all sweeps of the level, so a
// stripe only waits on a stripe that a running workgroup dequeued before it:
// the persistent grid cannot deadlock.

// Words of a ring cell: one per 32-bit half of the value.
template <typename T>
constexpr int kCellWords = (int)sizeof(T) / 4;

// Id of stripe s of a level's sweep in the ring cells it writes: nonzero and
// unique within a call (levels and stripes are below 2^8 and 2^24).
__device__ __forceinline__ uint32_t ring_tag(int level, int s) {
  return ((uint32_t)(level + 1) << 24) | (uint32_t)(s + 1);
}

// A wave-uniform integer moved into a vector register: LDS addresses built
// from it keep their per-step parts as immediate offsets.
__device__ __forceinline__ int in_vgpr(int x) {
  int r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
  return r;
}


// Workgroup barrier that waits for this wave's LDS traffic only: global
// stores in flight (boundary values, band cells) are not waited for.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
// Wait until every global load and store of this wave has completed.
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// The call's device error word, read past the caches: once any wave has
// recorded an error, every wait of the call gives up.
__device__ __forceinline__ bool call_failed(const Work& w) {
  return __hip_atomic_load(&w.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Poll one ring word until it carries the id `tag`.  The wait is bounded by
// the device wall clock (w.spin_ticks) and an iteration cap; on expiry the
// lane records an error and returns what it read last.  A wait also ends as
// soon as the call's error word is set, so the first expiry (or any other
// device error) ends every wait of the call: a broken hand-off costs one
// wait limit, not one per column.
__device__ __forceinline__ uint64_t poll_word(const uint64_t* p, uint32_t tag, const Work& w) {
  uint64_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((uint32_t)(v >> 32) != tag) {
    const uint64_t t0 = wall_clock64();
    for (uint32_t it = 0;; ++it) {
      __builtin_amdgcn_s_sleep(1);
      // the cell and the error word are loaded together: one memory round
      // trip per poll
      const int32_t err = __hip_atomic_load(&w.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((uint32_t)(v >> 32) == tag || err != 0) break;
      if (wall_clock64() - t0 > w.spin_ticks || it > kSpinIterCap) {
        set_error(w.ctl, kErrSpinTimeout);
        break;
      }
    }
  }
  return v;
}

// Publish lane 63's values of the steps g0..t (g0 = t rounded down to a
// multiple of kPubGroup), i.e. the columns g0 + u - 63 of the stripe's
// bottom row that the next stripe needs (col <= pub_max), with the stripe's
// id: lane 64 - kPubGroup * kW + i stores word i % kW of step
// g0 + i / kW.  The values are read from the cost ring: after the recurrence
// has read the cost of step s from slot s it writes its value of step s into
// that slot, which the producers do not write again before the phase's
// closing barrier.
template <typename T>
__device__ __forceinline__ void publish(int t, int lane, const T* cring, uint64_t* ring_out, uint32_t tag,
                                        int pub_max) {
  constexpr int kW = kCellWords<T>;
  const int i = lane - (kWave - kPubGroup * kW);
  const int st = (t & ~(kPubGroup - 1)) + (i >= 0 ? i / kW : 0);
  const int col = st - (kWave - 1);
  if (i >= 0 && st <= t && col >= 0 && col <= pub_max) {
    const uint32_t half =
        reinterpret_cast<const uint32_t*>(cring + (st & (kCostRing - 1)) * kWave + (kWave - 1))[i % kW];
    __hip_atomic_store(ring_out + (int64_t)col * kW + i % kW, ((uint64_t)tag << 32) | half, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ----------------------------------------------------------------- tie-exact sweep
//
// Tie-exact mode (FP64; not in the paper, whose split ties are broken
// arbitrarily): one forward sweep over the whole block, from its origin's
// value in the whole problem's table (PassDesc.f0), with a label per cell: on
// local diagonals kf-1 and kf the cell itself (2a + [on kf]), past them the
// label of the predecessor the DIAG > UP > LEFT backpointer names.  The
// block's last cell writes its label as the split (piv_pos, in the band-row
// form q = 1 + [on kf], row a) and its value (piv_key); diagonals kf-1 and
// kf go to the band, where the planner reads the pivot's value.  Labels
// travel between stripes through a second ring, `lring`, one word per cell
// (the label and the writer's id), published beside the values.

__device__ __forceinline__ int wave_shr1_i(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, kDppWaveShr1, 0xf, 0xf, false);
}

// Lane 63's labels of the steps g0..t, as publish<T> does for its values:
// lane 16 + i stores the label of step g0 + i from labh.
__device__ __forceinline__ void publish_labels(int t, int lane, const int* labh, uint64_t* lring_out, uint32_t tag,
                                               int pub_max) {
  const int i = lane - kPubGroup;
  const int st = (t & ~(kPubGroup - 1)) + i;
  const int col = st - (kWave - 1);
  if (i >= 0 && i < kPubGroup && st <= t && col >= 0 && col <= pub_max)
    __hip_atomic_store(lring_out + col, ((uint64_t)tag << 32) | (uint32_t)labh[st & (kCostRing - 1)],
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Poll a value word and (want_b) a label word together until both carry
// `tag`; bounded like poll_word.
__device__ __forceinline__ void poll_pair(const uint64_t* pa, const uint64_t* pb, bool want_b, uint32_t tag,
                                          const Work& w, uint64_t& va, uint64_t& vb) {
  va = __hip_atomic_load(pa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  vb = want_b ? __hip_atomic_load(pb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : ((uint64_t)tag << 32);
  if ((uint32_t)(va >> 32) == tag && (uint32_t)(vb >> 32) == tag) return;
  const uint64_t t0 = wall_clock64();
  for (uint32_t it = 0;; ++it) {
    __builtin_amdgcn_s_sleep(1);
    const int32_t err = __hip_atomic_load(&w.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    va = __hip_atomic_load(pa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (want_b) vb = __hip_atomic_load(pb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (((uint32_t)(va >> 32) == tag && (uint32_t)(vb >> 32) == tag) || err != 0) return;
    if (wall_clock64() - t0 > w.spin_ticks || it > kSpinIterCap) {
      set_error(w.ctl, kErrSpinTimeout);
      return;
    }
  }
}

// The recurrence wave of a tie-exact stripe: one step at a time, the value
// unpredicated as in the fast path (cells before a lane's row hold +inf or
// NaN, which v_min passes over) and the label chosen by equality with the
// minimum (a NaN or +inf operand never equals the finite minimum of a cell).
template <typename T>
__device__ void tie_recurrence(const PassDesc& P, const Work& w, int p, int s, int a0, int Lr, int n_steps,
                               int n_phases, bool has_succ, int pub_max, T* cring, const T* bring, const int* blab,
                               int* labh, uint64_t* ring_out, uint64_t* lring_out, uint32_t tag_out, int lane) {
  const T INF = inf_t<T>();
  const int a = a0 + lane;
  const int bmax = (lane <= Lr) ? min(P.Nb - 1, P.kstop - a) : -1;
  const int kf = P.kf;
  T f = INF;                                        // own F(a, b-1)
  T up_prev = (s == 0 && lane == 0) ? T(0) : INF;   // F(a-1, b-1): 0 before the origin
  int lab = 0, lab_up_prev = 0;
  lds_barrier();  // phase -1: first costs and boundary chunk
  // the origin holds its value in the whole table: the cost slot of lane 0,
  // step 0 takes it, so that F(origin) = 0 + f0 exactly
  if (s == 0 && lane == 0 && P.f0 == P.f0) cring[0] = (T)P.f0;
  // the step of the block's last cell (in the last stripe only)
  const int t_end = (a0 + kWave >= P.Mb) ? (P.Mb - 1 - a0) + (P.Nb - 1) : -1;
  for (int k = 0; k < n_phases; ++k) {
    const int t0 = k * kPhase;
    const int t1 = min(t0 + kPhase, n_steps);
    // a phase that holds neither the label diagonals nor the last cell runs
    // as the fast path does: operands loaded one group of steps ahead, lane
    // 63's labels kept in registers and written out once per group
    const bool plain = t1 == t0 + kPhase && !(a0 + t0 <= kf && a0 + t1 - 1 >= kf - 1) &&
                       !(t_end >= t0 && t_end < t1);
    if (plain) {
      T* const hp = cring + (t0 & (kCostRing - 1)) * kWave + lane;
      const T* bp = bring + in_vgpr(t0 & (2 * kPhase - 1));
      const int* lp = blab + (t0 & (2 * kPhase - 1));
      constexpr int G = kStepGroup;
      T cb[2][G], bb[2][G];
      int lb[2][G];
      int labw[G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        cb[0][i] = hp[i * kWave];
        bb[0][i] = bp[i];
        lb[0][i] = lp[i];
      }
#pragma unroll
      for (int g = 0; g < kPhase / G; ++g) {
        if (g + 1 < kPhase / G) {
#pragma unroll
          for (int i = 0; i < G; ++i) {
            cb[(g + 1) & 1][i] = hp[((g + 1) * G + i) * kWave];
            bb[(g + 1) & 1][i] = bp[(g + 1) * G + i];
            lb[(g + 1) & 1][i] = lp[(g + 1) * G + i];
          }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
          const int u = g * G + i;
          const T up = wave_shr1(bb[g & 1][i], f);
          const int lu = wave_shr1_i(lb[g & 1][i], lab);
          const T m = min_t(min_t(up_prev, f), up);
          lab = (up_prev == m) ? lab_up_prev : ((up == m) ? lu : lab);  // DIAG, then UP, then LEFT
          f = m + cb[g & 1][i];
          up_prev = up;
          lab_up_prev = lu;
          hp[u * kWave] = f;  // the history, in the slot whose cost was read a group ago
          labw[i] = lab;
          if (i == G - 1 && lane == kWave - 1) {
            static_assert(G == 4, "one 16-byte label store per group");
            *reinterpret_cast<int4*>(labh + ((t0 + u - (G - 1)) & (kCostRing - 1))) =
                make_int4(labw[0], labw[1], labw[2], labw[3]);
          }
          if ((u & (kPubGroup - 1)) == kPubGroup - 1) {
            __builtin_amdgcn_wave_barrier();  // lane 63's values and labels read by the publishing lanes
            if (has_succ) {
              publish<T>(t0 + u, lane, cring, ring_out, tag_out, pub_max);
              publish_labels(t0 + u, lane, labh, lring_out, tag_out, pub_max);
            }
          }
        }
      }
      lds_barrier();
      continue;
    }
    for (int t = t0; t < t1; ++t) {
      T* const hp = cring + (t & (kCostRing - 1)) * kWave + lane;
      const T c = *hp;
      const T up = wave_shr1(bring[t & (2 * kPhase - 1)], f);
      const int lu = wave_shr1_i(blab[t & (2 * kPhase - 1)], lab);
      const T m = min_t(min_t(up_prev, f), up);
      lab = (up_prev == m) ? lab_up_prev : ((up == m) ? lu : lab);  // DIAG, then UP, then LEFT
      f = m + c;
      up_prev = up;
      lab_up_prev = lu;
      const int b = t - lane;
      const int kd = a0 + t;  // local diagonal of every lane's cell at this step
      if (kd == kf - 1 || kd == kf) {
        lab = 2 * a + (kd == kf ? 1 : 0);
        if (b >= 0 && b <= bmax) {
          const int lo = max(0, kd - (P.Nb - 1));
          w.bandF[P.band_off + (int64_t)(kd - (kf - 2)) * P.L + (a - lo)] = (double)f;
        }
      }
      if (a == P.Mb - 1 && b == P.Nb - 1) {  // the block's last cell
        w.piv_pos[p >> 1] = ((uint64_t)(1 + (lab & 1)) << 32) | (uint32_t)(lab >> 1);
        w.piv_key[p >> 1] = (uint64_t)__double_as_longlong((double)f);
      }
      *hp = f;  // the history: this step's value in the slot whose cost was just read
      if (lane == kWave - 1) labh[t & (kCostRing - 1)] = lab;
      if ((t & (kPubGroup - 1)) == kPubGroup - 1 || t == n_steps - 1) {
        __builtin_amdgcn_wave_barrier();  // lane 63's value and label read by the publishing lanes
        if (has_succ) {
          publish<T>(t, lane, cring, ring_out, tag_out, pub_max);
          publish_labels(t, lane, labh, lring_out, tag_out, pub_max);
        }
      }
    }
    lds_barrier();
  }
}

// Gram-form producer (dtw_gram.h), BF16 frames for kBf16, else FP16.  The
// X operand is either held in registers (kXRegs: each lane's slices of its
// row's frame) or staged in LDS at the start of a stripe by the NPW producer
// waves (rows padded by 16 bytes so the operand reads of 16 lanes fall in
// distinct banks), behind one barrier that the other waves of the group
// match with stage_barrier.  The 64 x 32 cost block of a phase is two 32x32
// tiles (stripe rows 0..31 and 32..63); of the NPW producer waves, wave w
// owns tile (w-1) & 1 of every (NPW/2)-th phase, (w-1) >> 1 being its phase
// residue.  It issues the loads of its next block's Y frames right after
// writing its current block, so they have the NPW/2 - 1 phases in between
// plus the rest of the current one to arrive, and at its phase it runs
// DP/16 matrix-core operations and the FP32 epilogue
// sqrt(max(0, |x|^2 + |y|^2 - 2 x.y)) into the cost ring (kCos: the frames
// were normalised before rounding and the epilogue is max(0, 1 - x.y), the
// cosine cost of Sec. 4.1).  The tile is formed
// transposed (Y frames as the first operand): each lane's results then share
// one stripe row, and the 32 lanes of a half-wave write 32 distinct rows of
// the ring at once.  Row r of the stripe is frame gi0 + gis*(a0 + r) of Xb,
// column j is frame gj0 + gjs*j of Yb; rows past Lr reuse row Lr and columns
// past need_max reuse column need_max.
template <int DP, bool kBf16, bool kCos, int NPW, bool kXRegs>
__device__ __forceinline__ void gram_producer(const uint16_t* __restrict__ Xb, const uint16_t* __restrict__ Yb,
                                              const float* __restrict__ Xn, const float* __restrict__ Yn, int gi0,
                                              int gis, int gj0, int gjs, int a0, int Lr, int need_max, int n_phases,
                                              int wave, int lane, float* cring) {
  constexpr int KB = DP / 16;
  constexpr int XS = DP + 8;  // LDS row stride of the staged frames, in bf16
  static_assert(NPW % 2 == 0, "producer waves come in tile pairs");
  constexpr int kRot = NPW / 2;                // a wave writes every kRot-th phase
  __shared__ float ny_stage[NPW][32];          // |y|^2 of a block's columns, per producer wave
  const int pw = wave - 1;
  const int tile = pw & 1, res = pw >> 1;
  const int half = lane >> 5, l32 = lane & 31;
  const int row = tile * 32 + l32;  // stripe row of all of this lane's results
  const int gi = gi0 + gis * (a0 + min(row, Lr));
  const float nx = Xn[gi];
  // the X operand: this lane's slices of its row's frame, in registers, or
  // the stripe's frames staged in LDS by all producer waves
  bf16x8_t Xo[kXRegs ? KB : 1];
  const uint16_t* xrow = nullptr;
  if constexpr (kXRegs) {
    const uint16_t* xr = Xb + (int64_t)gi * DP + 8 * half;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) Xo[kb] = load_bf16x8(xr + 16 * kb);
  } else {
    __shared__ __align__(16) uint16_t xs[kWave * XS];
    for (int idx = pw * kWave + lane; idx < kWave * (DP / 8); idx += NPW * kWave) {
      const int r = idx / (DP / 8), c = idx % (DP / 8);
      const uint4 v = *reinterpret_cast<const uint4*>(Xb + (int64_t)(gi0 + gis * (a0 + min(r, Lr))) * DP + 8 * c);
      *reinterpret_cast<uint4*>(xs + r * XS + 8 * c) = v;
    }
    xrow = xs + row * XS + 8 * half;
  }
  bf16x8_t Yo[KB];
  float ny_own = 0.0f;
  auto issue = [&](int kw) {  // loads of the block written at iteration kw
    const int c0 = (kw + 1) * kPhase;
    if (c0 <= need_max) {
      const int gj = gj0 + gjs * min(c0 + l32, need_max);
      const uint16_t* yr = Yb + (int64_t)gj * DP + 8 * half;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) Yo[kb] = load_bf16x8(yr + 16 * kb);
      ny_own = Yn[gj];
    }
  };
  int kw = res - 1;
  issue(kw);
  if constexpr (!kXRegs) lds_barrier();  // the staged frames are visible (matched by stage_barrier)
  for (int k = -1; k < n_phases; ++k) {
    if (k == kw) {
      const int c0 = (k + 1) * kPhase;
      if (c0 <= need_max) {
        f32x16_t acc = f32x16_zero();
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          if constexpr (kXRegs) acc = mfma_16bit_32x32x16<kBf16>(Yo[kb], Xo[kb], acc);
          else acc = mfma_16bit_32x32x16<kBf16>(Yo[kb], load_bf16x8(xrow + 16 * kb), acc);
        }
        // register q of this lane holds column 8*(q/4) + 4*half + q%4 of the block
        float* nys = ny_stage[pw];
        if (half == 0) nys[l32] = ny_own;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int jj = 8 * (q / 4) + 4 * half + q % 4;
          float c;
          if constexpr (kCos) {
            c = fmaxf(1.0f - acc[q], 0.0f);
          } else {
            const float v = fmaxf(__builtin_fmaf(-2.0f, acc[q], nx + nys[jj]), 0.0f);
            c = __builtin_amdgcn_sqrtf(v);
          }
          cring[((c0 + jj + row) & (kCostRing - 1)) * kWave + row] = c;
        }
        __builtin_amdgcn_wave_barrier();
      }
      kw += kRot;
      issue(kw);
    }
    lds_barrier();
  }
}

// The barrier that the recurrence and input waves take to match the producer
// waves' staging of the stripe's frames in LDS: the Gram form (sweep and
// leaf) and the sweep's Euclidean form at frame widths of 64 and more.
template <bool kStaged>
__device__ __forceinline__ void stage_barrier() {
  if constexpr (kStaged) lds_barrier();
}
template <int CM>
__device__ __forceinline__ void gram_stage_barrier() {
  stage_barrier<is_gram(CM)>();
}
// Euclidean sweeps at frame widths up to 32 stage the Y frames of each phase
// in LDS, one phase ahead, with vector loads: scalar loads would wait on L2
// once per frame chunk, which is slow when the workgroups of a batch read
// frames of many different pairs.
template <typename T, int CM, int D>
constexpr bool kStageY = !is_gram(CM) && (D <= 32);
template <typename T, int CM, int D>
constexpr bool kPassStagesRows = (!is_gram(CM) && D >= 64) || kStageY<T, CM, D>;

template <typename T, int D, int CM, bool kTie = false>
__global__ __launch_bounds__(pass_threads(CM), (is_gram(CM) ? 4 : kTie ? 2 : (D >= 32 && sizeof(T) == 8) ? 3 : D == 32 ? 4 : 5)) void pass_kernel(const T* __restrict__ X, const T* __restrict__ Y, Work w,
                                                            int level) {
  __shared__ T cring[kCostRing * kWave];  // frame costs, [slot][lane]
  __shared__ T bring[2 * kPhase];         // bottom row of the stripe above, [column & 63]
  __shared__ int sh_ticket;
  constexpr bool kTieOk = kTie && sizeof(T) == 8 && !is_gram(CM);  // tie-exact mode: FP64 sweeps only
  __shared__ int blab[kTieOk ? 2 * kPhase : 1];  // labels of the bottom row above (tie-exact mode)
  __shared__ __align__(16) int labh[kTieOk ? kCostRing : 1];  // lane 63's labels by step (tie-exact mode)
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = (int)(threadIdx.x % kWave);
  // the recurrence wave issues first on its SIMD: its dependency chain sets the pace
  if (wave == 0) __builtin_amdgcn_s_setprio(3);
  Ctl* ctl = w.ctl;
  const int n_tickets = clamp_count(ctl, ctl->n_tickets, w.caps.ticket);
  const int n_pass = clamp_count(ctl, ctl->n_pass, 2 * w.caps.sub);
  const T INF = inf_t<T>();

  for (int iter = 0; iter <= n_tickets; ++iter) {  // each iteration consumes one ticket
    // after a device error no further stripe is started (the others end
    // their waits at once), so a failed call drains quickly
    if (threadIdx.x == 0) sh_ticket = call_failed(w) ? -1 : atomicAdd(&ctl->ticket, 1);
    lds_barrier();
    const int tk = __builtin_amdgcn_readfirstlane(sh_ticket);
    lds_barrier();
    if (tk >= n_tickets || tk < 0) break;
    const int2 tv = w.tickets[tk];
    const int p = __builtin_amdgcn_readfirstlane(tv.x);
    const int s = __builtin_amdgcn_readfirstlane(tv.y);
    if (p < 0 || p >= n_pass) {
      if (threadIdx.x == 0) set_error(ctl, kErrBadPass);
      continue;
    }
    const PassDesc P = w.passes[p];
    if (P.Mb != P.i1 - P.i0 + 1 || P.Nb != P.j1 - P.j0 + 1 || P.Mb < 1 || P.Nb < 1 || P.kstop < 0 ||
        P.kstop > P.Mb + P.Nb - 2 || P.n_rows != min(P.Mb - 1, P.kstop) + 1 || s < 0 || s >= P.n_stripes ||
        P.n_stripes != (P.n_rows + kWave - 1) / kWave) {
      if (threadIdx.x == 0) set_error(ctl, kErrBadPass);
      continue;
    }

    const int a0 = s * kWave;
    const int Lr = min(kWave - 1, P.n_rows - 1 - a0);           // last lane with a row
    const int need_max = min(P.Nb - 1, P.kstop - a0);           // last column of lane 0
    const int n_steps = min(P.Nb - 1 + Lr, P.kstop - a0) + 1;
    const int n_phases = (n_steps + kPhase - 1) / kPhase;
    const bool has_pred = s > 0;
    const bool has_succ = s + 1 < P.n_stripes;
    const int pub_max = has_succ ? min(P.Nb - 1, P.kstop - a0 - kWave) : -1;  // = need_max of stripe s+1
    constexpr int kCW = kCellWords<T>;
    uint64_t* ring = w.ring + P.ring_off * kCW;
    uint64_t* ring_out = ring + (int64_t)(s % kRing) * P.Nb * kCW;
    const uint64_t* ring_in = ring + (int64_t)((s + kRing - 1) % kRing) * P.Nb * kCW;
    const uint32_t tag_out = ring_tag(level, s), tag_in = ring_tag(level, s - 1);
    constexpr bool tie = kTieOk;
    if ((P.tie != 0) != kTieOk) {
      if (threadIdx.x == 0) set_error(ctl, kErrBadPass);
      continue;
    }

    if (wave == 0 && tie) {
      if constexpr (kTieOk) {
        stage_barrier<kPassStagesRows<T, CM, D>>();
        uint64_t* lring = w.lring + P.ring_off;
        tie_recurrence<T>(P, w, p, s, a0, Lr, n_steps, n_phases, has_succ, pub_max, cring, bring, blab, labh,
                          ring_out, lring + (int64_t)(s % kRing) * P.Nb, tag_out, lane);
      }
    } else if (wave == 0) {
      // ------------------------------------------------ recurrence
      //
      // Before a lane reaches its row (b < 0) its value is +inf (or a NaN
      // made from an unused cost slot); v_min returns the other operand of a
      // NaN, so at b = 0 the minimum is exactly UP, and the unpredicated step
      // is the recurrence of Algorithm 1 from the first step on.  Lane 0 of
      // the block's first stripe starts with DIAG = 0, which makes its first
      // cell F(0,0) = C(0,0) exactly.  Lanes past their row's last column
      // keep computing values that no valid cell reads.  Only the steps that
      // reach the band diagonals (the last three) take the predicated path.
      const int a = a0 + lane;
      const int bmax = (lane <= Lr) ? min(P.Nb - 1, P.kstop - a) : -1;
      const int K = P.Mb + P.Nb - 1;
      const int t_band = min(n_steps, max(0, P.kstop - a0 - 2));
      T f = INF;                                          // own F(a, b-1)
      T up_prev = (s == 0 && lane == 0) ? T(0) : INF;     // F(a-1, b-1)
      stage_barrier<kPassStagesRows<T, CM, D>>();
      lds_barrier();  // phase -1: first costs and boundary chunk
      for (int k = 0; k < n_phases; ++k) {
        const int t0 = k * kPhase;
        T* const hp = cring + (t0 & (kCostRing - 1)) * kWave + lane;  // the phase's slots, also the history
        const T* cp = hp;
        const T* bp = bring + in_vgpr(t0 & (2 * kPhase - 1));
        if (t0 + kPhase <= t_band) {
          // operands of the next kStepGroup steps are read one group ahead
          constexpr int G = kStepGroup;
          T cb[2][G], bb[2][G];
#pragma unroll
          for (int i = 0; i < G; ++i) {
            cb[0][i] = cp[i * kWave];
            bb[0][i] = bp[i];
          }
#pragma unroll
          for (int g = 0; g < kPhase / G; ++g) {
            if (g + 1 < kPhase / G) {
#pragma unroll
              for (int i = 0; i < G; ++i) {
                cb[(g + 1) & 1][i] = cp[((g + 1) * G + i) * kWave];
                bb[(g + 1) & 1][i] = bp[(g + 1) * G + i];
              }
            }
#pragma unroll
            for (int i = 0; i < G; ++i) {
              const int u = g * G + i;
              // the history takes the previous step's value, off this
              // step's dependency chain; a group's last value is written
              // and the group published at once, ahead of the barrier
              if ((u & (kPubGroup - 1)) != 0) hp[(u - 1) * kWave] = f;
              const T up = wave_shr1(bb[g & 1][i], f);
              f = step_t(up_prev, f, up, cb[g & 1][i]);
              up_prev = up;
              if ((u & (kPubGroup - 1)) == kPubGroup - 1) {
                hp[u * kWave] = f;
                __builtin_amdgcn_wave_barrier();  // lane 63's history read by the publishing lanes
                if (has_succ) publish<T>(t0 + u, lane, cring, ring_out, tag_out, pub_max);
              }
            }
          }
        } else {
          const int t1 = min(t0 + kPhase, n_steps);
          for (int t = t0; t < t1; ++t) {
            const int u = t - t0;
            const int b = t - lane;
            if ((t & (kPubGroup - 1)) != 0) hp[(u - 1) * kWave] = f;
            const T c = cp[u * kWave];
            const T up = wave_shr1(bp[u], f);
            if (t < t_band) {
              f = step_t(up_prev, f, up, c);
            } else if (b >= 0 && b <= bmax) {
              const T diag = (b == 0) ? INF : up_prev;
              const T left = (b == 0) ? INF : f;
              f = (a == 0 && b == 0) ? c : min_t(min_t(diag, left), up) + c;
              const int kd = a0 + t;  // = a + b >= kstop - 2
              if (P.dir == 0 || P.raw) {
                const int q = kd - (P.kstop - 2);
                const int lo = max(0, kd - (P.Nb - 1));
                const int64_t idx = P.band_off + (int64_t)q * P.L + (a - lo);
                w.bandF[idx] = (double)f;
                if (w.bandC) w.bandC[idx] = (double)c;
              } else {
                const int kfw = K - 1 - kd;
                const int q = kfw - (P.kf - 2);
                const int af = P.Mb - 1 - a;
                const int lo = max(0, kfw - (P.Nb - 1));
                w.bandB[P.band_off + (int64_t)q * P.L + (af - lo)] = (double)f;
              }
            }
            up_prev = up;
            if ((t & (kPubGroup - 1)) == kPubGroup - 1 || t == n_steps - 1) {
              hp[u * kWave] = f;
              __builtin_amdgcn_wave_barrier();  // lane 63's value read by the publishing lanes
              if (has_succ) publish<T>(t, lane, cring, ring_out, tag_out, pub_max);
            }
          }
        }
        lds_barrier();
      }
    } else if (wave <= pass_producers(CM) && is_gram(CM)) {
      // ------------------------------------------------ frame costs, Gram form (BF16 or FP16 frames)
      if constexpr (is_gram(CM))
        gram_producer<D, gram_bf16(CM), is_cos(CM), pass_producers(CM), true>(static_cast<const uint16_t*>(w.X), static_cast<const uint16_t*>(w.Y), w.Xn, w.Yn,
                         P.dir ? P.i1 : P.i0, P.dir ? -1 : 1, P.dir ? P.j1 : P.j0, P.dir ? -1 : 1, a0, Lr,
                         need_max, n_phases, wave, lane, reinterpret_cast<float*>(cring));
    } else if (wave <= pass_producers(CM) && D >= 64) {
      // ------------------------------------------------ frame costs, wide frames
      if constexpr (D >= 64 && !is_gram(CM)) {
        // the stripe's frames in LDS, rows padded by 16 bytes (bank spread of the chunk reads)
        constexpr int XS = D + 16 / (int)sizeof(T);
        constexpr int CPR = D * (int)sizeof(T) / 16;  // 16-byte chunks per frame
        __shared__ __align__(16) T xs[kWave * XS];
        const int pw = wave - 1;
        for (int idx = pw * kWave + lane; idx < kWave * CPR; idx += kProducers * kWave) {
          const int r = idx / CPR, c = idx % CPR;
          const int gi = P.dir ? P.i1 - (a0 + min(r, Lr)) : P.i0 + a0 + min(r, Lr);
          *reinterpret_cast<uint4*>(xs + r * XS + c * (16 / (int)sizeof(T))) =
              *reinterpret_cast<const uint4*>(X + (int64_t)gi * D + c * (16 / (int)sizeof(T)));
        }
        lds_barrier();  // staged frames visible (matched by stage_barrier in the other waves)
        const T* xl = xs + lane * XS;
        for (int k = -1; k < n_phases; ++k) {
          const int c0 = (k + 1) * kPhase;
          if (c0 <= need_max) {
            int gj[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int jc = min(c0 + pw + i * kProducers, need_max);
              gj[i] = __builtin_amdgcn_readfirstlane(P.dir ? P.j1 - jc : P.j0 + jc);
            }
            T cv[4];
            frame_cost4_wide<T, D, 2, is_cos(CM)>(xl, Y + (int64_t)gj[0] * D, Y + (int64_t)gj[1] * D, Y + (int64_t)gj[2] * D,
                                   Y + (int64_t)gj[3] * D, cv);
#pragma unroll
            for (int i = 0; i < 4; ++i)
              cring[((c0 + pw + i * kProducers + lane) & (kCostRing - 1)) * kWave + lane] = cv[i];
          }
          lds_barrier();
        }
      }
    } else if (wave <= pass_producers(CM) && kStageY<T, CM, D>) {
      // ------------------------------------------------ frame costs, Y frames staged in LDS
      if constexpr (kStageY<T, CM, D>) {
        const int pw = wave - 1;
        T x[D];
        {
          const int r = min(lane, Lr);  // lanes below the stripe's last row reuse it
          const int gi = P.dir ? P.i1 - (a0 + r) : P.i0 + a0 + r;
          const T* xr = X + (int64_t)gi * D;
#pragma unroll
          for (int q = 0; q < D; ++q) x[q] = xr[q];
        }
        // ys[p & 1] holds the frames of phase p's 32 columns (clamped at
        // need_max), written at iteration p - 2 from loads issued at p - 3
        constexpr int CPF = D * (int)sizeof(T) / 16;  // 16-byte chunks per frame
        static_assert(kPhase * CPF <= kProducers * kWave, "one chunk per producer lane");
        __shared__ __align__(16) T ys[2][kPhase * D];
        const int pl = pw * kWave + lane;
        uint4 pend = {0u, 0u, 0u, 0u};
        auto fetch = [&](int ph) {
          const int cb = ph * kPhase;
          if (pl < kPhase * CPF && cb <= need_max) {
            const int jc = min(cb + pl / CPF, need_max);
            const int gj = P.dir ? P.j1 - jc : P.j0 + jc;
            pend = *reinterpret_cast<const uint4*>(Y + (int64_t)gj * D + (pl % CPF) * (16 / (int)sizeof(T)));
          }
        };
        auto stash = [&](int ph) {
          if (pl < kPhase * CPF && ph * kPhase <= need_max)
            *reinterpret_cast<uint4*>(&ys[ph & 1][0] + pl * (16 / (int)sizeof(T))) = pend;
        };
        fetch(0);
        stash(0);
        fetch(1);
        lds_barrier();  // phase 0's frames visible (matched by stage_barrier in the other waves)
        for (int k = -1; k < n_phases; ++k) {
          const int c0 = (k + 1) * kPhase;
          if (c0 <= need_max) {
            const T* yb = &ys[(k + 1) & 1][0];
#pragma unroll
            for (int i = 0; i < kPhase / kProducers; i += 2) {
              const int jj0 = pw + i * kProducers, jj1 = jj0 + kProducers;
              T cv0, cv1;
              frame_cost2_lds<T, D, is_cos(CM)>(x, yb + jj0 * D, yb + jj1 * D, cv0, cv1);
              cring[((c0 + jj0 + lane) & (kCostRing - 1)) * kWave + lane] = cv0;
              cring[((c0 + jj1 + lane) & (kCostRing - 1)) * kWave + lane] = cv1;
            }
          }
          stash(k + 2);  // into the buffer of phase k, last read before the previous barrier
          fetch(k + 3);
          lds_barrier();
        }
      }
    } else {
      // ------------------------------------------------ boundary input
      stage_barrier<kPassStagesRows<T, CM, D>>();
      if (tie) {
        // tie-exact mode: the value words as below, and lanes 0..kPhase-1 the
        // label of column lane of the chunk, polled together
        const uint64_t* lring_in = w.lring + P.ring_off + (int64_t)((s + kRing - 1) % kRing) * P.Nb;
        for (int k = -1; k < n_phases; ++k) {
          const int col = (k + 1) * kPhase + lane / kCW;
          const int colL = (k + 1) * kPhase + lane;
          if (lane < kPhase * kCW) {
            uint32_t half = (kCW == 2) ? ((lane % 2) ? 0x7FF00000u : 0u) : 0x7F800000u;  // a half of +inf
            int lb = 0;
            if (has_pred && col <= need_max) {
              uint64_t va, vb;
              poll_pair(ring_in + (int64_t)col * kCW + lane % kCW, lring_in + colL,
                        lane < kPhase && colL <= need_max, tag_in, w, va, vb);
              half = (uint32_t)va;
              lb = (int)(uint32_t)vb;
            }
            reinterpret_cast<uint32_t*>(bring)[(col & (2 * kPhase - 1)) * kCW + lane % kCW] = half;
            if (lane < kPhase) blab[colL & (2 * kPhase - 1)] = lb;
          }
          lds_barrier();
        }
        continue;
      }
      // lanes 0..kPhase*kW-1: word lane % kW of column lane / kW of the chunk
      for (int k = -1; k < n_phases; ++k) {
        const int col = (k + 1) * kPhase + lane / kCW;
        if (lane < kPhase * kCW) {
          uint32_t half = (kCW == 2) ? ((lane % 2) ? 0x7FF00000u : 0u) : 0x7F800000u;  // a half of +inf
          if (has_pred && col <= need_max)
            half = (uint32_t)poll_word(ring_in + (int64_t)col * kCW + lane % kCW, tag_in, w);
          reinterpret_cast<uint32_t*>(bring)[(col & (2 * kPhase - 1)) * kCW + lane % kCW] = half;
        }
        lds_barrier();
      }
    }
  }
}

// ----------------------------------------------------------------- leaf

// Textbook DTW on one leaf block (Sec. 2.1) by one workgroup with the roles
// of the pass kernel: the shorter side is the row dimension, swept in
// ceil(R/64) stripes of 64 rows one after the other, the longer side the
// column dimension.  The recurrence wave also records a 2-bit backpointer per
// cell: 0 DIAG (i-1,j-1), 1 UP (i-1,j), 2 LEFT (i,j-1), chosen DIAG, then UP,
// then LEFT on ties; row 0 of X moves LEFT and column 0 of Y moves UP, so the
// codes recorded on row 0 and column 0 are never read.  When the block is
// transposed (rows = Y frames) UP and LEFT swap roles, and the codes keep
// their original meaning.
//
// Pointer layout, by step: lane r of stripe st records the codes of its
// steps 16m..16m+15 (columns 16m-r..16m+15-r) in word ((st*Wm + m)*64 + r),
// Wm = ceil((Cc+63)/16); all lanes store their word together every 16 steps.
// The bottom row of a stripe reaches the next stripe through `brow`, written
// from the recurrence values kept in the cost ring every 16 steps, and the input wave
// copies it into the boundary ring one phase ahead.  Lane 0 of the
// recurrence wave then walks the pointers back from the block's last cell.
// `bp` and `brow` point into LDS when the leaf fits there and into global
// scratch otherwise; the caller inlines one copy per case so that each copy
// addresses a single memory space.
struct LeafShape {
  bool tr;
  int R, Cc, r0, c0, Wm;
  double f0;  // tie-exact mode: value of the leaf's origin in the whole table (NaN: its own cost)
};

// Lane 48+u stores step g0+u's value of lane 63 (column g0+u-63 of the
// stripe's bottom row), g0 = t rounded down to a multiple of kPubGroup.
template <typename T>
__device__ __forceinline__ void leaf_publish(int t, int lane, const T* cring, T* brow, int Cc) {
  const int st = (t & ~(kPubGroup - 1)) + (lane - (kWave - kPubGroup));
  const int col = st - (kWave - 1);
  if (lane >= kWave - kPubGroup && st <= t && col >= 0 && col < Cc)
    brow[col] = cring[(st & (kCostRing - 1)) * kWave + (kWave - 1)];
}

// One step of the leaf recurrence with its backpointer code.
template <typename T, bool TR>
__device__ __forceinline__ void leaf_step(T c, T bv, T& f, T& up_prev, uint32_t& word, int t) {
  const T up = wave_shr1(bv, f);
  const T diag = up_prev, left = f;
  const T m_dl = min_t(diag, left);
  f = min_t(m_dl, up) + c;
  up_prev = up;
  const bool is_diag = (diag <= left) && (diag <= up);
  const bool is_up = TR ? (left <= up) : (up <= left);
  const uint32_t code = is_diag ? 0u : (is_up ? 1u : 2u);
  word |= code << (2 * (t & 15));
}

template <typename T>
__device__ __forceinline__ void leaf_pub(int t, int lane, const T* cring, T* brow, uint64_t* ring_out,
                                         uint32_t tag_out, int Cc) {
  if (ring_out) publish<T>(t, lane, cring, ring_out, tag_out, Cc - 1);
  else leaf_publish<T>(t, lane, cring, brow, Cc);
}

template <typename T, bool TR>
__device__ __forceinline__ T leaf_recurrence(const LeafShape& S, int sw, int Lr, int n_steps, int n_phases,
                                             bool has_succ, uint32_t* bpst, T* brow, uint64_t* ring_out,
                                             uint32_t tag_out, T* cring, const T* bring, int lane) {
  const T INF = inf_t<T>();
  // Unpredicated steps as in the pass kernel: +inf before a lane's row
  // starts, DIAG = 0 for the block's first cell.
  T f = INF;
  T up_prev = (sw == 0 && lane == 0) ? T(0) : INF;
  uint32_t word = 0;
  lds_barrier();  // phase -1
  // tie-exact mode: the origin holds its value in the whole table (cost slot
  // of lane 0, step 0), so that F(origin) = 0 + f0 exactly
  if (sw == 0 && lane == 0 && S.f0 == S.f0) cring[0] = (T)S.f0;
  for (int k = 0; k < n_phases; ++k) {
    const int t0 = k * kPhase;
    T* const hp = cring + (t0 & (kCostRing - 1)) * kWave + lane;  // the phase's slots, also the history
    const T* cp = hp;
    const T* bp = bring + in_vgpr(t0 & (2 * kPhase - 1));
    if (t0 + kPhase <= n_steps) {
      constexpr int G = kStepGroup;
      T cb[2][G], bb[2][G];
#pragma unroll
      for (int i = 0; i < G; ++i) {
        cb[0][i] = cp[i * kWave];
        bb[0][i] = bp[i];
      }
#pragma unroll
      for (int g = 0; g < kPhase / G; ++g) {
        if (g + 1 < kPhase / G) {
#pragma unroll
          for (int i = 0; i < G; ++i) {
            cb[(g + 1) & 1][i] = cp[((g + 1) * G + i) * kWave];
            bb[(g + 1) & 1][i] = bp[(g + 1) * G + i];
          }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) {
          const int u = g * G + i;
          // history as in the pass kernel: previous value off the chain,
          // a group's last value written and published at once
          if ((u & (kPubGroup - 1)) != 0) hp[(u - 1) * kWave] = f;
          leaf_step<T, TR>(cb[g & 1][i], bb[g & 1][i], f, up_prev, word, u);
          if ((u & 15) == 15) {
            bpst[((t0 + u) >> 4) * kWave + lane] = word;
            word = 0u;
          }
          if ((u & (kPubGroup - 1)) == kPubGroup - 1) {
            hp[u * kWave] = f;
            if (has_succ) leaf_pub<T>(t0 + u, lane, cring, brow, ring_out, tag_out, S.Cc);
          }
        }
      }
    } else {
      for (int t = t0; t < n_steps; ++t) {
        const int u = t - t0;
        if ((t & (kPubGroup - 1)) != 0) hp[(u - 1) * kWave] = f;
        leaf_step<T, TR>(cp[u * kWave], bp[u], f, up_prev, word, t);
        if ((t & 15) == 15 || t == n_steps - 1) {
          bpst[(t >> 4) * kWave + lane] = word;
          word = 0u;
        }
        if ((t & (kPubGroup - 1)) == kPubGroup - 1 || t == n_steps - 1) {
          hp[u * kWave] = f;
          // at a last step inside a group, lane 48 + (t & 15) reads what lane
          // 63 has just written: LDS operations of one wave are in order, and
          // this keeps the compiler from reordering them
          __builtin_amdgcn_wave_barrier();
          if (has_succ) leaf_pub<T>(t, lane, cring, brow, ring_out, tag_out, S.Cc);
        }
      }
    }
    lds_barrier();
  }
  (void)Lr;
  return f;  // lane Lr ends on the stripe's last cell (its column Cc-1 is the last step)
}

// Stripes s_lo..s_hi of a leaf, one after the other.  A stripe's bottom row
// reaches the next one through `brow` (same workgroup), or, when `ring`
// rows are given (the leaf's stripes run on several workgroups), through the
// leaf ring with the sweep's cell protocol and reuse rule: stripe s
// publishes into ring row s % kRing with id tag0 + s and its successor polls
// that row for that id.
struct LeafRing {
  uint64_t* rows;  // row s: the bottom row of stripe s, Cc cells; nullptr: brow
  uint32_t tag0;
};

template <typename T, int D, int CM>
__device__ __forceinline__ T leaf_sweep(const T* __restrict__ RowSrc, const T* __restrict__ ColSrc,
                                        const float* __restrict__ RowN, const float* __restrict__ ColN,
                                        const LeafShape& S, uint32_t* bp, T* brow, T* cring, T* bring,
                                        int wave, int lane, int s_lo, int s_hi, LeafRing rg, const Work& w) {
  const T INF = inf_t<T>();
  T fend = T(0);
  for (int sw = s_lo * kWave; sw <= s_hi * kWave && sw < S.R; sw += kWave) {
    const int st = sw / kWave;
    constexpr int kCW = kCellWords<T>;
    uint64_t* const ring_out = rg.rows ? rg.rows + (int64_t)(st % kRing) * S.Cc * kCW : nullptr;
    const uint64_t* const ring_in = rg.rows ? rg.rows + (int64_t)((st + kRing - 1) % kRing) * S.Cc * kCW : nullptr;
    const int Lr = min(kWave - 1, S.R - 1 - sw);
    const int n_steps = S.Cc + Lr;
    const int n_phases = (n_steps + kPhase - 1) / kPhase;
    const bool has_pred = sw > 0;
    const bool has_succ = sw + kWave < S.R;
    if (wave == 0) {
      uint32_t* bpst = bp + (int64_t)(sw / kWave) * S.Wm * kWave;
      gram_stage_barrier<CM>();
      fend = S.tr ? leaf_recurrence<T, true>(S, sw, Lr, n_steps, n_phases, has_succ, bpst, brow, ring_out,
                                             rg.tag0 + st, cring, bring, lane)
                  : leaf_recurrence<T, false>(S, sw, Lr, n_steps, n_phases, has_succ, bpst, brow, ring_out,
                                              rg.tag0 + st, cring, bring, lane);
    } else if (wave <= kProducers && is_gram(CM)) {
      // ------------------------------------------------ frame costs, Gram form (BF16 or FP16 frames)
      if constexpr (is_gram(CM))
        gram_producer<D, gram_bf16(CM), is_cos(CM), kProducers, false>(reinterpret_cast<const uint16_t*>(RowSrc), reinterpret_cast<const uint16_t*>(ColSrc), RowN,
                         ColN, S.r0 + sw, 1, S.c0, 1, 0, Lr, S.Cc - 1, n_phases, wave, lane,
                         reinterpret_cast<float*>(cring));
    } else if (wave <= kProducers && D >= 64) {
      // ------------------------------------------------ frame costs, wide frames (read from HBM)
      if constexpr (D >= 64 && !is_gram(CM)) {
        const int pw = wave - 1;
        const T* xl = RowSrc + (int64_t)(S.r0 + sw + min(lane, Lr)) * D;
        for (int k = -1; k < n_phases; ++k) {
          const int cb0 = (k + 1) * kPhase;
          if (cb0 < S.Cc) {
            int gj[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) gj[i] = __builtin_amdgcn_readfirstlane(S.c0 + min(cb0 + pw + i * kProducers, S.Cc - 1));
            T cv[4];
            frame_cost4_wide<T, D, 1, is_cos(CM)>(xl, ColSrc + (int64_t)gj[0] * D, ColSrc + (int64_t)gj[1] * D,
                                   ColSrc + (int64_t)gj[2] * D, ColSrc + (int64_t)gj[3] * D, cv);
#pragma unroll
            for (int i = 0; i < 4; ++i)
              cring[((cb0 + pw + i * kProducers + lane) & (kCostRing - 1)) * kWave + lane] = cv[i];
          }
          lds_barrier();
        }
      }
    } else if (wave <= kProducers) {
      // ------------------------------------------------ frame costs
      if constexpr (D < 64) {
        const int pw = wave - 1;
        T x[D];
        {
          const T* xr = RowSrc + (int64_t)(S.r0 + sw + min(lane, Lr)) * D;
  #pragma unroll
          for (int q = 0; q < D; ++q) x[q] = xr[q];
        }
        for (int k = -1; k < n_phases; ++k) {
          const int cb0 = (k + 1) * kPhase;
          if (cb0 < S.Cc) {
  #pragma unroll
            for (int i = 0; i < kPhase / kProducers; i += 2) {
              const int j0 = cb0 + pw + i * kProducers, j1 = j0 + kProducers;
              const int gj0 = __builtin_amdgcn_readfirstlane(S.c0 + min(j0, S.Cc - 1));
              const int gj1 = __builtin_amdgcn_readfirstlane(S.c0 + min(j1, S.Cc - 1));
              T cv0, cv1;
              frame_cost2<T, D, is_cos(CM)>(x, ColSrc + (int64_t)gj0 * D, ColSrc + (int64_t)gj1 * D, cv0, cv1);
              cring[((j0 + lane) & (kCostRing - 1)) * kWave + lane] = cv0;
              cring[((j1 + lane) & (kCostRing - 1)) * kWave + lane] = cv1;
            }
          }
          lds_barrier();
        }
      }
    } else {
      // ------------------------------------------------ boundary input
      gram_stage_barrier<CM>();
      if (ring_in) {
        // lanes 0..kPhase*kCW-1: word lane % kCW of column lane / kCW of the chunk
        for (int k = -1; k < n_phases; ++k) {
          const int col = (k + 1) * kPhase + lane / kCW;
          if (lane < kPhase * kCW) {
            uint32_t half = (kCW == 2) ? ((lane % 2) ? 0x7FF00000u : 0u) : 0x7F800000u;  // a half of +inf
            if (has_pred && col < S.Cc)
              half = (uint32_t)poll_word(ring_in + (int64_t)col * kCW + lane % kCW, rg.tag0 + st - 1, w);
            reinterpret_cast<uint32_t*>(bring)[(col & (2 * kPhase - 1)) * kCW + lane % kCW] = half;
          }
          lds_barrier();
        }
      } else {
        for (int k = -1; k < n_phases; ++k) {
          const int col = (k + 1) * kPhase + lane;
          if (lane < kPhase) bring[col & (2 * kPhase - 1)] = (has_pred && col < S.Cc) ? brow[col] : INF;
          lds_barrier();
        }
      }
    }
    // the stripe's bottom row and pointers are complete for the next stripe
    __syncthreads();
  }
  return fend;
}

// Backtrace from the block's last cell by the whole recurrence wave in
// lockstep, one row per iteration. The position is wave-uniform, so the
// arithmetic runs on the scalar unit. In a row, the walk keeps moving along
// the row up to the first cell (from the right) whose pointer is DIAG or
// vertical: a bit scan over the row's packed 2-bit codes finds it, one word
// of 16 steps at a time. The row's run of cells is then stored by the lanes
// at once, backwards from slot_end of the diagonal-indexed path scratch.
// The walk goes stripe by stripe (walk_rows takes the rows of stripe s from
// its block of pointer words, wherever that block is), then walk_row0 ends it
// on row 0; the result is the number of cells written (the block's first
// cell only for the pair's first leaf: otherwise it is the previous leaf's
// last cell).
struct LeafWalk {
  int R, Cc, Wm, oi, oj;  // wave-uniform shape and block origin in the pair
  bool tr, first;
  int ri, cj, cnt;        // position and cells written so far
  int64_t slot_end;
};

__device__ __forceinline__ LeafWalk walk_begin(const LeafShape& S, const LeafDesc& Lf, const PairDesc& pd,
                                               int64_t slot_end) {
  LeafWalk k;
  k.R = __builtin_amdgcn_readfirstlane(S.R);
  k.Cc = __builtin_amdgcn_readfirstlane(S.Cc);
  k.Wm = __builtin_amdgcn_readfirstlane(S.Wm);
  k.tr = __builtin_amdgcn_readfirstlane(S.tr ? 1 : 0) != 0;
  k.first = __builtin_amdgcn_readfirstlane(Lf.first) != 0;
  k.oi = __builtin_amdgcn_readfirstlane((int)(Lf.i0 - pd.x_off));
  k.oj = __builtin_amdgcn_readfirstlane((int)(Lf.j0 - pd.y_off));
  k.ri = k.R - 1;
  k.cj = k.Cc - 1;
  k.cnt = 0;
  k.slot_end = slot_end;
  return k;
}

// Rows of stripe s (ri >> 6 == s, ri > 0); blk holds the stripe's pointer
// words, word b of lane r at blk[b * 64 + r].  One row is a straight line of
// scalar work in the common case (the row's run ends in the word of its
// entry step); a run that crosses into earlier words takes the inner loop.
__device__ __forceinline__ void walk_rows(const uint32_t* blk, int s, LeafWalk& k, int2* tpath, int lane) {
  constexpr uint32_t kLo = 0x55555555u;  // bit 0 of every 2-bit field
  // code 0 DIAG; 1 UP and 2 LEFT in the block's own orientation, swapped
  // when transposed. A move along the row (cj - 1) is code 2 or 3, or code 1
  // when transposed; field mask of the other codes:
  //   not transposed: hi bit clear;  transposed: hi bit set or lo bit clear.
  const bool tr = k.tr;
  auto stop_mask = [tr](uint32_t wd) -> uint32_t {
    const uint32_t lo = wd & kLo, hi = (wd >> 1) & kLo;
    return tr ? (hi | (~lo & kLo)) : (~hi & kLo);
  };
  const int lo_row = max(s * kWave, 1);
  // a cell (ri, c) of the row is written as (rbase + ri, cbase + c), or
  // swapped when transposed
  const int rbase = tr ? k.oj : k.oi, cbase = tr ? k.oi : k.oj;
  int ri = k.ri, cj = k.cj, cnt = k.cnt;
  while (ri >= lo_row) {
    const int r = ri & (kWave - 1);
    const int t = cj + r;  // step of (ri, cj) in lane r's pointer words
    int b = t >> 4;
    uint32_t wd = (uint32_t)__builtin_amdgcn_readfirstlane((int)blk[b * kWave + r]);
    const int p = t & 15;
    uint32_t m = stop_mask(wd) & ((p < 15) ? ((1u << (2 * p + 2)) - 1u) : ~0u);  // steps b*16 .. t
    while (m == 0u && (b << 4) > r) {  // the run continues into the previous word
      --b;
      wd = (uint32_t)__builtin_amdgcn_readfirstlane((int)blk[b * kWave + r]);
      m = stop_mask(wd);
    }
    const int f = (31 - __builtin_clz(m | 1u)) >> 1;  // field of the stop (unused when m == 0)
    // column where the row is left: 0 when the run reaches column 0 or the
    // stop lies left of it (not the row's)
    const int cx = (m != 0u) ? max((b << 4) + f - r, 0) : 0;
    const bool diag = (m != 0u) && ((wd >> (2 * f)) & 3u) == 0u;
    const int n = cj - cx + 1;  // cells (ri, cj) .. (ri, cx)
    int2* const row_end = tpath + (k.slot_end - cnt);
    const int cv = cbase + cj - lane, rv = rbase + ri;
    if (lane < n) row_end[-lane] = tr ? make_int2(cv, rv) : make_int2(rv, cv);
    for (int q0 = kWave; q0 < n; q0 += kWave) {  // runs longer than a wave
      if (q0 + lane < n) row_end[-(q0 + lane)] = tr ? make_int2(cv - q0, rv) : make_int2(rv, cv - q0);
    }
    cnt += n;
    // leave the row: straight up at column 0 (the only move), DIAG for code 0, else up
    cj = (cx == 0) ? 0 : (diag ? cx - 1 : cx);
    --ri;
  }
  k.ri = ri;
  k.cj = cj;
  k.cnt = cnt;
}

// Row 0: cells (0, cj) .. (0, 1), and (0, 0) for the pair's first leaf.
__device__ __forceinline__ int walk_row0(LeafWalk& k, int2* tpath, int lane) {
  const int n0 = k.cj + (k.first ? 1 : 0);
  for (int q0 = 0; q0 < n0; q0 += kWave) {
    const int q = q0 + lane;
    if (q < n0)
      tpath[k.slot_end - k.cnt - q] = k.tr ? make_int2(k.oi + k.cj - q, k.oj) : make_int2(k.oi, k.oj + k.cj - q);
  }
  k.cnt += n0;
  return k.cnt;
}

// The whole walk over pointer words bp in one memory space (the leaf's LDS
// or its global scratch), stripe block s at bp + s * Wm * 64.
__device__ __forceinline__ int leaf_backtrace(const uint32_t* bp, const LeafShape& S, const LeafDesc& Lf,
                                              const PairDesc& pd, int64_t slot_end, int2* tpath, int lane) {
  LeafWalk k = walk_begin(S, Lf, pd, slot_end);
  for (int s = (k.R - 1) >> 6; s >= 0; --s) walk_rows(bp + (int64_t)s * k.Wm * kWave, s, k, tpath, lane);
  return walk_row0(k, tpath, lane);
}

// The FP64 frame cost of one path cell from the caller's frames (FP64 or
// FP32, widened): the Euclidean cost, or the cosine cost with each frame
// divided by its norm (a zero frame kept zero).
template <bool kCos, typename TI>
__device__ __forceinline__ double path_cell_cost(const TI* xr, const TI* yr, int d) {
  if constexpr (kCos) {
    double nx = 0.0, ny = 0.0;
    for (int k = 0; k < d; ++k) nx = __builtin_fma((double)xr[k], (double)xr[k], nx);
    for (int k = 0; k < d; ++k) ny = __builtin_fma((double)yr[k], (double)yr[k], ny);
    nx = __builtin_sqrt(nx);
    ny = __builtin_sqrt(ny);
    double ss = 0.0;
    for (int k = 0; k < d; ++k) {
      const double xk = nx > 0.0 ? (double)xr[k] / nx : 0.0;
      const double yk = ny > 0.0 ? (double)yr[k] / ny : 0.0;
      ss = __builtin_fma(xk, yk, ss);
    }
    const double c = 1.0 - ss;
    return c < 0.0 ? 0.0 : c;
  } else {
    double ss = 0.0;
    for (int k = 0; k < d; ++k) {
      const double ee = (double)xr[k] - (double)yr[k];
      ss = __builtin_fma(ee, ee, ss);
    }
    return __builtin_sqrt(ss);
  }
}

// Wait until `*p` reaches `target` (another workgroup's stripes of the same
// leaf, all dequeued before this one, count themselves done there), bounded
// like poll_word; every lane of the calling wave polls the same word.
__device__ __forceinline__ void wait_count(const int32_t* p, int32_t target, const Work& w) {
  if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) return;
  const uint64_t t0 = wall_clock64();
  for (uint32_t it = 0;; ++it) {
    __builtin_amdgcn_s_sleep(2);
    const int32_t err = __hip_atomic_load(&w.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target || err != 0) return;
    if (wall_clock64() - t0 > w.spin_ticks || it > kSpinIterCap) {
      set_error(w.ctl, kErrSpinTimeout);
      return;
    }
  }
}

// Leaf tickets are (leaf, stripe) pairs, a leaf's stripes top to bottom on
// consecutive tickets.  A leaf of one ticket (one stripe, or any leaf of a
// call with many pairs) is solved by one workgroup, stripe after stripe, with
// its pointers in LDS when they fit.  The stripes of a split leaf run on as
// many workgroups as take their tickets, chained through the leaf ring like
// the sweep's stripes; each writes its pointer words to the leaf's global
// scratch, and every stripe but the last then counts itself done in
// leaf_done (after a release fence).  The workgroup of the last stripe waits
// for that count (its stripes were dequeued before it, so they run) and
// walks the path back, copying each stripe's pointer block from global
// scratch into LDS while the recurrence wave walks the one before, when two
// blocks fit there.
template <typename T, int D, int CM>
__global__ __launch_bounds__(kLeafThreads, 3) void leaf_kernel(
    const T* __restrict__ X, const T* __restrict__ Y, Work w, int64_t lds_leaf_bytes, const void* Xorig,
    const void* Yorig, int in_f64, int d) {
  extern __shared__ __align__(16) unsigned char lds_raw[];  // pointers and bottom row when they fit
  __shared__ T cring[kCostRing * kWave];
  __shared__ T bring[2 * kPhase];
  __shared__ int sh_ticket, sh_cnt;
  __shared__ double2 sh_acc[kLeafThreads / kWave];
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = (int)(threadIdx.x % kWave);
  if (wave == 0) __builtin_amdgcn_s_setprio(3);  // the recurrence wave sets the pace
  Ctl* ctl = w.ctl;
  const int n_leaf = clamp_count(ctl, ctl->n_leaf, w.caps.leaf);
  const int n_tk = clamp_count(ctl, ctl->leaf_stripes, w.caps.leaf_tk);

  for (int iter = 0; iter <= n_tk; ++iter) {  // each iteration consumes one ticket
    if (threadIdx.x == 0) sh_ticket = call_failed(w) ? -1 : atomicAdd(&ctl->leaf_ticket, 1);
    lds_barrier();
    const int tk = __builtin_amdgcn_readfirstlane(sh_ticket);
    lds_barrier();
    if (tk >= n_tk || tk < 0) break;
    const int2 lt = w.leaf_tk[tk];
    const int li = __builtin_amdgcn_readfirstlane(lt.x), st = __builtin_amdgcn_readfirstlane(lt.y);
    if (li < 0 || li >= n_leaf) {
      if (threadIdx.x == 0) set_error(ctl, kErrBadLeaf);
      continue;
    }
    const LeafDesc Lf = w.leaves[li];
    if (Lf.pair < 0 || Lf.pair >= w.n_pairs) {
      if (threadIdx.x == 0) set_error(ctl, kErrBadLeaf);
      continue;
    }
    const PairDesc pd = w.pairs[Lf.pair];
    const int Mb = Lf.i1 - Lf.i0 + 1, Nb = Lf.j1 - Lf.j0 + 1;
    // a leaf lies inside its pair and is non-empty, its stripe count and
    // this ticket's stripe agree with its shape; refuse anything else
    const int nst = __builtin_amdgcn_readfirstlane(Lf.n_stripes);
    const bool split = __builtin_amdgcn_readfirstlane(Lf.split) != 0;
    const int ntk = split ? nst : 1;  // tickets of the leaf
    if (Mb < 1 || Nb < 1 || Lf.i0 < pd.x_off || Lf.j0 < pd.y_off || Lf.i1 >= pd.x_off + pd.M ||
        Lf.j1 >= pd.y_off + pd.N || nst != (min(Mb, Nb) + kWave - 1) / kWave || st < 0 || st >= ntk ||
        Lf.stripe_off + st != tk || (split && (nst < 2 || Lf.scratch_off < 0))) {
      if (threadIdx.x == 0) set_error(ctl, kErrBadLeaf);
      continue;
    }
    LeafShape S;
    S.tr = Mb > Nb;
    S.R = S.tr ? Nb : Mb;
    S.Cc = S.tr ? Mb : Nb;
    S.r0 = S.tr ? Lf.j0 : Lf.i0;
    S.c0 = S.tr ? Lf.i0 : Lf.j0;
    S.Wm = (S.Cc + kWave - 1 + 15) / 16;
    S.f0 = Lf.f0;
    // in the Gram form X and Y are the 16-bit frames, reached through w.X / w.Y
    const T* __restrict__ Xs = is_gram(CM) ? static_cast<const T*>(w.X) : X;
    const T* __restrict__ Ys = is_gram(CM) ? static_cast<const T*>(w.Y) : Y;
    const T* __restrict__ RowSrc = S.tr ? Ys : Xs;
    const T* __restrict__ ColSrc = S.tr ? Xs : Ys;
    const float* __restrict__ RowN = S.tr ? w.Yn : w.Xn;
    const float* __restrict__ ColN = S.tr ? w.Xn : w.Yn;
    const int64_t bpw = (int64_t)nst * S.Wm * kWave;
    const int64_t e = (int64_t)(Lf.i1 - pd.x_off) + (Lf.j1 - pd.y_off);
    const int64_t slot_end = pd.pbase + e;  // the block's last cell sits on diagonal e
    T fend;
    int cnt_written = 0;
    if (!split && Lf.scratch_off < 0) {
      // the whole leaf on this workgroup, stripes one after another, pointers in LDS
      uint32_t* bp = reinterpret_cast<uint32_t*>(lds_raw);
      fend = leaf_sweep<T, D, CM>(RowSrc, ColSrc, RowN, ColN, S, bp, reinterpret_cast<T*>(bp + bpw), cring, bring,
                                  wave, lane, 0, nst - 1, LeafRing{nullptr, 0u}, w);
      if (wave == 0) cnt_written = leaf_backtrace(bp, S, Lf, pd, slot_end, w.tpath, lane);
    } else if (!split) {
      uint32_t* bp = w.leaf_scratch + Lf.scratch_off;
      fend = leaf_sweep<T, D, CM>(RowSrc, ColSrc, RowN, ColN, S, bp, reinterpret_cast<T*>(bp + bpw), cring, bring,
                                  wave, lane, 0, nst - 1, LeafRing{nullptr, 0u}, w);
      if (wave == 0) cnt_written = leaf_backtrace(bp, S, Lf, pd, slot_end, w.tpath, lane);
    } else {
      // one stripe of a taller leaf; ids of the leaf ring: 0xFF << 24 | (ticket + 1),
      // unique within a call and never 0 (the ring is cleared when the call starts)
      uint32_t* bp = w.leaf_scratch + Lf.scratch_off;
      const LeafRing rg{w.leaf_ring + Lf.ring_off * kCellWords<T>, (0xFFu << 24) | (uint32_t)(Lf.stripe_off + 1)};
      fend = leaf_sweep<T, D, CM>(RowSrc, ColSrc, RowN, ColN, S, bp, nullptr, cring, bring, wave, lane, st, st, rg,
                                  w);
      if (wave == 0) {
        wait_vmem();       // this wave's pointer words (and published cells) are written
        __threadfence();   // and visible to the other workgroups of the leaf
      }
      if (st < nst - 1) {
        if (threadIdx.x == 0) __hip_atomic_fetch_add(&w.leaf_done[li], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        continue;  // the last stripe's workgroup walks the path
      }
      if (wave == 0) wait_count(&w.leaf_done[li], nst - 1, w);
      __syncthreads();
      __threadfence();  // the other stripes' pointer words, read below
      const int64_t blk = (int64_t)S.Wm * kWave;  // words of one stripe's pointer block
      uint32_t* buf = reinterpret_cast<uint32_t*>(lds_raw);
      if (2 * blk * 4 <= lds_leaf_bytes) {
        LeafWalk k;
        if (wave == 0) k = walk_begin(S, Lf, pd, slot_end);
        for (int64_t u = threadIdx.x; u < blk; u += blockDim.x) buf[((nst - 1) & 1) * blk + u] = bp[(nst - 1) * blk + u];
        __syncthreads();
        for (int s = nst - 1; s >= 0; --s) {
          if (wave == 0) {
            walk_rows(buf + (s & 1) * blk, s, k, w.tpath, lane);
          } else if (s > 0) {
            for (int64_t u = threadIdx.x - kWave; u < blk; u += blockDim.x - kWave)
              buf[((s - 1) & 1) * blk + u] = bp[(s - 1) * blk + u];
          }
          __syncthreads();
        }
        if (wave == 0) cnt_written = walk_row0(k, w.tpath, lane);
      } else if (wave == 0) {
        cnt_written = leaf_backtrace(bp, S, Lf, pd, slot_end, w.tpath, lane);
      }
    }

    if (wave == 0) {
      fend = __shfl(fend, (S.R - 1) % kWave);
      if (lane == 0) {
        w.cnt[slot_end] = cnt_written;
        atomicAdd((unsigned long long*)&ctl->leaf_cells, (unsigned long long)((int64_t)S.R * S.Cc));
        if (Lf.first && Lf.i1 == pd.x_off + pd.M - 1 && Lf.j1 == pd.y_off + pd.N - 1)
          w.smin[Lf.pair] = (double)fend;
        sh_cnt = cnt_written;
      }
      wait_vmem();  // the path cells of the walk are written before the other waves read them
    }
    __syncthreads();
    // FP64 cost of the cells this leaf wrote, from the caller's inputs, by
    // every wave: thread u takes cells u, u + blockDim.x, ... (cells read
    // past this CU's L1, which may hold an older copy of their lines)
    const int nc = __builtin_amdgcn_readfirstlane(sh_cnt);
    double2 acc = make_double2(0.0, 0.0);
    for (int q = threadIdx.x; q < nc; q += blockDim.x) {
      const uint64_t cw = __hip_atomic_load(reinterpret_cast<const uint64_t*>(w.tpath + (slot_end - nc + 1 + q)),
                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int2 cell = make_int2((int)(uint32_t)cw, (int)(uint32_t)(cw >> 32));
      const int64_t gi = pd.x_off + cell.x, gj = pd.y_off + cell.y;
      const double c = in_f64 ? path_cell_cost<is_cos(CM)>(static_cast<const double*>(Xorig) + gi * d,
                                                            static_cast<const double*>(Yorig) + gj * d, d)
                              : path_cell_cost<is_cos(CM)>(static_cast<const float*>(Xorig) + gi * d,
                                                            static_cast<const float*>(Yorig) + gj * d, d);
      acc = two_sum_acc(acc, c);
    }
    // fixed-order tree reduction over each wave, then over the waves in order
    for (int off = 1; off < kWave; off <<= 1) {
      const double2 other = make_double2(__shfl_xor(acc.x, off), __shfl_xor(acc.y, off));
      acc = ((lane & off) == 0) ? dd_add(acc, other) : dd_add(other, acc);
    }
    if (lane == 0) sh_acc[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double2 tot = sh_acc[0];
      for (int v = 1; v < kLeafThreads / kWave; ++v) tot = dd_add(tot, sh_acc[v]);
      w.leaf_cost[li] = tot;
    }
  }
}

// ----------------------------------------------------------------- launchers
}  // namespace dtw

#include "dtw_launch.h"

namespace dtw {

int pick_dmax(int d) {
  if (d <= 4) return 4;
  if (d <= 8) return 8;
  if (d <= 12) return 12;
  if (d <= 16) return 16;
  if (d <= 24) return 24;
  if (d <= 32) return 32;
  if (d <= 64) return 64;
  if (d <= 128) return 128;
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
    case 64: { constexpr int D_ = 64; CALL; } break; \
    case 128: { constexpr int D_ = 128; CALL; } break; \
    default: return hipErrorInvalidValue;            \
  }

// Padded frame width of the Gram form's 16-bit copies (multiples of 16 for
// the matrix-core K blocks).
int pick_dgram(int d) {
  if (d <= 32) return 32;
  if (d <= 64) return 64;
  if (d <= 128) return 128;
  return 0;
}

#define DTW_DISPATCH_DGRAM(DM, CALL)                   \
  switch (DM) {                                        \
    case 32: { constexpr int D_ = 32; CALL; } break;   \
    case 64: { constexpr int D_ = 64; CALL; } break;   \
    case 128: { constexpr int D_ = 128; CALL; } break; \
    default: return hipErrorInvalidValue;              \
  }

// Sweep launch for the precision of `w`: FP64 or FP32 Euclidean costs on the
// VALU, or BF16 Gram costs on the matrix cores with the FP32 recurrence.
hipError_t launch_pass(const Work& w, int level, int grid, hipStream_t st) {
  const float* nf = nullptr;
  if (w.precision == DTW_PREC_BF16_COST && w.cost == DTW_COST_COSINE) {
    DTW_DISPATCH_DGRAM(pick_dgram(w.d), return launch_checked(&pass_kernel<float, D_, kCostGramCos>, grid,
                                                               pass_threads(kCostGramCos), 0, st, nf, nf, w, level))
  } else if (w.precision == DTW_PREC_FP16_COST && w.cost == DTW_COST_COSINE) {
    DTW_DISPATCH_DGRAM(pick_dgram(w.d), return launch_checked(&pass_kernel<float, D_, kCostGramF16Cos>, grid,
                                                               pass_threads(kCostGramF16Cos), 0, st, nf, nf, w, level))
  } else if (w.precision == DTW_PREC_BF16_COST) {
    DTW_DISPATCH_DGRAM(pick_dgram(w.d), return launch_checked(&pass_kernel<float, D_, kCostGram>, grid,
                                                               pass_threads(kCostGram), 0, st, nf, nf, w, level))
  } else if (w.precision == DTW_PREC_FP16_COST) {
    DTW_DISPATCH_DGRAM(pick_dgram(w.d), return launch_checked(&pass_kernel<float, D_, kCostGramF16>, grid,
                                                               pass_threads(kCostGramF16), 0, st, nf, nf, w, level))
  } else if (w.precision == DTW_PREC_FP32 && w.cost == DTW_COST_COSINE) {
    DTW_DISPATCH_DMAX(pick_dmax(w.d), return launch_checked(&pass_kernel<float, D_, kCostCosine>, grid, pass_threads(kCostCosine), 0,
                                                             st, static_cast<const float*>(w.X),
                                                             static_cast<const float*>(w.Y), w, level))
  } else if (w.precision == DTW_PREC_FP32) {
    DTW_DISPATCH_DMAX(pick_dmax(w.d), return launch_checked(&pass_kernel<float, D_, kCostEuclid>, grid, pass_threads(kCostEuclid), 0,
                                                             st, static_cast<const float*>(w.X),
                                                             static_cast<const float*>(w.Y), w, level))
  } else if (w.tie && w.cost == DTW_COST_COSINE) {
    DTW_DISPATCH_DMAX(pick_dmax(w.d), return launch_checked(&pass_kernel<double, D_, kCostCosine, true>, grid,
                                                             pass_threads(kCostCosine), 0, st,
                                                             static_cast<const double*>(w.X),
                                                             static_cast<const double*>(w.Y), w, level))
  } else if (w.tie) {
    DTW_DISPATCH_DMAX(pick_dmax(w.d), return launch_checked(&pass_kernel<double, D_, kCostEuclid, true>, grid,
                                                             pass_threads(kCostEuclid), 0, st,
                                                             static_cast<const double*>(w.X),
                                                             static_cast<const double*>(w.Y), w, level))
  } else if (w.cost == DTW_COST_COSINE) {
    DTW_DISPATCH_DMAX(pick_dmax(w.d), return launch_checked(&pass_kernel<double, D_, kCostCosine>, grid, pass_threads(kCostCosine), 0,
                                                             st, static_cast<const double*>(w.X),
                                                             static_cast<const double*>(w.Y), w, level))
  } else {
    DTW_DISPATCH_DMAX(pick_dmax(w.d), return launch_checked(&pass_kernel<double, D_, kCostEuclid>, grid, pass_threads(kCostEuclid), 0,
                                                             st, static_cast<const double*>(w.X),
                                                             static_cast<const double*>(w.Y), w, level))
  }
  return hipErrorInvalidValue;
}

hipError_t launch_leaf(const Work& w, int grid, int64_t lds_leaf_bytes, const void* Xo, const void* Yo, int in_f64,
                       hipStream_t st) {
  const size_t dyn = (size_t)lds_leaf_bytes;
  const float* nf = nullptr;
  if (w.precision == DTW_PREC_BF16_COST && w.cost == DTW_COST_COSINE) {
    DTW_DISPATCH_DGRAM(pick_dgram(w.d), return launch_checked(&leaf_kernel<float, D_, kCostGramCos>, grid,
                                                               kLeafThreads, dyn, st, nf, nf, w, lds_leaf_bytes, Xo, Yo,
                                                               in_f64, w.d))
  } else if (w.precision == DTW_PREC_FP16_COST && w.cost == DTW_COST_COSINE) {
    DTW_DISPATCH_DGRAM(pick_dgram(w.d), return launch_checked(&leaf_kernel<float, D_, kCostGramF16Cos>, grid,
                                                               kLeafThreads, dyn, st, nf, nf, w, lds_leaf_bytes, Xo, Yo,
                                                               in_f64, w.d))
  } else if (w.precision == DTW_PREC_BF16_COST) {
    DTW_DISPATCH_DGRAM(pick_dgram(w.d), return launch_checked(&leaf_kernel<float, D_, kCostGram>, grid, kLeafThreads,
                                                               dyn, st, nf, nf, w, lds_leaf_bytes, Xo, Yo, in_f64, w.d))
  } else if (w.precision == DTW_PREC_FP16_COST) {
    DTW_DISPATCH_DGRAM(pick_dgram(w.d), return launch_checked(&leaf_kernel<float, D_, kCostGramF16>, grid, kLeafThreads,
                                                               dyn, st, nf, nf, w, lds_leaf_bytes, Xo, Yo, in_f64, w.d))
  } else if (w.precision == DTW_PREC_FP32 && w.cost == DTW_COST_COSINE) {
    DTW_DISPATCH_DMAX(pick_dmax(w.d), return launch_checked(&leaf_kernel<float, D_, kCostCosine>, grid, kLeafThreads,
                                                             dyn, st, static_cast<const float*>(w.X),
                                                             static_cast<const float*>(w.Y), w, lds_leaf_bytes, Xo, Yo,
                                                             in_f64, w.d))
  } else if (w.precision == DTW_PREC_FP32) {
    DTW_DISPATCH_DMAX(pick_dmax(w.d), return launch_checked(&leaf_kernel<float, D_, kCostEuclid>, grid, kLeafThreads,
                                                             dyn, st, static_cast<const float*>(w.X),
                                                             static_cast<const float*>(w.Y), w, lds_leaf_bytes, Xo, Yo,
                                                             in_f64, w.d))
  } else if (w.cost == DTW_COST_COSINE) {
    DTW_DISPATCH_DMAX(pick_dmax(w.d), return launch_checked(&leaf_kernel<double, D_, kCostCosine>, grid, kLeafThreads,
                                                             dyn, st, static_cast<const double*>(w.X),
                                                             static_cast<const double*>(w.Y), w, lds_leaf_bytes, Xo, Yo,
                                                             in_f64, w.d))
  } else {
    DTW_DISPATCH_DMAX(pick_dmax(w.d), return launch_checked(&leaf_kernel<double, D_, kCostEuclid>, grid, kLeafThreads,
                                                             dyn, st, static_cast<const double*>(w.X),
                                                             static_cast<const double*>(w.Y), w, lds_leaf_bytes, Xo, Yo,
                                                             in_f64, w.d))
  }
  return hipErrorInvalidValue;
}

// Dynamic LDS left to the leaf kernels (pointers and bottom row) once their
// static LDS is taken from `lds_max`, per compute type (FP64; FP32 and the
// Gram form): the smallest over the frame widths, also set as each kernel's
// dynamic LDS limit.
hipError_t leaf_lds_setup(int64_t lds_max, int64_t* dyn_f64, int64_t* dyn_f32) {
  int64_t lim[2] = {lds_max, lds_max};
#define DTW_LEAF_STATIC(T_, D_, CM_, I_)                                                                \
  {                                                                                                     \
    hipFuncAttributes a;                                                                                \
    hipError_t r = hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&leaf_kernel<T_, D_, CM_>)); \
    if (r != hipSuccess) return r;                                                                      \
    const int64_t left = lds_max - (int64_t)a.sharedSizeBytes - 64;                                     \
    if (left < lim[I_]) lim[I_] = left;                                                                 \
  }
#define DTW_LEAF_ALL(M_)                                                                                  \
  M_(double, 4, kCostEuclid, 0) M_(double, 8, kCostEuclid, 0) M_(double, 12, kCostEuclid, 0)              \
  M_(double, 16, kCostEuclid, 0) M_(double, 24, kCostEuclid, 0) M_(double, 32, kCostEuclid, 0)            \
  M_(double, 64, kCostEuclid, 0) M_(double, 128, kCostEuclid, 0)                                          \
  M_(float, 4, kCostEuclid, 1) M_(float, 8, kCostEuclid, 1) M_(float, 12, kCostEuclid, 1)                 \
  M_(float, 16, kCostEuclid, 1) M_(float, 24, kCostEuclid, 1) M_(float, 32, kCostEuclid, 1)               \
  M_(float, 64, kCostEuclid, 1) M_(float, 128, kCostEuclid, 1)                                            \
  M_(double, 4, kCostCosine, 0) M_(double, 8, kCostCosine, 0) M_(double, 12, kCostCosine, 0)              \
  M_(double, 16, kCostCosine, 0) M_(double, 24, kCostCosine, 0) M_(double, 32, kCostCosine, 0)            \
  M_(double, 64, kCostCosine, 0) M_(double, 128, kCostCosine, 0)                                          \
  M_(float, 4, kCostCosine, 1) M_(float, 8, kCostCosine, 1) M_(float, 12, kCostCosine, 1)                 \
  M_(float, 16, kCostCosine, 1) M_(float, 24, kCostCosine, 1) M_(float, 32, kCostCosine, 1)               \
  M_(float, 64, kCostCosine, 1) M_(float, 128, kCostCosine, 1)                                            \
  M_(float, 32, kCostGram, 1) M_(float, 64, kCostGram, 1) M_(float, 128, kCostGram, 1)                   \
  M_(float, 32, kCostGramF16, 1) M_(float, 64, kCostGramF16, 1) M_(float, 128, kCostGramF16, 1)                \
  M_(float, 32, kCostGramCos, 1) M_(float, 64, kCostGramCos, 1) M_(float, 128, kCostGramCos, 1)                \
  M_(float, 32, kCostGramF16Cos, 1) M_(float, 64, kCostGramF16Cos, 1) M_(float, 128, kCostGramF16Cos, 1)
  DTW_LEAF_ALL(DTW_LEAF_STATIC)
#undef DTW_LEAF_STATIC
  lim[0] &= ~(int64_t)255;
  lim[1] &= ~(int64_t)255;
  if (lim[0] < 0 || lim[1] < 0) return hipErrorInvalidValue;
#define DTW_SET_ATTR(T_, D_, CM_, I_)                                                                     \
  {                                                                                                     \
    hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void*>(&leaf_kernel<T_, D_, CM_>),        \
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim[I_]);       \
    if (r != hipSuccess) return r;                                                                      \
  }
  DTW_LEAF_ALL(DTW_SET_ATTR)
#undef DTW_SET_ATTR
#undef DTW_LEAF_ALL
  *dyn_f64 = lim[0];
  *dyn_f32 = lim[1];
  return hipSuccess;
}

}  // namespace dtw
