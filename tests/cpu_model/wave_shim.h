// Wave-level stand-ins for the CPU model (tests only): a workgroup of the
// wave kernels is one 64-lane wave, run as 64 threads; every cross-lane
// operation is an exchange through a shared slot array between two barrier
// waits, which is exact for code where all 64 lanes reach the operation
// together (the kernels only use them in converged code).
#pragma once
#include <chrono>
#include <cstring>

#include "hip/hip_runtime.h"

extern uint64_t cpu_wave_slots[16][64];
extern unsigned char cpu_dynamic_lds[];

// Lane index within the wave, and an exchange among the 64 lanes of one wave.
inline int cpu_lane() { return (int)(threadIdx.x & 63); }
template <class T>
inline T cpu_wave_exchange(T v, int src) {
  uint64_t bits = 0;
  std::memcpy(&bits, &v, sizeof(T));
  uint64_t* slots = cpu_wave_slots[threadIdx.x / 64];
  slots[cpu_lane()] = bits;
  cpu_wave_barrier->arrive_and_wait();
  const uint64_t r = slots[src & 63];
  cpu_wave_barrier->arrive_and_wait();
  T out;
  std::memcpy(&out, &r, sizeof(T));
  return out;
}

// Bit l set when lane l's predicate holds (all 64 lanes take part).
inline uint64_t cpu_ballot(bool pred) {
  uint64_t* slots = cpu_wave_slots[threadIdx.x / 64];
  slots[cpu_lane()] = pred ? 1u : 0u;
  cpu_wave_barrier->arrive_and_wait();
  uint64_t m = 0;
  for (int l = 0; l < 64; ++l) m |= (slots[l] & 1u) << l;
  cpu_wave_barrier->arrive_and_wait();
  return m;
}

inline int cpu_update_dpp(int old, int src, int ctrl) {
  if (ctrl == 0x138) {  // wave_shr:1: lane l takes lane l-1's value, lane 0 keeps old
    const int v = cpu_wave_exchange(src, cpu_lane() - 1);
    return cpu_lane() == 0 ? old : v;
  }
  if (ctrl == 0x130) {  // wave_shl:1: lane l takes lane l+1's value, lane 63 keeps old
    const int v = cpu_wave_exchange(src, cpu_lane() + 1);
    return cpu_lane() == 63 ? old : v;
  }
  std::abort();  // no other DPP control is used
}

#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) cpu_update_dpp((old), (src), (ctrl))
#define __builtin_amdgcn_readfirstlane(v) cpu_wave_exchange((int)(v), 0)
#define __builtin_amdgcn_ballot_w64(p) cpu_ballot((bool)(p))
#define __builtin_amdgcn_readlane(v, l) cpu_wave_exchange((int)(v), (int)(l))
#define __builtin_amdgcn_s_sleep(n) std::this_thread::yield()
#define __builtin_amdgcn_s_barrier() cpu_block_barrier->arrive_and_wait()
#define __builtin_amdgcn_fence(order, scope) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __builtin_amdgcn_sqrtf(x) std::sqrt((float)(x))
#define __HIP_MEMORY_SCOPE_AGENT 0
#define __HIP_MEMORY_SCOPE_WORKGROUP 1
#define __hip_atomic_load(p, order, scope) __atomic_load_n((p), __ATOMIC_SEQ_CST)
#define __hip_atomic_store(p, v, order, scope) __atomic_store_n((p), (v), __ATOMIC_SEQ_CST)
#define __hip_atomic_fetch_add(p, v, order, scope) __atomic_fetch_add((p), (v), __ATOMIC_SEQ_CST)
#define __threadfence() std::atomic_thread_fence(std::memory_order_seq_cst)
#define __builtin_amdgcn_s_waitcnt(x) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __builtin_amdgcn_wave_barrier() cpu_wave_barrier->arrive_and_wait()
#define __builtin_amdgcn_s_setprio(n) ((void)0)
#define __builtin_amdgcn_sched_barrier(n) ((void)0)

template <class T> inline T __shfl(T v, int src) { return cpu_wave_exchange(v, src); }
template <class T> inline T __shfl_xor(T v, int mask) { return cpu_wave_exchange(v, cpu_lane() ^ mask); }

inline int __double2loint(double d) { uint64_t b; std::memcpy(&b, &d, 8); return (int)(uint32_t)b; }
inline int __double2hiint(double d) { uint64_t b; std::memcpy(&b, &d, 8); return (int)(uint32_t)(b >> 32); }
inline double __hiloint2double(int hi, int lo) {
  const uint64_t b = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
  double d;
  std::memcpy(&d, &b, 8);
  return d;
}
inline int __float_as_int(float f) { int i; std::memcpy(&i, &f, 4); return i; }
inline float __int_as_float(int i) { float f; std::memcpy(&f, &i, 4); return f; }
inline uint64_t wall_clock64() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch()).count() / 10;
}
