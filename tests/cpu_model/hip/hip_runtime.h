// Host stand-in for <hip/hip_runtime.h> used by the CPU model of the
// orchestration kernels (tests only).  A "block" runs as blockDim.x OS
// threads sharing one std::barrier; __shared__ becomes a function-static
// object, so blocks of a launch run one after another.
#pragma once
#include <algorithm>
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorInvalidConfiguration = 9, hipErrorInvalidDevice = 101,
       hipErrorInvalidSymbol = 13 };
typedef void* hipStream_t;
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
enum hipDeviceAttribute_t {
  hipDeviceAttributeMultiprocessorCount,
  hipDeviceAttributeMaxSharedMemoryPerBlock,
  hipDeviceAttributeWallClockRate
};
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize };

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(x) alignas(x)

struct dim3_cpu { unsigned int x = 0, y = 1, z = 1; };
extern thread_local dim3_cpu threadIdx, blockIdx, blockDim, gridDim;
extern thread_local std::barrier<>* cpu_block_barrier;
extern thread_local std::barrier<>* cpu_wave_barrier;  // the 64 threads of this thread's wave
inline void __syncthreads() { cpu_block_barrier->arrive_and_wait(); }

struct int2 { int x, y; };
struct uint4 { unsigned x, y, z, w; };
struct alignas(16) int4 { int x, y, z, w; };
inline int4 make_int4(int a, int b, int c, int d) { return int4{a, b, c, d}; }
struct double2 { double x, y; };
inline int2 make_int2(int a, int b) { return int2{a, b}; }
inline double2 make_double2(double a, double b) { return double2{a, b}; }
inline long long __double_as_longlong(double v) { long long r; std::memcpy(&r, &v, 8); return r; }
inline double __longlong_as_double(long long v) { double r; std::memcpy(&r, &v, 8); return r; }

template <class T> inline T min(T a, T b) { return b < a ? b : a; }
template <class T> inline T max(T a, T b) { return a < b ? b : a; }

template <class T> inline T atomicAdd(T* p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
template <class T> inline T atomicOr(T* p, T v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
template <class T> inline T atomicCAS(T* p, T cmp, T v) {
  __atomic_compare_exchange_n(p, &cmp, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return cmp;
}
template <class T> inline T atomicMin(T* p, T v) {
  T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (v < cur && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
  return cur;
}
template <class T> inline T atomicMax(T* p, T v) {
  T cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (cur < v && !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {}
  return cur;
}

inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
// The LDS limit per workgroup can be lowered with CPU_MODEL_LDS_MAX (bytes) so
// that a test can make the host-side launch check refuse a launch.
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  switch (a) {
    case hipDeviceAttributeMultiprocessorCount: *v = 4; break;
    case hipDeviceAttributeMaxSharedMemoryPerBlock: {
      const char* e = std::getenv("CPU_MODEL_LDS_MAX");
      *v = (e && *e) ? std::atoi(e) : 163840;
      break;
    }
    case hipDeviceAttributeWallClockRate: *v = 100000; break;
  }
  return hipSuccess;
}

// Compiled resources of a kernel as the HIP runtime reports them; the model's
// figures come from the harness (cpu_kernel_resources).
struct hipFuncAttributes {
  size_t sharedSizeBytes = 0;
  int maxThreadsPerBlock = 0;
  int maxDynamicSharedSizeBytes = 0;
  int numRegs = 0;
  size_t localSizeBytes = 0;
};
hipError_t hipFuncGetAttributes(hipFuncAttributes* a, const void* fn);
inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(dst, src, n);
  return hipSuccess;
}
inline hipError_t hipMemsetAsync(void* p, int v, size_t n, hipStream_t) { std::memset(p, v, n); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
// A device variable is an ordinary host object here, so its address is itself.
#define HIP_SYMBOL(x) (&(x))
template <class T>
inline hipError_t hipGetSymbolAddress(void** p, T* sym) { *p = (void*)sym; return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
// Graphs: the model records nothing, so a capture never begins and every
// call runs eagerly.
typedef void* hipGraph_t;
typedef void* hipGraphExec_t;
enum { hipStreamNonBlocking = 1, hipStreamCaptureModeThreadLocal = 1, hipErrorNotSupported = 801 };
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = nullptr; return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, int) { return hipErrorNotSupported; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) { *g = nullptr; return hipErrorNotSupported; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, void*, size_t) { return hipErrorNotSupported; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
typedef int* hipEvent_t;
inline hipError_t hipEventCreate(hipEvent_t* e) { static int dummy; *e = &dummy; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }

// The model launches the 1024-thread kernels with fewer threads; they tile
// over blockDim.x, so smaller blocks exercise more tiles.
// Run `body` as a grid of `grid` blocks of `block` threads.
inline void cpu_launch(int grid, int block, const std::function<void()>& body) {
  for (int b = 0; b < grid; ++b) {
    std::barrier<> bar(block);
    const int n_waves = (block + 63) / 64;
    std::vector<std::unique_ptr<std::barrier<>>> wbar;
    for (int v = 0; v < n_waves; ++v) wbar.emplace_back(new std::barrier<>(std::min(64, block - 64 * v)));
    std::vector<std::thread> th;
    th.reserve(block);
    for (int t = 0; t < block; ++t)
      th.emplace_back([&, t, b] {
        threadIdx.x = t; blockIdx.x = b; blockDim.x = block; gridDim.x = grid;
        cpu_block_barrier = &bar;
        cpu_wave_barrier = wbar[t / 64].get();
        body();
      });
    for (auto& x : th) x.join();
  }
}
