// CPU model of the edit-distance kernels (tests only): the real source
// (dtw_edit.hip, kernels and host entry points) compiled for the host
// against the thread-based HIP stand-in, one OS thread per lane; blocks of a
// launch run one after another.
//   input : int64 M, N; int32 sub, gap, leaf_rows, mode; M bytes a; N bytes b
//           (mode 1: the local alignment score, with match, mismatch, gap in
//           place of sub, gap, leaf_rows)
//   output: int32 status, levels; int64 dist, len, sweep cells, leaf cells;
//           len x 2 int32
#include <barrier>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "wave_shim.h"

struct dim3 {
  unsigned x;
  dim3(unsigned a = 1) : x(a) {}
};
#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
  cpu_launch((int)dim3(grid).x, (int)dim3(block).x, [&] { kernel(__VA_ARGS__); })

struct uint2 { unsigned x, y; };
inline uint2 make_uint2(unsigned a, unsigned b) { return uint2{a, b}; }
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return uint4{a, b, c, d}; }
#define __ballot(p) cpu_ballot((bool)(p))
template <class T> inline T __shfl_up(T v, int o) {
  const int l = cpu_lane();
  return cpu_wave_exchange(v, l >= o ? l - o : l);
}
#define __hip_atomic_compare_exchange_strong(p, e, v, o1, o2, scope) \
  __atomic_compare_exchange_n((p), (e), (v), false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)

thread_local dim3_cpu threadIdx, blockIdx, blockDim, gridDim;
thread_local std::barrier<>* cpu_block_barrier = nullptr;
thread_local std::barrier<>* cpu_wave_barrier = nullptr;
uint64_t cpu_wave_slots[16][64];
unsigned char cpu_dynamic_lds[1];

#include "dtw_edit.hip"
#include "dtw_local.hip"

namespace dtw {
int g_model_hip = 0;
void note_hip_error(hipError_t e) { g_model_hip = (int)e; }
int64_t wall_ticks_per_ms() { return 100000; }
int device_cus() { return 2; }
}  // namespace dtw

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t mn[2];
  int32_t p[4];
  if (std::fread(mn, 8, 2, f) != 2 || std::fread(p, 4, 4, f) != 4) return 2;
  const int64_t M = mn[0], N = mn[1];
  std::vector<uint8_t> a(M + 1), b(N + 1);
  if (std::fread(a.data(), 1, M, f) != (size_t)M || std::fread(b.data(), 1, N, f) != (size_t)N) return 2;
  std::fclose(f);
  if (p[3] == 1) {
    // local alignment score: p[0..2] = match, mismatch, gap -> int32 status, int64 score, i_end, j_end
    size_t lws = 0;
    int lrc = dtw_local_workspace_size(M, N, &lws);
    std::vector<unsigned char> LW(lrc == 0 ? lws : 1);
    int64_t out[3] = {0, 0, 0};
    if (lrc == 0)
      lrc = dtw_local_score(M ? a.data() : nullptr, M, N ? b.data() : nullptr, N, p[0], p[1], p[2], LW.data(), lws, out,
                            nullptr);
    FILE* g = std::fopen(argv[2], "wb");
    std::fwrite(&lrc, 4, 1, g);
    std::fwrite(out, 8, 3, g);
    std::fclose(g);
    return 0;
  }
  size_t ws = 0;
  int rc = dtw_edit_workspace_size(M, N, p[2], &ws);
  std::vector<unsigned char> W(rc == 0 ? ws : 1);
  std::vector<int32_t> path(2 * (M + N + 1));
  int64_t dist = 0, len = 0;
  dtw_edit_stats st{};
  if (rc == 0)
    rc = dtw_edit_align(M ? a.data() : nullptr, M, N ? b.data() : nullptr, N, p[0], p[1], p[2], W.data(), ws, &dist,
                        path.data(), M + N + 1, &len, &st, nullptr);
  FILE* g = std::fopen(argv[2], "wb");
  int32_t hdr[2] = {rc, st.levels};
  std::fwrite(hdr, 4, 2, g);
  std::fwrite(&dist, 8, 1, g);
  std::fwrite(&len, 8, 1, g);
  std::fwrite(&st.sweep_cells, 8, 1, g);
  std::fwrite(&st.leaf_cells, 8, 1, g);
  if (rc == 0 && len > 0) std::fwrite(path.data(), 4, 2 * len, g);
  std::fclose(g);
  return 0;
}
