// Command-line driver of the CPU model: reads a problem file, calls the real
// dtw_align / dtw_align_batched host entry points, writes the results.
//   input : int32 B, d, min_block, precision; B x (int64 M, int64 N);
//           X packed (sum M x d float64); Y packed (sum N x d float64)
//   output: int32 status, device_error, levels, leaves; int64 cells;
//           B x (float64 cost, int64 len, len x 2 int32)
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "dtw.h"

#include <atomic>
extern std::atomic<long> cpu_poll_calls;

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[4];
  if (std::fread(hdr, 4, 4, f) != 4) return 2;
  if (hdr[0] == -1) {
    // DiagDTW mode: int64 M, N, i0, j0, i1, j1, reverse, kstop; X; Y ->
    //   int32 status, device error; 3 * (i1 - i0 + 1) float64
    const int d = hdr[1];
    int64_t q[8];
    if (std::fread(q, 8, 8, f) != 8) return 2;
    std::vector<double> X(q[0] * d), Y(q[1] * d);
    if (std::fread(X.data(), 8, X.size(), f) != X.size()) return 2;
    if (std::fread(Y.data(), 8, Y.size(), f) != Y.size()) return 2;
    std::fclose(f);
    dtw_opts o;
    dtw_default_opts(&o);
    o.precision = hdr[3];
    size_t ws = 0;
    int rc = dtw_workspace_size(q[4] + 1, q[5] + 1, d, DTW_F64, &o, &ws);
    std::vector<unsigned char> W(rc == 0 ? ws : 1);
    const int64_t Mb = q[4] - q[2] + 1;
    std::vector<double> out(3 * Mb);
    if (rc == 0)
      rc = dtw_diag(X.data(), Y.data(), d, DTW_F64, q[2], q[3], q[4], q[5], (int32_t)q[6], q[7], o.precision,
                    W.data(), ws, out.data(), nullptr);
    int32_t code = 0;
    if (rc == 0) dtw_device_error(W.data(), &code, nullptr);
    FILE* g = std::fopen(argv[2], "wb");
    int32_t out_hdr[2] = {rc, code};
    std::fwrite(out_hdr, 4, 2, g);
    std::fwrite(out.data(), 8, out.size(), g);
    std::fclose(g);
    std::printf("poll_calls=%ld\n", cpu_poll_calls.load());
    return 0;
  }
  const int B = hdr[0], d = hdr[1];
  std::vector<int64_t> MN(2 * B);
  if (std::fread(MN.data(), 8, 2 * B, f) != (size_t)(2 * B)) return 2;
  std::vector<int64_t> xo(B + 1, 0), yo(B + 1, 0), po(B + 1, 0);
  for (int b = 0; b < B; ++b) {
    xo[b + 1] = xo[b] + MN[2 * b];
    yo[b + 1] = yo[b] + MN[2 * b + 1];
    po[b + 1] = po[b] + MN[2 * b] + MN[2 * b + 1] - 1;
  }
  std::vector<double> X(xo[B] * d), Y(yo[B] * d);
  if (std::fread(X.data(), 8, X.size(), f) != X.size()) return 2;
  if (std::fread(Y.data(), 8, Y.size(), f) != Y.size()) return 2;
  std::fclose(f);
  dtw_opts o;
  dtw_default_opts(&o);
  o.min_block = hdr[2];
  o.precision = hdr[3] & 0xff;
  o.cost = (hdr[3] >> 8) & 0xff;  // the frame cost rides in the precision word's second byte
  o.tie_exact = hdr[3] >> 16;      // and the tie-exact flag in its third
  size_t ws = 0;
  int rc = (B == 1) ? dtw_workspace_size(xo[1], yo[1], d, DTW_F64, &o, &ws)
                    : dtw_workspace_size_batched(B, xo.data(), yo.data(), d, DTW_F64, &o, &ws);
  std::vector<unsigned char> W(rc == 0 ? ws : 1);
  std::vector<double> costs(B);
  std::vector<int32_t> paths(2 * po[B]);
  std::vector<int64_t> lens(B);
  dtw_stats st{};
  if (rc == 0) {
    if (B == 1)
      rc = dtw_align(X.data(), xo[1], Y.data(), yo[1], d, DTW_F64, &o, W.data(), ws, costs.data(), paths.data(),
                     po[1], lens.data(), &st, nullptr);
    else
      rc = dtw_align_batched(B, X.data(), xo.data(), Y.data(), yo.data(), d, DTW_F64, &o, W.data(), ws,
                             costs.data(), paths.data(), po.data(), lens.data(), &st, nullptr);
  }
  FILE* g = std::fopen(argv[2], "wb");
  int32_t out_hdr[4] = {rc, st.device_error, st.levels, st.leaves};
  std::fwrite(out_hdr, 4, 4, g);
  std::fwrite(&st.cells_processed, 8, 1, g);
  for (int b = 0; b < B; ++b) {
    std::fwrite(&costs[b], 8, 1, g);
    std::fwrite(&lens[b], 8, 1, g);
    std::fwrite(paths.data() + 2 * po[b], 4, 2 * (rc == 0 ? lens[b] : 0), g);
  }
  std::fclose(g);
  std::printf("poll_calls=%ld\n", cpu_poll_calls.load());
  return 0;
}
