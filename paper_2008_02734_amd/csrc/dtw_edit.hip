// Weighted edit distance and an optimal alignment in linear device memory:
// the divide and conquer of Sec. 3 carried over to the edit-distance lattice,
// a problem Sec. 6 names as sharing the DTW dynamic-programming structure.
//
// Lattice: nodes (i, j), 0 <= i <= M, 0 <= j <= N.  A DIAG move into (i, j)
// costs 0 when a[i-1] == b[j-1] and `sub` otherwise; UP and LEFT moves cost
// `gap`.  The split of a block is a node row (every path crosses each row):
// with F the least cost from the block's origin to each node of row mid and
// B the least cost from there to the block's end, the smallest column
// minimising F + B is on an optimal path.  Rows follow a fixed dyadic
// partition (block k of level L spans node rows floor(k M / 2^L) ..
// floor((k+1) M / 2^L)), so every level's row geometry is known on the host
// and only the columns travel on the device.
//
// Kernels per call: init; per split level a persistent sweep launch (all
// forward and backward half sweeps of the level, one wave per stripe of 256
// rows, or 128 for M <= 65536) and a split launch (argmin, child blocks); one leaf launch (full
// table of each block of at most 64 rows as backpointer masks, then the
// walk back); two path-assembly launches.  Values are uint32 (every
// distance is below 2^30).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "dtw.h"
#include "dtw_internal.h"

namespace dtw {
namespace edit {

// DP rows per lane in a sweep stripe: 4 (256-row stripes) for tall problems,
// 2 (128-row stripes, twice the stripes and waves) when M <= kSmallM
#ifndef ED_SMALL_M
#define ED_SMALL_M 65536
#endif
constexpr int64_t kSmallM = ED_SMALL_M;

constexpr int kPh = 64;                   // leaf steps per staged letter block
constexpr int kG = 64;                    // sweep steps per group: one staged column per lane
static_assert(kG == kWave, "a group stages one column per lane and publishes one per lane");
constexpr int kFeed = 2 * kG;            // LDS feed slots (by step): the group in use and the next
constexpr uint32_t kBig = 1u << 30;       // above every distance: "no path"
constexpr int kMaxLevels = 40;
constexpr int kTile = 1024;               // path-assembly nodes per workgroup
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;

enum : int32_t { kEdErrSpin = 1, kEdErrBlock = 2, kEdErrMismatch = 3 };

struct Ctl {
  int32_t error;           // first device-side error, 0 if none
  int32_t pad;
  uint64_t dist_leaves;    // sum of the leaves' end values = cost of the returned path
  int64_t dist_split;      // least F + B of the top split (-1 without a split)
  uint64_t sweep_cells;    // cells evaluated by the sweeps
  uint64_t leaf_cells;     // cells of the leaf tables
  int32_t ticket[kMaxLevels];
};

struct Args {
  Ctl* ctl;
  const uint8_t* a;
  const uint8_t* b;
  int64_t M, N;
  uint32_t sub, gap;
  int32_t levels;          // split levels; the leaves are the blocks of level `levels`
  int32_t pad;
  int2* blocks;            // level L: 2^L (j0, j1) pairs from index 2^L - 1
  uint32_t* frow;          // per level: block k's forward row at j0 + k (w + 1 values)
  uint32_t* brow;          // the backward rows, same places
  uint64_t* ring;          // per level: block k's 4 (w + 1) cells at 4 (j0 + k)
  uint32_t* masks;         // leaf k: (w + 64) steps of 4 words at 4 (j0 + 64 k)
  int2* tpath;             // node on each diagonal i + j, (-1, -1) where none
  int32_t* tile_cnt;       // path nodes per assembly tile
  uint64_t spin_ticks;     // bound on one boundary wait, device wall-clock ticks
};

__device__ __forceinline__ uint32_t shr1(uint32_t old, uint32_t v) {
  // lane l takes lane l-1's v; lane 0 keeps `old`
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, kDppWaveShr1, 0xf, 0xf, false);
}

__device__ __forceinline__ uint32_t shl1(uint32_t old, uint32_t v) {
  // lane l takes lane l+1's v; lane 63 keeps `old`
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, kDppWaveShl1, 0xf, 0xf, false);
}

__device__ __forceinline__ int64_t row_at(int64_t k, int64_t M, int L) { return (k * M) >> L; }

__device__ __forceinline__ uint32_t cell_tag(int level, int s) {
  return ((uint32_t)(level + 1) << 24) | (uint32_t)(s + 1);
}

__device__ __forceinline__ void set_err(Ctl* c, int32_t e) {
  int32_t z = 0;
  __hip_atomic_compare_exchange_strong(&c->error, &z, e, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
}

// Poll one ring cell until it carries `tag`; bounded by the wall clock and an
// iteration cap, and ended early once the call's error word is set.
__device__ __forceinline__ uint64_t poll_cell(const uint64_t* p, uint32_t tag, const Args& g) {
  uint64_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((uint32_t)(v >> 32) != tag) {
    const uint64_t t0 = wall_clock64();
    for (uint32_t it = 0;; ++it) {
      __builtin_amdgcn_s_sleep(1);
      const int32_t err = __hip_atomic_load(&g.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((uint32_t)(v >> 32) == tag || err != 0) break;
      if (wall_clock64() - t0 > g.spin_ticks || it > kSpinIterCap) {
        set_err(g.ctl, kEdErrSpin);
        break;
      }
    }
  }
  return v;
}

// ------------------------------------------------------------------ sweeps
//
// One stripe of a half sweep: rows base+1 .. base+64R of the swept table
// (forward: node rows i0+1 .. mid from the origin (i0, j0); backward: the
// reversed block from (i1, j1), its row r holding a[i1 - r]).  Lane l owns
// rows base + Rl + 1 .. base + Rl + R and at step t updates column
// c = t - l + 1 of all R: the top row takes the row above from lane l-1
// (DPP wave_shr:1; lane 0 from the staged row above the stripe), the others
// from the row just updated in the same lane.  The column's letter travels
// down the wave the same way.  Cells left of column 1 hold values of at least
// kBig except the column-0 boundary, which every row reaches exactly.  With
// unit substitution cost the mismatch is added as a carry (5 VALU operations
// per cell instead of 6).
//
// Rows above the stripe come from the previous stripe through ring cells
// (value | writer id << 32), staged one group (64 steps) ahead into LDS.  The
// stripe's last row is collected without branches: each step's value enters
// lane 63 and shifts one lane down (DPP wave_shl:1), so after a group lane i
// holds step 64g + i's, and all lanes store them to the other ring row, or,
// for the last stripe, to the level's F or B row.  (A masked store by the one
// lane holding the last row put a branch into every step and kept the LDS
// reads of later steps from being scheduled early.)
template <int kR, bool kFullOut, bool kUnit>
__device__ void sweep_stripe(const Args& g, int L, int k, int dir, int s, int n_str, int64_t i0, int64_t i1,
                             int h, int j0, int w, uint2* feed) {
  const int lane = threadIdx.x;
  const uint32_t gap = g.gap, sub = g.sub;
  constexpr int kStripeRows = kWave * kR;
  const int base = s * kStripeRows;
  uint32_t x[kR];
#pragma unroll
  for (int q = 0; q < kR; ++q) {
    const int r = base + kR * lane + q + 1;
    x[q] = r <= h ? (uint32_t)(dir ? g.a[i1 - r] : g.a[i0 + r - 1]) : 0u;
  }
  // v: each row's value of the previous step; u0: the row above row 0, one column back
  uint32_t v[kR];
#pragma unroll
  for (int q = 0; q < kR; ++q) v[q] = lane == 0 ? (uint32_t)(base + q + 1) * gap : kBig;
  uint32_t u0 = lane == 0 ? (uint32_t)base * gap : kBig;

  const int64_t region = 4 * ((int64_t)j0 + k);
  const uint64_t* rin = g.ring + region + (int64_t)(2 * dir + ((s + 1) & 1)) * (w + 1);
  uint64_t* rout = g.ring + region + (int64_t)(2 * dir + (s & 1)) * (w + 1);
  const uint32_t tag_in = cell_tag(L, s - 1), tag_out = cell_tag(L, s);
  const uint8_t* bb = g.b + j0;

  // group gi (steps 64 gi .. 64 gi + 63) uses columns 64 gi + 1 .. 64 gi + 64 at
  // lane 0; lane i stages column 64 gi + i + 1 one group ahead
  auto load_feed = [&](int gi, uint64_t& cell, uint32_t& ch) {
    const int c = gi * kG + lane + 1;
    cell = 0;
    ch = 0;
    if (c <= w) {
      ch = dir ? bb[w - c] : bb[c - 1];
      if (s > 0) cell = __hip_atomic_load(rin + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  };
  auto store_feed = [&](int gi, uint64_t cell, uint32_t ch) {
    const int c = gi * kG + lane + 1;
    uint32_t top = kBig;
    if (c <= w) {
      if (s == 0) {
        top = (uint32_t)c * gap;
      } else {
        if ((uint32_t)(cell >> 32) != tag_in) cell = poll_cell(rin + c, tag_in, g);
        top = (uint32_t)cell;
      }
    }
    feed[(gi * kG + lane) & (kFeed - 1)] = make_uint2(top, ch);
  };

  const int hl = min(h - base, kStripeRows);
  const int lo = kFullOut ? kWave - 1 : (hl - 1) / kR;  // the stripe's last row: lane lo, row qo
  const int qo = kFullOut ? kR - 1 : (hl - 1) % kR;
  const int T = w + lo;  // that row reaches column w at step T - 1
  const int n_grp = (T + kG - 1) / kG;
  const bool last = s == n_str - 1;
  uint32_t* orow = (dir ? g.brow : g.frow) + (int64_t)j0 + k;

  uint64_t cell;
  uint32_t ch;
  load_feed(0, cell, ch);
  store_feed(0, cell, ch);
  __builtin_amdgcn_wave_barrier();
  uint32_t ych = 0, acc = 0;
  for (int gi = 0; gi < n_grp; ++gi) {
    const bool more = gi + 1 < n_grp;
    if (more) load_feed(gi + 1, cell, ch);
    const uint2* fb = feed + ((gi * kG) & (kFeed - 1));
#pragma unroll
    for (int i = 0; i < kG; ++i) {
      const uint2 f = fb[i];
      ych = shr1(f.y, ych);
      const uint32_t up0 = shr1(f.x, v[kR - 1]);
      uint32_t up = up0, dg = u0;
#pragma unroll
      for (int q = 0; q < kR; ++q) {
        // unit substitution cost: the mismatch bit is added as a carry
        const uint32_t c = kUnit ? (uint32_t)(x[q] != ych) : (x[q] == ych ? 0u : sub);
        const uint32_t nv = min(min(up, v[q]) + gap, dg + c);
        dg = v[q];
        v[q] = nv;
        up = nv;
      }
      u0 = up0;
      // the last row's value of this step enters at lane 63 and moves one lane
      // down per step: after step t, lane l holds step t - 63 + l's
      uint32_t vo = v[kR - 1];
      if (!kFullOut) {
#pragma unroll
        for (int q = 0; q < kR - 1; ++q) vo = qo == q ? v[q] : vo;
        vo = (uint32_t)__builtin_amdgcn_readlane((int)vo, lo);
      }
      acc = shl1(vo, acc);
    }
    // lane i publishes step 64 gi + i's value: column 64 gi + i - lo + 1
    {
      const int c = gi * kG + lane - lo + 1;
      if (c >= 1 && c <= w) {
        if (last)
          orow[dir ? w - c : c] = acc;
        else
          __hip_atomic_store(rout + c, ((uint64_t)tag_out << 32) | acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (more) store_feed(gi + 1, cell, ch);
    __builtin_amdgcn_wave_barrier();
  }
  if (last && lane == 0) orow[dir ? w : 0] = (uint32_t)h * gap;  // column 0: h gaps
}

// Tickets are (sweep, stripe) in stripe-major order, so the stripe a ticket
// waits for was dequeued earlier by a running workgroup: no ticket waits on
// one that has not started.
template <int kR>
__global__ __launch_bounds__(kWave) void ed_sweep_kernel(Args g, int L, int n_sweeps, int max_str) {
  constexpr int kStripeRows = kWave * kR;
  __shared__ uint2 feed[kFeed];
  const int64_t n_tk = (int64_t)n_sweeps * max_str;
  for (;;) {
    int t = 0;
    if (threadIdx.x == 0) t = __hip_atomic_fetch_add(&g.ctl->ticket[L], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= n_tk) break;
    const int sw = t % n_sweeps, s = t / n_sweeps;
    const int k = sw >> 1, dir = sw & 1;
    const int64_t i0 = row_at(k, g.M, L), i1 = row_at(k + 1, g.M, L), mid = row_at(2 * k + 1, g.M, L + 1);
    const int h = (int)(dir ? i1 - mid : mid - i0);
    const int n_str = (h + kStripeRows - 1) / kStripeRows;
    if (s >= n_str) continue;
    const int2 bj = g.blocks[((1 << L) - 1) + k];
    if (bj.x < 0 || bj.y < bj.x || bj.y > g.N) {
      if (threadIdx.x == 0) set_err(g.ctl, kEdErrBlock);
      continue;
    }
    const bool full = h - s * kStripeRows >= kStripeRows;
    const int j0 = bj.x, w = bj.y - bj.x;
    if (g.sub == 1) {
      if (full)
        sweep_stripe<kR, true, true>(g, L, k, dir, s, n_str, i0, i1, h, j0, w, feed);
      else
        sweep_stripe<kR, false, true>(g, L, k, dir, s, n_str, i0, i1, h, j0, w, feed);
    } else {
      if (full)
        sweep_stripe<kR, true, false>(g, L, k, dir, s, n_str, i0, i1, h, j0, w, feed);
      else
        sweep_stripe<kR, false, false>(g, L, k, dir, s, n_str, i0, i1, h, j0, w, feed);
    }
  }
}

// ------------------------------------------------------------------ split
//
// Block k of level L: the smallest column minimising F + B on row mid, and
// the two child blocks of level L + 1 (both hold the split node).
__global__ __launch_bounds__(256) void ed_split_kernel(Args g, int L) {
  __shared__ uint64_t red[4];
  const int k = blockIdx.x;
  const int2 bj = g.blocks[((1 << L) - 1) + k];
  const bool ok = bj.x >= 0 && bj.y >= bj.x && bj.y <= g.N;
  const int w = ok ? bj.y - bj.x : 0;
  const uint32_t* F = g.frow + (int64_t)bj.x + k;
  const uint32_t* B = g.brow + (int64_t)bj.x + k;
  uint64_t best = ~0ull;
  if (ok)
    for (int c = threadIdx.x; c <= w; c += 256) best = min(best, ((uint64_t)(F[c] + B[c]) << 32) | (uint32_t)c);
  for (int o = 32; o > 0; o >>= 1) best = min(best, (uint64_t)__shfl_xor((unsigned long long)best, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    best = min(min(red[0], red[1]), min(red[2], red[3]));
    const int js = ok ? bj.x + (int)(uint32_t)best : 0;
    int2* nb = g.blocks + ((2 << L) - 1);
    nb[2 * k] = make_int2(ok ? bj.x : 0, js);
    nb[2 * k + 1] = make_int2(js, ok ? bj.y : 0);
    if (!ok) set_err(g.ctl, kEdErrBlock);
    if (L == 0) g.ctl->dist_split = ok ? (int64_t)(best >> 32) : -1;
    // both half sweeps of the block: (i1 - i0) rows of w columns
    const uint64_t rows = (uint64_t)(row_at(k + 1, g.M, L) - row_at(k, g.M, L));
    __hip_atomic_fetch_add(&g.ctl->sweep_cells, rows * (uint64_t)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------------ leaves
//
// Leaf k (at most 64 rows): lane l owns row l + 1 of the block's table from
// its origin; at step t it updates column t - l + 1 and records which move
// reached the cell (DIAG, else UP, else LEFT among the moves giving the
// minimum) as two ballots (UP lanes, LEFT lanes).  Sixteen steps of ballots
// fill one register across the wave and are stored together.  The walk from
// (h, w) back to the origin then reads them through LDS, 64 steps at a time,
// and writes each node to its diagonal's slot.
__global__ __launch_bounds__(kWave) void ed_leaf_kernel(Args g) {
  __shared__ uint32_t ybuf[2 * kPh];
  __shared__ uint4 mbuf[kWave];
  const int lane = threadIdx.x;
  const int L = g.levels;
  const int k = blockIdx.x;
  const int64_t i0 = row_at(k, g.M, L), i1 = row_at(k + 1, g.M, L);
  const int h = (int)(i1 - i0);
  const int2 bj = g.blocks[((1 << L) - 1) + k];
  if (bj.x < 0 || bj.y < bj.x || bj.y > g.N || h > kWave) {
    if (lane == 0) set_err(g.ctl, kEdErrBlock);
    return;
  }
  const int j0 = bj.x, w = bj.y - bj.x;
  const uint32_t gap = g.gap, sub = g.sub;
  uint32_t* msk = g.masks + 4 * ((int64_t)j0 + (int64_t)kWave * k);
  const uint8_t* bb = g.b + j0;

  const uint32_t x = lane < h ? (uint32_t)g.a[i0 + lane] : 0u;
  uint32_t v = lane == 0 ? gap : kBig, u0 = lane == 0 ? 0u : kBig, ych = 0, mreg = 0;
  const int T = h >= 1 ? w + h - 1 : 0;

  auto load_y = [&](int p) -> uint32_t {
    const int c = p * kPh + lane + 1;
    return c <= w ? (uint32_t)bb[c - 1] : 0u;
  };
  if (T > 0) ybuf[lane] = load_y(0);
  __builtin_amdgcn_wave_barrier();
  for (int p = 0; p * kPh < T; ++p) {
    const bool more = (p + 1) * kPh < T;
    const uint32_t ny = more ? load_y(p + 1) : 0u;
    const int tn = min(kPh, T - p * kPh);
    for (int i = 0; i < tn; ++i) {
      const int t = p * kPh + i;
      const uint32_t yf = ybuf[t & (2 * kPh - 1)];
      ych = shr1(yf, ych);
      const uint32_t up = shr1((uint32_t)(t + 1) * gap, v);  // row 0 of the leaf: c gaps
      const uint32_t dgc = u0 + (x == ych ? 0u : sub), upg = up + gap, lfg = v + gap;
      const uint32_t nv = min(dgc, min(upg, lfg));
      const bool notd = nv != dgc;
      const uint64_t mu = __ballot(notd && nv == upg);
      const uint64_t ml = __ballot(notd && nv != upg);
      u0 = up;
      v = nv;
      const int sl = lane - (t & 15) * 4;  // lanes 4 (t % 16) .. + 3 take this step's four words
      mreg = sl == 0 ? (uint32_t)mu : sl == 1 ? (uint32_t)(mu >> 32) : sl == 2 ? (uint32_t)ml
           : sl == 3 ? (uint32_t)(ml >> 32) : mreg;
      if ((t & 15) == 15) msk[4 * (int64_t)(t - 15) + lane] = mreg;
    }
    if (more) ybuf[((p + 1) * kPh + lane) & (2 * kPh - 1)] = ny;
    __builtin_amdgcn_wave_barrier();
  }
  if ((T & 15) != 0 && lane < 4 * (T & 15)) msk[4 * (int64_t)(T & ~15) + lane] = mreg;
  const uint32_t endv = h >= 1 ? (uint32_t)__builtin_amdgcn_readlane((int)v, h - 1) : (uint32_t)w * gap;
  if (lane == 0) {
    __hip_atomic_fetch_add(&g.ctl->dist_leaves, (uint64_t)endv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&g.ctl->leaf_cells, (uint64_t)h * (uint64_t)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __threadfence();  // the masks this wave stored are read back below

  int r = h, c = w, cb = -kWave;
  for (;;) {
    if (lane == 0) g.tpath[(i0 + r) + (j0 + c)] = make_int2((int)(i0 + r), j0 + c);
    if (r == 0 && c == 0) break;
    if (r == 0) {
      --c;
    } else if (c == 0) {
      --r;
    } else {
      const int t = c + r - 2;
      if (t < cb || t >= cb + kWave) {
        cb = max(0, t - (kWave - 1));
        const int st = cb + lane;
        mbuf[lane] = st < T ? *reinterpret_cast<const uint4*>(msk + 4 * (int64_t)st) : make_uint4(0, 0, 0, 0);
        __builtin_amdgcn_wave_barrier();
      }
      const uint4 m = mbuf[t - cb];
      const int bit = r - 1;
      const uint32_t uw = (uint32_t)__builtin_amdgcn_readfirstlane((int)(bit < 32 ? m.x : m.y));
      const uint32_t lw = (uint32_t)__builtin_amdgcn_readfirstlane((int)(bit < 32 ? m.z : m.w));
      if ((uw >> (bit & 31)) & 1u) {
        --r;
      } else if ((lw >> (bit & 31)) & 1u) {
        --c;
      } else {
        --r;
        --c;
      }
    }
  }
}

// ------------------------------------------------------------------ path assembly

__device__ __forceinline__ int block_sum256(int x, int* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void ed_count_kernel(Args g, int64_t n) {
  __shared__ int red[4];
  const int64_t e0 = (int64_t)blockIdx.x * kTile;
  int cnt = 0;
  for (int q = threadIdx.x; q < kTile; q += 256) {
    const int64_t e = e0 + q;
    if (e < n && g.tpath[e].x >= 0) ++cnt;
  }
  cnt = block_sum256(cnt, red);
  if (threadIdx.x == 0) g.tile_cnt[blockIdx.x] = cnt;
}

// Each tile adds the counts of the tiles before it, then places its nodes in
// diagonal order (an exclusive scan over its threads, four nodes each).
__global__ __launch_bounds__(256) void ed_emit_kernel(Args g, int64_t n, int n_tiles, int32_t* path,
                                                      int64_t* path_len, int64_t* dist_out) {
  __shared__ int red[4];
  __shared__ int wsum[4];
  const int tile = blockIdx.x;
  int pre = 0;
  for (int q = threadIdx.x; q < tile; q += 256) pre += g.tile_cnt[q];
  pre = block_sum256(pre, red);
  const int64_t e0 = (int64_t)tile * kTile + 4 * threadIdx.x;
  int2 nd[4];
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    nd[q] = e0 + q < n ? g.tpath[e0 + q] : make_int2(-1, -1);
    cnt += nd[q].x >= 0;
  }
  // inclusive scan of cnt over the workgroup
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = cnt;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int wpre = 0;
  for (int q = 0; q < wv; ++q) wpre += wsum[q];
  int pos = pre + wpre + inc - cnt;
  const bool failed = __hip_atomic_load(&g.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (nd[q].x >= 0) {
      path[2 * (int64_t)pos] = nd[q].x;
      path[2 * (int64_t)pos + 1] = nd[q].y;
      ++pos;
    }
  if (tile == n_tiles - 1 && threadIdx.x == 255) {
    const int64_t total = pos;  // the last thread's end position
    const int64_t dl = (int64_t)g.ctl->dist_leaves;
    int32_t err = __hip_atomic_load(&g.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!err && g.levels > 0 && g.ctl->dist_split != dl) err = kEdErrMismatch;
    if (failed || err) {
      *path_len = 0;
      *dist_out = -(int64_t)(err ? err : kEdErrSpin);
    } else {
      *path_len = total;
      *dist_out = dl;
    }
  }
}

__global__ __launch_bounds__(256) void ed_init_kernel(Args g, int64_t ring_cells, int64_t n_nodes) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ring_cells; e += stride) g.ring[e] = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_nodes; e += stride)
    g.tpath[e] = make_int2(-1, -1);
  if (blockIdx.x == 0) {
    if (threadIdx.x < kMaxLevels) g.ctl->ticket[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
      g.ctl->error = 0;
      g.ctl->dist_leaves = 0;
      g.ctl->dist_split = -1;
      g.ctl->sweep_cells = 0;
      g.ctl->leaf_cells = 0;
      g.blocks[0] = make_int2(0, (int)g.N);
    }
  }
}

// ------------------------------------------------------------------ host side

struct Layout {
  int levels = 0;
  int64_t nb = 1;             // leaves: 2^levels
  int64_t ring_cells = 0, nodes = 0, tiles = 0;
  size_t ctl = 0, blocks = 0, frow = 0, brow = 0, ring = 0, masks = 0, tpath = 0, tile_cnt = 0, total = 0;
};

int split_levels(int64_t M, int leaf_rows) {
  int L = 0;
  while (((M + ((int64_t)1 << L) - 1) >> L) > leaf_rows) ++L;
  return L;
}

Layout layout(int64_t M, int64_t N, int leaf_rows) {
  Layout y;
  y.levels = split_levels(M, leaf_rows);
  y.nb = (int64_t)1 << y.levels;
  y.ring_cells = 4 * (N + y.nb);
  y.nodes = M + N + 1;
  y.tiles = (y.nodes + kTile - 1) / kTile;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  y.ctl = take(sizeof(Ctl));
  y.blocks = take(sizeof(int2) * (size_t)(2 * y.nb));
  y.frow = take(sizeof(uint32_t) * (size_t)(N + y.nb));
  y.brow = take(sizeof(uint32_t) * (size_t)(N + y.nb));
  y.ring = take(sizeof(uint64_t) * (size_t)y.ring_cells);
  y.masks = take(sizeof(uint32_t) * 4 * (size_t)(N + kWave * y.nb + kWave));
  y.tpath = take(sizeof(int2) * (size_t)y.nodes);
  y.tile_cnt = take(sizeof(int32_t) * (size_t)y.tiles);
  y.total = off;
  return y;
}

dtw_status check_sizes(int64_t M, int64_t N, int32_t sub, int32_t gap, int32_t leaf_rows) {
  if (M < 0 || N < 0 || M > (1 << 30) || N > (1 << 30)) return DTW_ERR_INVALID_ARG;
  if (leaf_rows < 2 || leaf_rows > kWave) return DTW_ERR_INVALID_ARG;
  if (sub < 0 || gap < 0 || sub > (1 << 20) || gap > (1 << 20)) return DTW_ERR_INVALID_ARG;
  if ((M + N + 1) * (int64_t)std::max(sub, gap) >= (int64_t)kBig) return DTW_ERR_INVALID_ARG;
  if (split_levels(M, leaf_rows) >= kMaxLevels - 1) return DTW_ERR_INVALID_ARG;
  return DTW_OK;
}

#define ED_TRY(expr)                  \
  do {                                \
    hipError_t e_ = (expr);           \
    if (e_ != hipSuccess) {           \
      note_hip_error(e_);             \
      return DTW_ERR_HIP;             \
    }                                 \
  } while (0)

}  // namespace edit
}  // namespace dtw

using namespace dtw;
using namespace dtw::edit;

extern "C" {

dtw_status dtw_edit_workspace_size(int64_t M, int64_t N, int32_t leaf_rows, size_t* bytes) {
  if (!bytes) return DTW_ERR_INVALID_ARG;
  const dtw_status st = check_sizes(M, N, 0, 0, leaf_rows);
  if (st != DTW_OK) return st;
  *bytes = layout(M, N, leaf_rows).total;
  return DTW_OK;
}

dtw_status dtw_edit_align(const uint8_t* a, int64_t M, const uint8_t* b, int64_t N, int32_t sub, int32_t gap,
                          int32_t leaf_rows, void* workspace, size_t ws_bytes, int64_t* dist_out,
                          int32_t* path_out, int64_t path_cap, int64_t* path_len_out, dtw_edit_stats* stats,
                          void* stream) {
  const dtw_status st = check_sizes(M, N, sub, gap, leaf_rows);
  if (st != DTW_OK) return st;
  if ((M > 0 && !a) || (N > 0 && !b) || !workspace || !dist_out || !path_out || !path_len_out)
    return DTW_ERR_INVALID_ARG;
  if (path_cap < M + N + 1) return DTW_ERR_CAPACITY;
  const Layout y = layout(M, N, leaf_rows);
  if (ws_bytes < y.total) return DTW_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  Args g{};
  g.ctl = (edit::Ctl*)(ws + y.ctl);
  g.a = a;
  g.b = b;
  g.M = M;
  g.N = N;
  g.sub = (uint32_t)sub;
  g.gap = (uint32_t)gap;
  g.levels = y.levels;
  g.blocks = (int2*)(ws + y.blocks);
  g.frow = (uint32_t*)(ws + y.frow);
  g.brow = (uint32_t*)(ws + y.brow);
  g.ring = (uint64_t*)(ws + y.ring);
  g.masks = (uint32_t*)(ws + y.masks);
  g.tpath = (int2*)(ws + y.tpath);
  g.tile_cnt = (int32_t*)(ws + y.tile_cnt);
  g.spin_ticks = (uint64_t)std::max<int64_t>(1, wall_ticks_per_ms()) * 20000;  // 20 s
  const int cus = std::max(1, device_cus());

  // with stats: events around every sweep launch (on `stream`) and around the call
  std::vector<hipEvent_t> ev;
  if (stats) {
    ev.resize(2 * y.levels + 2);
    for (auto& e : ev) ED_TRY(hipEventCreate(&e));
    ED_TRY(hipEventRecord(ev[2 * y.levels], s));
  }
  struct EventGuard {
    std::vector<hipEvent_t>& v;
    ~EventGuard() {
      for (auto e : v)
        if (e) (void)hipEventDestroy(e);
    }
  } guard{ev};
  const int64_t init_work = std::max(y.ring_cells, y.nodes);
  const int init_grid = (int)std::min<int64_t>(4 * cus, std::max<int64_t>(1, (init_work + 255) / 256));
  hipLaunchKernelGGL(ed_init_kernel, dim3(init_grid), dim3(256), 0, s, g, y.ring_cells, y.nodes);
  ED_TRY(hipGetLastError());
  for (int L = 0; L < y.levels; ++L) {
    const int64_t half = (M + ((int64_t)2 << L) - 1) >> (L + 1);  // ceil(M / 2^(L+1)): tallest half sweep
    const int rows = kWave * (M <= kSmallM ? 2 : 4);
    const int max_str = (int)((half + rows - 1) / rows);
    const int n_sweeps = 2 << L;
    const int64_t n_tk = (int64_t)n_sweeps * max_str;
    const int grid = (int)std::min<int64_t>(n_tk, (int64_t)cus * 32);
    if (stats) ED_TRY(hipEventRecord(ev[2 * L], s));
    if (M <= kSmallM)
      hipLaunchKernelGGL(ed_sweep_kernel<2>, dim3(grid), dim3(kWave), 0, s, g, L, n_sweeps, max_str);
    else
      hipLaunchKernelGGL(ed_sweep_kernel<4>, dim3(grid), dim3(kWave), 0, s, g, L, n_sweeps, max_str);
    ED_TRY(hipGetLastError());
    if (stats) ED_TRY(hipEventRecord(ev[2 * L + 1], s));
    hipLaunchKernelGGL(ed_split_kernel, dim3(1 << L), dim3(256), 0, s, g, L);
    ED_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(ed_leaf_kernel, dim3((unsigned)y.nb), dim3(kWave), 0, s, g);
  ED_TRY(hipGetLastError());
  hipLaunchKernelGGL(ed_count_kernel, dim3((unsigned)y.tiles), dim3(256), 0, s, g, y.nodes);
  ED_TRY(hipGetLastError());
  hipLaunchKernelGGL(ed_emit_kernel, dim3((unsigned)y.tiles), dim3(256), 0, s, g, y.nodes, (int)y.tiles, path_out,
                     path_len_out, dist_out);
  ED_TRY(hipGetLastError());
  if (stats) {
    ED_TRY(hipEventRecord(ev[2 * y.levels + 1], s));
    edit::Ctl c{};
    ED_TRY(hipMemcpyAsync(&c, g.ctl, sizeof c, hipMemcpyDeviceToHost, s));
    ED_TRY(hipStreamSynchronize(s));
    double sw = 0;
    for (int L = 0; L < y.levels; ++L) {
      float ms = 0;
      ED_TRY(hipEventElapsedTime(&ms, ev[2 * L], ev[2 * L + 1]));
      sw += ms;
    }
    float tot = 0;
    ED_TRY(hipEventElapsedTime(&tot, ev[2 * y.levels], ev[2 * y.levels + 1]));
    stats->levels = y.levels;
    stats->device_error = c.error != 0 ? c.error : (y.levels > 0 && c.dist_split != (int64_t)c.dist_leaves ? kEdErrMismatch : 0);
    stats->sweep_cells = (int64_t)c.sweep_cells;
    stats->leaf_cells = (int64_t)c.leaf_cells;
    stats->sweep_ms = sw;
    stats->total_ms = tot;
  }
  return DTW_OK;
}

}  // extern "C"
