// Internal layout shared by the HIP kernels (dtw_kernels.hip) and the host
// runtime (dtw_api.hip).  Everything here lives in the caller's workspace.
//
// Coordinates: a block is a sub-rectangle of one pair's DP grid, stored with
// GLOBAL frame indices into the packed X / Y arrays (i into X, j into Y), so
// the sweep kernels never need to know which pair a block belongs to; only
// path assembly subtracts the pair's frame offsets.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dtw.h"

namespace dtw {

constexpr int kWave = 64;        // gfx950 wavefront width; one lane per DP row
constexpr int kRing = 2;         // boundary rows per sweep (see pass kernel)
constexpr int kBandChunk = 256;  // band cells per split-cost work item
constexpr int kMaxMinBlock = 1024;
constexpr uint32_t kSpinIterCap = 1u << 26;  // polls before a wait gives up

// Sweep and leaf workgroups: one recurrence wave, kProducers frame-cost
// waves and one boundary-input wave; phases of kPhase steps between barriers.
constexpr int kProducers = 8;
constexpr int kLeafThreads = kWave * (kProducers + 2);
// Calls with at most this many pairs run a leaf's stripes on several
// workgroups (latency); larger batches keep one workgroup per leaf, their
// many leaves already filling the GPU (throughput).
constexpr int kLeafSplitPairs = 16;
constexpr int kPhase = 32;
constexpr int kCostRing = 128;  // LDS cost slots, indexed by step
constexpr int kPubGroup = 16;   // steps per bottom-row publication (sweep and leaf)
constexpr int kStepGroup = 4;   // recurrence steps whose operands are read together

// Frame cost forms: the exact Euclidean cost on the VALU (FP64 or FP32), the
// Gram form on the matrix cores (dtw_gram.h) from BF16 or FP16 frames, or the
// cosine cost on the VALU from frames normalised at staging.
constexpr int kCostEuclid = 0;
constexpr int kCostGram = 1;     // BF16 frames
constexpr int kCostGramF16 = 2;  // FP16 frames
constexpr int kCostCosine = 3;   // 1 - dot product of the normalised frames
constexpr int kCostGramCos = 4;     // the Gram form's tile on normalised BF16 frames: 1 - dot
constexpr int kCostGramF16Cos = 5;  // the same on normalised FP16 frames
constexpr bool is_gram(int cm) {
  return cm == kCostGram || cm == kCostGramF16 || cm == kCostGramCos || cm == kCostGramF16Cos;
}
constexpr bool gram_bf16(int cm) { return cm == kCostGram || cm == kCostGramCos; }
constexpr bool is_cos(int cm) { return cm == kCostCosine || cm == kCostGramCos || cm == kCostGramF16Cos; }
// Producer waves of a sweep workgroup: the Gram form needs only two (its
// matrix-core tiles are cheap), which makes its workgroup 4 waves and lets
// four workgroups share a CU; the Euclidean forms use eight.
constexpr int pass_producers(int cm) { return is_gram(cm) ? 2 : kProducers; }
constexpr int pass_threads(int cm) { return kWave * (pass_producers(cm) + 2); }
constexpr bool is_gram_precision(int p) { return p == DTW_PREC_BF16_COST || p == DTW_PREC_FP16_COST; }

struct Block {
  int32_t i0, j0, i1, j1;  // inclusive, global frame indices
  int32_t pair;
  int32_t pad;
  double f0;  // tie-exact mode: accumulated cost of the block's origin in the whole table (NaN: its own cost)
};

struct PairDesc {
  int64_t x_off, y_off;  // first frame of the pair in X / Y
  int64_t M, N;
  int64_t pbase;         // first slot of the pair in the diagonal-indexed path scratch
  int64_t out_off;       // first pair of the pair's path in the caller's path buffer
};

// One half sweep (forward or backward) of one block.
struct PassDesc {
  int32_t i0, j0, i1, j1;
  int32_t Mb, Nb;
  int32_t dir;        // 0: from (i0,j0); 1: on the reversed series, from (i1,j1)
  int32_t kstop;      // last local diagonal of this sweep
  int32_t kf;         // forward stop of the block: band = forward diagonals kf-2..kf
  int32_t n_rows;     // local rows touched: min(Mb-1, kstop) + 1
  int32_t n_stripes;  // ceil(n_rows / 64)
  int32_t L;          // band stride: min(Mb, Nb) >= longest band diagonal
  int32_t raw;        // 1: band written in the sweep's own coordinates (dtw_diag)
  int32_t tie;        // 1: tie-exact forward sweep of the whole block with labels
  double f0;          // tie-exact: value of the origin cell (NaN: its own cost)
  int64_t band_off;   // element offset of the block's 3*L band slots
  int64_t ring_off;   // cell offset of the kRing boundary rows (kRing*Nb cells)
};

struct LeafDesc {
  int32_t i0, j0, i1, j1;  // global frame indices
  int32_t pair;
  int32_t first;           // 1 when the leaf starts at the pair's (0,0)
  int64_t scratch_off;     // word offset in leaf scratch, or -1 when it fits in LDS
  int32_t stripe_off;      // first leaf-stripe ticket of the leaf
  int32_t n_stripes;       // ceil(R / 64) stripes of the shorter side
  int32_t split;           // 1: its stripes run on several workgroups (one ticket each); 0: one workgroup
  int32_t pad;
  int64_t ring_off;        // first cell of its min(n_stripes - 1, kRing) boundary rows in the leaf ring
  double f0;               // tie-exact mode: value of the leaf's origin cell (NaN: its own cost)
};

// Device control block.
struct Ctl {
  int32_t n_sub;        // non-leaf blocks at the current level
  int32_t n_pass;       // 2 * n_sub
  int32_t n_tickets;    // stripes of the current level
  int32_t ticket;       // pass-kernel dequeue counter
  int32_t n_chunks;     // band work items of the current level
  int32_t n_leaf;       // leaves emitted so far
  int32_t levels_run;   // levels that had at least one split
  int32_t error;        // first device-side error code, 0 if none
  int32_t leaf_ticket;  // leaf-kernel dequeue counter
  int32_t max_stripes;  // largest n_stripes of the current level
  int64_t leaf_words;   // leaf scratch words handed out
  int64_t cells;        // cells evaluated by the sweeps
  int64_t leaf_cells;   // cells of the leaf tables
  int32_t leaf_stripes; // leaf-stripe tickets emitted so far
  int32_t pad;
  int64_t leaf_ring_cells;  // leaf-ring cells handed out
};

enum DeviceError : int32_t {
  kErrSubCap = 1,
  kErrLeafCap = 2,
  kErrBandCap = 3,
  kErrRingCap = 4,
  kErrTicketCap = 5,
  kErrLeafScratch = 6,
  kErrNotLeafAtEnd = 7,
  kErrNoPivot = 8,
  kErrSpinTimeout = 9,
  kErrBadPivot = 10,
  kErrBadLeaf = 11,
  kErrBadPass = 12,
  kErrBadCount = 13,
  kErrLeafRing = 14,
};

// Capacities chosen by the host planner (see plan_workspace in dtw_api.hip).
struct Caps {
  int64_t sub;       // blocks per level
  int64_t cand;      // candidates per level (2 * sub, at least n_pairs)
  int64_t leaf;      // leaves over all levels
  int64_t band;      // band slots per level
  int64_t ring;      // boundary-row cells per level
  int64_t ticket;    // stripes per level
  int64_t chunk;     // band work items per level
  int64_t hist;      // histogram bins (max stripes + 1)
  int64_t leaf_words;// global leaf scratch words
  int64_t pslots;    // diagonal-indexed path scratch slots (sum of M+N-1)
  int64_t leaf_tk;   // leaf-stripe tickets over all leaves
  int64_t leaf_ring; // boundary-row cells between the stripes of all leaves
};

// Device pointers carved out of the caller's workspace; passed by value.
struct Work {
  Ctl* ctl;
  const PairDesc* pairs;
  int32_t n_pairs;
  int32_t min_block;
  int32_t d;
  int32_t precision;
  int32_t cost;         // DTW_COST_EUCLIDEAN or DTW_COST_COSINE
  int32_t tie;          // 1: tie-exact splits (FP64)
  int32_t leaf_split;   // 1: a leaf's stripes run on several workgroups (calls with few pairs)
  const void* X;        // compute-type copies (or the caller's arrays); bf16 in the Gram form
  const void* Y;
  const float* Xn;      // Gram form: squared norms of the bf16 frames, FP32
  const float* Yn;
  Block* subs[2];
  uint64_t* piv_key;    // per block of the current level: bits of min split cost
  uint64_t* piv_pos;    // per block: (q << 32) | local row of the argmin
  double* smin;         // per pair: split cost at the top level
  PassDesc* passes;
  int2* tickets;        // (pass, stripe)
  int32_t* pass_rank;   // scratch for the ticket ordering
  int32_t* hist;        // scratch histogram of stripe counts
  int32_t* chunk_sub;   // band work item -> block
  double* bandF;        // forward accumulated cost on the band (S after combine)
  double* bandC;        // frame cost on the band
  double* bandB;        // backward accumulated cost on the band
  uint64_t* ring;       // boundary-row cells of the sweeps (words of value half + writer id)
  uint64_t* lring;      // tie-exact mode: the labels of those cells (label + writer id), one word each
  int32_t ring_words;   // words per ring cell: 2 for FP64 values, 1 for FP32
  LeafDesc* leaves;
  uint32_t* leaf_scratch;
  int2* tpath;          // diagonal-indexed path scratch
  int32_t* cnt;         // cells written by the leaf that ends on this diagonal
  double2* leaf_cost;   // per leaf (hi, lo) compensated sum
  int2* leaf_tk;        // leaf-stripe ticket -> (leaf, stripe)
  uint64_t* leaf_ring;  // boundary rows between the stripes of a leaf (cells as in `ring`)
  int32_t* leaf_done;   // per leaf: stripes whose pointers are complete
  uint64_t spin_ticks;  // bound on one boundary wait, device wall-clock ticks
  Caps caps;
};

// Host-side check of one launch before it is enqueued: the threads per
// workgroup against the kernel's compiled maximum, its static plus dynamic
// LDS against the device's per-workgroup limit and the kernel's dynamic LDS
// limit, its registers against one SIMD's register file, and the grid size.
// hipSuccess, or hipErrorInvalidConfiguration after recording the rejection
// (launch_rejected() then reports it and the entry point returns
// DTW_ERR_INTERNAL instead of enqueueing a launch the device cannot run).
hipError_t check_launch(const void* fn, int grid, int threads, size_t dyn_lds);
bool launch_rejected();
// Record a failed HIP call's code for dtw_last_hip_error() (calling thread).
void note_hip_error(hipError_t e);
// Device wall-clock ticks per millisecond of the current device.
int64_t wall_ticks_per_ms();
// Compute units of the current device.
int device_cus();

}  // namespace dtw
