// HIP orchestration kernels for gfx950 (arXiv 2008.02734, Algorithm 2):
//
//   plan_kernel      one level of the recursion: children of the previous
//                    level's pivots, leaf cutoff, sweep descriptors and the
//                    stripe queue;
//   combine_*        split cost S = (F + B) - C on the three central diagonals
//                    (Lemma 2) and the argmin pivot (smallest S, then smallest
//                    diagonal, then smallest row);
//   scan/copy        concatenation of the leaf paths (the pivot is not
//                    repeated) and the FP64 path cost of Eq. 1;
//   init, pad_convert, nonfinite, diag setup/out: bookkeeping.
#include "dtw_common.h"

namespace dtw {

// dtw_diag: the pass kernel runs one sweep in raw mode (band written in the
// sweep's own local coordinates, stride Mb, at q*Mb + (a - lo)); this kernel
// moves the values to q*Mb + a and fills cells outside the block with NaN.
__global__ void diag_out_kernel(Work w, double* out) {
  const PassDesc P = w.passes[0];
  const bool failed = w.ctl->error != 0;  // a device error leaves only NaN
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < 3 * (int64_t)P.Mb;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(u / P.Mb), a = (int)(u % P.Mb);
    const int k = P.kstop - 2 + q;
    const int b = k - a;
    double v = __builtin_nan("");
    if (b >= 0 && b < P.Nb && !failed) {
      const int lo = max(0, k - (P.Nb - 1));
      v = w.bandF[(int64_t)q * P.L + (a - lo)];
    }
    out[u] = v;
  }
}

// ----------------------------------------------------------------- init

__global__ void init_kernel(Work w) {
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nt = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0) {
    Ctl c = {};
    *w.ctl = c;
  }
  // boundary-row cells: writer id 0, which no stripe has
  for (int64_t u = tid; u < w.caps.ring * w.ring_words; u += nt) w.ring[u] = 0ull;
  if (w.lring)
    for (int64_t u = tid; u < w.caps.ring; u += nt) w.lring[u] = 0ull;
  for (int64_t u = tid; u < w.caps.pslots; u += nt) w.cnt[u] = 0;
  for (int64_t u = tid; u < w.caps.leaf_ring * w.ring_words; u += nt) w.leaf_ring[u] = 0ull;
  for (int64_t u = tid; u < w.caps.leaf; u += nt) w.leaf_done[u] = 0;
  for (int64_t u = tid; u < w.n_pairs; u += nt) w.smin[u] = __builtin_nan("");
}

// ----------------------------------------------------------------- plan

// One level of Algorithm 2, run by a single workgroup of 1024 threads.
//  - candidates: the roots (level 0) or both children of every split of the
//    previous level, read from its pivot (both children contain the pivot);
//  - a candidate whose shorter side is below m becomes a leaf;
//  - every other candidate gets a forward sweep to kf = ceil(K/2) and a
//    backward sweep to kb = kf + [K even] (K = Mb + Nb - 1), band slots and
//    a boundary-row ring per sweep, and its stripes enter the level's queue in
//    stripe-major order.
__global__ __launch_bounds__(1024) void plan_kernel(Work w, int level, int final_level,
                                                    int64_t lds_leaf_bytes) {
  __shared__ int64_t tmp[1024];
  __shared__ int32_t s_max_stripes;
  __shared__ int32_t s_rank[1024];
  Ctl* ctl = w.ctl;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n_prev = (level == 0) ? 0 : clamp_count(ctl, ctl->n_sub, w.caps.sub);
  const int64_t n_cand = (level == 0) ? (int64_t)w.n_pairs : 2 * (int64_t)n_prev;
  const Block* prev = w.subs[(level + 1) & 1];
  Block* cur = w.subs[level & 1];
  const int m = w.min_block;

  if (level == 1) {
    for (int s = tid; s < n_prev; s += nt) w.smin[prev[s].pair] = __longlong_as_double((long long)w.piv_key[s]);
  }
  if (tid == 0) s_max_stripes = 0;
  __syncthreads();

  int64_t leaf_base = clamp_count(ctl, ctl->n_leaf, w.caps.leaf), sub_base = 0, words_base = ctl->leaf_words;
  int64_t lstripe_base = ctl->leaf_stripes, lring_base = ctl->leaf_ring_cells;
  for (int64_t tile = 0; tile < n_cand; tile += nt) {
    const int64_t ci = tile + tid;
    const bool valid = ci < n_cand;
    Block c = {0, 0, 0, 0, 0, 0, __builtin_nan("")};
    bool is_leaf = false;
    int64_t words = 0, nst = 0, lcells = 0;
    if (valid) {
      if (level == 0) {
        const PairDesc pd = w.pairs[ci];
        c = Block{(int32_t)pd.x_off, (int32_t)pd.y_off, (int32_t)(pd.x_off + pd.M - 1),
                  (int32_t)(pd.y_off + pd.N - 1), (int32_t)ci, 0, __builtin_nan("")};
      } else {
        const int s = (int)(ci >> 1);
        const Block pb = prev[s];
        const uint64_t pos = w.piv_pos[s];
        const int Mb = pb.i1 - pb.i0 + 1, Nb = pb.j1 - pb.j0 + 1;
        const int K = Mb + Nb - 1, kf = (K + 1) / 2;
        int q = 0, ar = 0;
        if (pos == ~0ull) {
          set_error(ctl, kErrNoPivot);
          ar = max(0, kf - (Nb - 1));
        } else {
          q = (int)(pos >> 32);
          ar = (int)(pos & 0xffffffffu);
        }
        const int k = kf - 2 + q;
        int pi = pb.i0 + ar, pj = pb.j0 + (k - ar);
        bool piv_ok = pos != ~0ull;
        if (q < 0 || q > 2 || pi < pb.i0 || pi > pb.i1 || pj < pb.j0 || pj > pb.j1) {
          // a pivot outside its block would make an empty child
          set_error(ctl, kErrBadPivot);
          pi = pb.i0 + (Mb - 1) / 2;
          pj = pb.j0 + (Nb - 1) / 2;
          piv_ok = false;
        }
        // tie-exact mode: the right child starts from the pivot's value,
        // which the parent's forward sweep left in its band (row q)
        double f_piv = __builtin_nan("");
        if (w.tie && (ci & 1) == 1 && piv_ok) {
          const PassDesc& PP = w.passes[2 * s];
          const int lo = max(0, k - (Nb - 1));
          f_piv = w.bandF[PP.band_off + (int64_t)q * PP.L + ((pi - pb.i0) - lo)];
        }
        c = ((ci & 1) == 0) ? Block{pb.i0, pb.j0, pi, pj, pb.pair, 0, pb.f0}
                            : Block{pi, pj, pb.i1, pb.j1, pb.pair, 0, f_piv};
      }
      const int64_t Mb = c.i1 - c.i0 + 1, Nb = c.j1 - c.j0 + 1;
      is_leaf = (Mb < m) || (Nb < m);
      if (is_leaf) {
        // pointer words by stripe and step (see the leaf kernel).  A leaf of
        // one stripe keeps them in LDS when they fit (with room for a bottom
        // row of the compute type, at most 2 words per column); a leaf of
        // several stripes runs them on several workgroups, so its pointers
        // are in global scratch and its stripes hand their bottom rows over
        // through (n_stripes - 1) rows of the leaf ring.
        const int64_t R = min(Mb, Nb), Cc = max(Mb, Nb);
        const int64_t stripes = (R + kWave - 1) / kWave;
        const bool split = w.leaf_split && stripes > 1;
        nst = split ? stripes : 1;  // tickets of the leaf
        const int64_t bpw = stripes * ((Cc + kWave - 1 + 15) / 16) * kWave;
        const int64_t need = bpw + 2 * Cc;
        if (split || need * 4 > lds_leaf_bytes) words = need;
        lcells = split ? min(stripes - 1, (int64_t)kRing) * Cc : 0;
      }
    }
    int64_t tot_leaf, tot_sub, tot_words;
    const int64_t lrank = block_excl_scan(valid && is_leaf ? 1 : 0, tmp, &tot_leaf);
    const int64_t srank = block_excl_scan(valid && !is_leaf ? 1 : 0, tmp, &tot_sub);
    const int64_t wrank = block_excl_scan(words, tmp, &tot_words);
    int64_t tot_nst, tot_lcells;
    const int64_t strank = block_excl_scan(nst, tmp, &tot_nst);
    const int64_t crank = block_excl_scan(lcells, tmp, &tot_lcells);
    if (valid && is_leaf) {
      const int64_t li = leaf_base + lrank;
      const int64_t so = lstripe_base + strank, ro = lring_base + crank;
      if (li >= w.caps.leaf || so + nst > w.caps.leaf_tk) {
        set_error(ctl, kErrLeafCap);
      } else if (ro + lcells > w.caps.leaf_ring) {
        set_error(ctl, kErrLeafRing);
      } else {
        const PairDesc pd = w.pairs[c.pair];
        LeafDesc L;
        L.i0 = c.i0; L.j0 = c.j0; L.i1 = c.i1; L.j1 = c.j1; L.pair = c.pair;
        L.first = (c.i0 == pd.x_off && c.j0 == pd.y_off) ? 1 : 0;
        L.scratch_off = words ? words_base + wrank : -1;
        L.stripe_off = (int32_t)so;
        L.n_stripes = (int32_t)((min(c.i1 - c.i0, c.j1 - c.j0) + kWave) / kWave);
        L.split = nst > 1 ? 1 : 0;
        L.pad = 0;
        L.ring_off = ro;
        L.f0 = c.f0;
        w.leaves[li] = L;
        // the leaf's tickets: its stripes top to bottom, consecutive, so a
        // stripe only waits on stripes of lower tickets
        for (int u = 0; u < nst; ++u) w.leaf_tk[so + u] = make_int2((int32_t)li, u);
      }
    }
    if (valid && !is_leaf) {
      const int64_t si = sub_base + srank;
      if (si < w.caps.sub) cur[si] = c;
      else set_error(ctl, kErrSubCap);
    }
    leaf_base += tot_leaf;
    sub_base += tot_sub;
    words_base += tot_words;
    lstripe_base += tot_nst;
    lring_base += tot_lcells;
  }
  // cur[] was written by rank, i.e. by other threads than the ones that read
  // it below: every write must be visible before the descriptor loop.
  __syncthreads();
  if (words_base > w.caps.leaf_words && tid == 0) set_error(ctl, kErrLeafScratch);
  const int n_sub = (int)min(sub_base, w.caps.sub);
  if (final_level && n_sub > 0 && tid == 0) set_error(ctl, kErrNotLeafAtEnd);
  const int n_sub_run = final_level ? 0 : n_sub;

  // sweep descriptors, band slots, rings
  int64_t chunk_base = 0, ring_base = 0;
  for (int64_t tile = 0; tile < n_sub_run; tile += nt) {
    const int64_t s = tile + tid;
    const bool valid = s < n_sub_run;
    int64_t nchunk = 0, ring_e = 0;
    Block c = {0, 0, 0, 0, 0, 0, __builtin_nan("")};
    if (valid) {
      c = cur[s];
      const int64_t Mb = c.i1 - c.i0 + 1, Nb = c.j1 - c.j0 + 1;
      const int64_t L = min(Mb, Nb);
      nchunk = (3 * L + kBandChunk - 1) / kBandChunk;
      ring_e = 2 * kRing * Nb;  // forward sweep, then backward sweep
    }
    int64_t tc, tr;
    const int64_t cb = block_excl_scan(nchunk, tmp, &tc);
    const int64_t rb = block_excl_scan(ring_e, tmp, &tr);
    if (valid) {
      const int Mb = c.i1 - c.i0 + 1, Nb = c.j1 - c.j0 + 1;
      const int K = Mb + Nb - 1;
      const int kf = (K + 1) / 2;
      const int kb = kf + ((K % 2) == 0 ? 1 : 0);
      PassDesc P;
      P.raw = 0;
      P.tie = w.tie;
      P.f0 = c.f0;
      P.i0 = c.i0; P.j0 = c.j0; P.i1 = c.i1; P.j1 = c.j1;
      P.Mb = Mb; P.Nb = Nb;
      P.kf = kf;
      P.L = min(Mb, Nb);
      P.band_off = (chunk_base + cb) * kBandChunk;
      P.ring_off = ring_base + rb;
      const bool ok = (P.band_off + nchunk * kBandChunk <= w.caps.band) &&
                      (P.ring_off + ring_e <= w.caps.ring) && (chunk_base + cb + nchunk <= w.caps.chunk);
      if (!ok) set_error(ctl, kErrBandCap);
      const int64_t ring0 = P.ring_off;
      for (int dir = 0; dir < 2; ++dir) {
        P.dir = dir;
        P.ring_off = ring0 + dir * (int64_t)kRing * Nb;
        // tie-exact mode: one forward sweep over the whole block, no backward sweep
        P.kstop = w.tie ? (dir ? 0 : K - 1) : (dir ? kb : kf);
        P.n_rows = min(Mb - 1, P.kstop) + 1;
        P.n_stripes = (ok && !(w.tie && dir)) ? (P.n_rows + kWave - 1) / kWave : 0;
        w.passes[2 * s + dir] = P;
        atomicMax(&s_max_stripes, P.n_stripes);
      }
      if (ok)
        for (int64_t q = 0; q < nchunk; ++q) w.chunk_sub[chunk_base + cb + q] = (int32_t)s;
      w.piv_key[s] = ~0ull;
      w.piv_pos[s] = ~0ull;
      atomicAdd((unsigned long long*)&ctl->cells,
                (unsigned long long)(w.tie ? cells_upto(Mb, Nb, K - 1) : cells_upto(Mb, Nb, kf) + cells_upto(Mb, Nb, kb)));
    }
    chunk_base += tc;
    ring_base += tr;
  }
  __syncthreads();

  // stripe queue in stripe-major order: passes sorted by stripe count
  // (descending); stripe s of the pass at sorted position r gets ticket
  // start(s) + r, start(s) = sum over s' < s of #{passes with > s' stripes}.
  const int n_pass = 2 * n_sub_run;
  const int max_s = s_max_stripes;
  int32_t* hist = w.hist;                   // [0, max_s]: passes with exactly v stripes
  int32_t* gt = w.hist + w.caps.hist;       // #passes with more than v stripes
  int32_t* start = w.hist + 2 * w.caps.hist;
  int32_t* eqc = w.hist + 3 * w.caps.hist;
  const bool hist_ok = max_s < w.caps.hist;
  if (!hist_ok && tid == 0) set_error(ctl, kErrTicketCap);
  if (hist_ok) {
    for (int v = tid; v <= max_s; v += nt) { hist[v] = 0; eqc[v] = 0; }
    __syncthreads();
    for (int p = tid; p < n_pass; p += nt) atomicAdd(&hist[w.passes[p].n_stripes], 1);
    __syncthreads();
    // gt[v] = sum_{u > v} hist[u];  start[s] = sum_{s' < s} gt[s']
    int64_t carry = 0;
    for (int64_t tile = 0; tile <= max_s; tile += nt) {
      const int64_t v = max_s - (tile + tid);  // descending order
      const int64_t hv = (v >= 0) ? hist[v] : 0;
      int64_t tot;
      const int64_t ex = block_excl_scan(hv, tmp, &tot);
      if (v >= 0) gt[v] = (int32_t)(carry + ex);
      carry += tot;
    }
    __syncthreads();
    carry = 0;
    for (int64_t tile = 0; tile <= max_s; tile += nt) {
      const int64_t v = tile + tid;
      const int64_t g = (v <= max_s) ? gt[v] : 0;
      int64_t tot;
      const int64_t ex = block_excl_scan(g, tmp, &tot);
      if (v <= max_s) start[v] = (int32_t)(carry + ex);
      carry += tot;
    }
    const int64_t n_tickets = carry;
    __syncthreads();
    if (n_tickets > w.caps.ticket) {
      if (tid == 0) set_error(ctl, kErrTicketCap);
    } else {
      // Either a pass's stripes are written by one thread, the start offsets
      // read kTicketBatch at a time so that one load latency covers a batch,
      // or (few passes with many stripes, as at the top levels) the passes are
      // taken one after another with the stripes spread over the threads;
      // the choice compares the rounds of dependent loads of the two.
      constexpr int kTicketBatch = 16;
      const int64_t rounds_strided = (int64_t)n_pass * ((max_s + nt - 1) / nt);
      const int64_t rounds_serial = (max_s + kTicketBatch - 1) / kTicketBatch;
      if (n_pass <= (int)(sizeof(s_rank) / sizeof(s_rank[0])) && rounds_strided < rounds_serial) {
        for (int p = tid; p < n_pass; p += nt) {
          const int ns = w.passes[p].n_stripes;
          s_rank[p] = gt[ns] + atomicAdd(&eqc[ns], 1);
        }
        __syncthreads();
        for (int p = 0; p < n_pass; ++p) {
          const int ns = w.passes[p].n_stripes;
          const int r = s_rank[p];
          for (int s = tid; s < ns; s += nt) w.tickets[start[s] + r] = make_int2(p, s);
        }
      } else {
        for (int p = tid; p < n_pass; p += nt) {
          const int ns = w.passes[p].n_stripes;
          const int r = gt[ns] + atomicAdd(&eqc[ns], 1);
          for (int s0 = 0; s0 < ns; s0 += kTicketBatch) {
            int32_t so[kTicketBatch];
#pragma unroll
            for (int k = 0; k < kTicketBatch; ++k) so[k] = (s0 + k < ns) ? start[s0 + k] : 0;
#pragma unroll
            for (int k = 0; k < kTicketBatch; ++k)
              if (s0 + k < ns) w.tickets[so[k] + r] = make_int2(p, s0 + k);
          }
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      ctl->n_sub = n_sub;
      ctl->n_pass = n_pass;
      ctl->n_tickets = (n_tickets > w.caps.ticket) ? 0 : (int32_t)n_tickets;
      ctl->ticket = 0;
      ctl->n_chunks = (int32_t)chunk_base;
      ctl->n_leaf = (int32_t)min(leaf_base, w.caps.leaf);
      ctl->leaf_words = words_base;
      ctl->leaf_stripes = (int32_t)min(lstripe_base, w.caps.leaf_tk);
      ctl->leaf_ring_cells = lring_base;
      if (n_sub_run > 0) ctl->levels_run += 1;
    }
  } else if (tid == 0) {
    ctl->n_sub = 0;
    ctl->n_pass = 0;
    ctl->n_tickets = 0;
    ctl->n_chunks = 0;
    ctl->n_leaf = (int32_t)min(leaf_base, w.caps.leaf);
    ctl->leaf_words = words_base;
    ctl->leaf_stripes = (int32_t)min(lstripe_base, w.caps.leaf_tk);
    ctl->leaf_ring_cells = lring_base;
  }
}

// ----------------------------------------------------------------- split cost

// S = (F + B) - C on every band slot (stored over F), and the smallest S of
// each block as the bits of a non-negative double (monotone as uint64).
__global__ __launch_bounds__(kBandChunk) void combine_min_kernel(Work w) {
  __shared__ uint64_t red[kBandChunk];
  const int n_chunks = clamp_count(w.ctl, w.ctl->n_chunks, w.caps.chunk);
  const int n_sub = clamp_count(w.ctl, w.ctl->n_sub, w.caps.sub);
  for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
    int s = w.chunk_sub[c];
    if (s < 0 || s >= n_sub) {
      if (threadIdx.x == 0) set_error(w.ctl, kErrBadCount);
      s = 0;
    }
    const PassDesc P = w.passes[2 * s];
    const int64_t slot = (int64_t)c * kBandChunk + threadIdx.x - P.band_off;
    uint64_t key = ~0ull;
    if (slot < 3 * (int64_t)P.L) {
      const int q = (int)(slot / P.L), idx = (int)(slot % P.L);
      const int k = P.kf - 2 + q;
      const int lo = max(0, k - (P.Nb - 1)), hi = min(P.Mb - 1, k);
      const int64_t g = P.band_off + slot;
      if (idx <= hi - lo) {
        const double S = (w.bandF[g] + w.bandB[g]) - w.bandC[g];
        w.bandF[g] = S;
        key = (uint64_t)__double_as_longlong(S);
      }
    }
    red[threadIdx.x] = key;
    __syncthreads();
    for (int off = kBandChunk / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + off]);
      __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != ~0ull) atomicMin((unsigned long long*)&w.piv_key[s], (unsigned long long)red[0]);
    __syncthreads();
  }
}

// Among the slots that reach the block's minimum, the smallest (diagonal,
// row), packed as (q << 32) | row with q = diagonal - (kf - 2).
__global__ __launch_bounds__(kBandChunk) void combine_argmin_kernel(Work w) {
  __shared__ uint64_t red[kBandChunk];
  const int n_chunks = clamp_count(w.ctl, w.ctl->n_chunks, w.caps.chunk);
  const int n_sub = clamp_count(w.ctl, w.ctl->n_sub, w.caps.sub);
  for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
    int s = w.chunk_sub[c];
    if (s < 0 || s >= n_sub) {
      if (threadIdx.x == 0) set_error(w.ctl, kErrBadCount);
      s = 0;
    }
    const PassDesc P = w.passes[2 * s];
    const uint64_t target = w.piv_key[s];
    const int64_t slot = (int64_t)c * kBandChunk + threadIdx.x - P.band_off;
    uint64_t key = ~0ull;
    if (slot < 3 * (int64_t)P.L) {
      const int q = (int)(slot / P.L), idx = (int)(slot % P.L);
      const int k = P.kf - 2 + q;
      const int lo = max(0, k - (P.Nb - 1)), hi = min(P.Mb - 1, k);
      const int64_t g = P.band_off + slot;
      if (idx <= hi - lo && (uint64_t)__double_as_longlong(w.bandF[g]) == target)
        key = ((uint64_t)q << 32) | (uint64_t)(lo + idx);
    }
    red[threadIdx.x] = key;
    __syncthreads();
    for (int off = kBandChunk / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + off]);
      __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != ~0ull) atomicMin((unsigned long long*)&w.piv_pos[s], (unsigned long long)red[0]);
    __syncthreads();
  }
}

// ----------------------------------------------------------------- assembly

// Per pair: exclusive scan of the per-diagonal cell counts (segments are in
// path order because their end diagonals increase along the path) and the
// compensated sum of the leaf costs in path order.
__global__ __launch_bounds__(1024) void scan_kernel(Work w, int32_t* poff, int32_t* lidx,
                                                     double* costs_out, int64_t* lens_out) {
  constexpr int kV = 8;
  __shared__ int64_t tmp[1024];
  __shared__ double2 red[1024];
  __shared__ int32_t tile[kV * 1024];  // one chunk, for coalesced loads and stores
  const int p = blockIdx.x;
  const PairDesc pd = w.pairs[p];
  const int64_t n = pd.M + pd.N - 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  // chunks of nt * kV diagonals, read and written coalesced through an LDS
  // tile; for the scan a thread owns kV consecutive diagonals of the tile,
  // and the block scan carries from chunk to chunk
  double2 acc = make_double2(0.0, 0.0);
  const int n_leaf = clamp_count(w.ctl, w.ctl->n_leaf, w.caps.leaf);
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += (int64_t)nt * kV) {
#pragma unroll
    for (int i = 0; i < kV; ++i) {
      const int64_t e = base + (int64_t)i * nt + tid;
      const int c = (e < n) ? w.cnt[pd.pbase + e] : 0;
      tile[i * nt + tid] = c;
      if (c > 0) {
        const int l = lidx[pd.pbase + e];
        if (l >= 0 && l < n_leaf) acc = dd_add(acc, w.leaf_cost[l]);
      }
    }
    __syncthreads();
    int c[kV];
    int64_t local = 0;
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      c[k] = tile[tid * kV + k];
      local += c[k];
    }
    int64_t tot;
    int64_t run = carry + block_excl_scan(local, tmp, &tot);  // its barriers end every read above
#pragma unroll
    for (int k = 0; k < kV; ++k) {
      tile[tid * kV + k] = (int32_t)run;
      run += c[k];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kV; ++i) {
      const int64_t e = base + (int64_t)i * nt + tid;
      if (e < n) poff[pd.pbase + e] = tile[i * nt + tid];
    }
    carry += tot;
  }
  const int64_t total = carry;
  red[tid] = acc;
  __syncthreads();
  for (int off = nt / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] = dd_add(red[tid], red[tid + off]);
    __syncthreads();
  }
  if (tid == 0) {
    // after a device error the outputs are not an alignment: NaN cost, empty path
    const bool failed = w.ctl->error != 0;
    costs_out[p] = failed ? __builtin_nan("") : red[0].x + red[0].y;
    lens_out[p] = failed ? 0 : total;
  }
}

__global__ __launch_bounds__(256) void copy_kernel(Work w, const int32_t* poff, int32_t* paths_out) {
  if (w.ctl->error != 0) return;  // the path length is 0 after a device error
  const int n_leaf = clamp_count(w.ctl, w.ctl->n_leaf, w.caps.leaf);
  for (int l = blockIdx.x; l < n_leaf; l += gridDim.x) {
    const LeafDesc Lf = w.leaves[l];
    if (Lf.pair < 0 || Lf.pair >= w.n_pairs) continue;
    const PairDesc pd = w.pairs[Lf.pair];
    const int64_t e = (int64_t)(Lf.i1 - pd.x_off) + (Lf.j1 - pd.y_off);
    if (e < 0 || e >= pd.M + pd.N - 1) continue;
    const int64_t slot_end = pd.pbase + e;
    int c = w.cnt[slot_end];
    if (c < 0 || c > e + 1 || poff[slot_end] + (int64_t)c > pd.M + pd.N - 1) c = 0;
    const int64_t o = pd.out_off + poff[slot_end];
    int2* out = reinterpret_cast<int2*>(paths_out);
    for (int q = threadIdx.x; q < c; q += blockDim.x) out[o + q] = w.tpath[slot_end - c + 1 + q];
  }
}

// leaf index by end diagonal, for the cost sum in path order
__global__ void leaf_index_kernel(Work w, int32_t* lidx) {
  const int n_leaf = clamp_count(w.ctl, w.ctl->n_leaf, w.caps.leaf);
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < n_leaf; l += gridDim.x * blockDim.x) {
    const LeafDesc Lf = w.leaves[l];
    if (Lf.pair < 0 || Lf.pair >= w.n_pairs) continue;
    const PairDesc pd = w.pairs[Lf.pair];
    const int64_t e = (int64_t)(Lf.i1 - pd.x_off) + (Lf.j1 - pd.y_off);
    if (e >= 0 && e < pd.M + pd.N - 1) lidx[pd.pbase + e] = l;
  }
}

// ----------------------------------------------------------------- misc

// Compute-type copy with frames zero-padded from d to D dimensions.
template <typename TO, typename TI>
__global__ void pad_convert_kernel(const TI* in, TO* out, int64_t rows, int d, int D) {
  const int64_t n = rows * D;
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = u / D;
    const int k = (int)(u % D);
    out[u] = (k < d) ? (TO)in[r * d + k] : (TO)0;
  }
}

// Normalised compute-type copy for the cosine cost (Sec. 4.1), one frame per
// thread, in FP64: each frame divided by its norm, the correctly rounded
// square root of the fma chain of its squares in dimension order (IEEE
// division; a zero frame stays zero), zero-padded from d to D dimensions.
template <typename TO, typename TI>
__global__ void normalize_kernel(const TI* in, TO* out, int64_t rows, int d, int D) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
    const TI* x = in + r * d;
    double n = 0.0;
    for (int t = 0; t < d; ++t) n = __builtin_fma((double)x[t], (double)x[t], n);
    n = __builtin_sqrt(n);
    TO* o = out + r * D;
    for (int t = 0; t < D; ++t) o[t] = (t < d && n > 0.0) ? (TO)((double)x[t] / n) : (TO)0;
  }
}

template <typename TI>
__global__ void nonfinite_kernel(const TI* in, int64_t n, int32_t* flag) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
    if (!__builtin_isfinite((double)in[u])) atomicOr(flag, 1);
}

// Input staging of the Gram form: each frame rounded to bf16 or fp16 (round
// to nearest even; FP64 inputs are first rounded to FP32), zero-padded to D
// dimensions, and its squared norm from the rounded values in FP32.  One wave
// per frame: lane l holds dimensions l and l + 64; the norm is reduced over
// the wave in a fixed order.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)0x7fc0u;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// IEEE binary16 with round to nearest even, subnormals included (written out
// in integer arithmetic so that it does not depend on the float mode).
__device__ __forceinline__ uint16_t f32_to_f16_rne(float f) {
  const uint32_t u = __builtin_bit_cast(uint32_t, f);
  const uint32_t sign = (u >> 16) & 0x8000u;
  const uint32_t a = u & 0x7fffffffu;
  if (a > 0x7f800000u) return (uint16_t)(sign | 0x7e00u);  // NaN
  if (a >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u); // at or past the rounding point of 65504: infinity
  if (a >= 0x38800000u) {                                   // normal: |f| >= 2^-14
    uint32_t h = (a - 0x38000000u) >> 13;                   // exponent rebiased by 112, 10 mantissa bits
    const uint32_t rem = a & 0x1fffu;
    h += (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ? 1u : 0u;
    return (uint16_t)(sign | h);
  }
  if (a < 0x33000000u) return (uint16_t)sign;               // below 2^-25: zero
  const uint32_t e = a >> 23;                               // 102 .. 112
  const uint32_t m = (a & 0x7fffffu) | 0x800000u;
  const uint32_t shift = 126u - e;                          // units of 2^-24
  uint32_t h = m >> shift;
  const uint32_t rem = m & ((1u << shift) - 1u), halfway = 1u << (shift - 1u);
  h += (rem > halfway || (rem == halfway && (h & 1u))) ? 1u : 0u;
  return (uint16_t)(sign | h);
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) {
  const uint32_t sign = (uint32_t)(h & 0x8000u) << 16;
  const uint32_t e = (h >> 10) & 0x1fu, m = h & 0x3ffu;
  if (e == 0) return __builtin_bit_cast(float, sign | __builtin_bit_cast(uint32_t, (float)m * 0x1p-24f));
  if (e == 31) return __builtin_bit_cast(float, sign | 0x7f800000u | (m << 13));
  return __builtin_bit_cast(float, sign | ((e + 112u) << 23) | (m << 13));
}

template <typename TI, bool kBf16, bool kCos>
__global__ __launch_bounds__(256) void gram_stage_kernel(const TI* __restrict__ in, int64_t rows, int d, int D,
                                                          uint16_t* __restrict__ out, float* __restrict__ norms) {
  const int lane = threadIdx.x % 64;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; r < rows; r += nw) {
    // kCos: the frame is first divided by its FP64 norm exactly as the
    // normalising copy of the VALU forms does it (every lane forms the same
    // fma chain in dimension order), then rounded like any other frame
    double n = 1.0;
    if constexpr (kCos) {
      n = 0.0;
      for (int t = 0; t < d; ++t) n = __builtin_fma((double)in[r * d + t], (double)in[r * d + t], n);
      n = __builtin_sqrt(n);
    }
    float s = 0.0f;
    for (int k = lane; k < D; k += 64) {
      float f;
      if constexpr (kCos) f = (k < d && n > 0.0) ? (float)((double)in[r * d + k] / n) : 0.0f;
      else f = (k < d) ? (float)in[r * d + k] : 0.0f;
      const uint16_t h = kBf16 ? f32_to_bf16_rne(f) : f32_to_f16_rne(f);
      out[r * D + k] = h;
      const float g = kBf16 ? bf16_to_f32(h) : f16_to_f32(h);
      s = __builtin_fmaf(g, g, s);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) norms[r] = s;
  }
}

// The pair descriptor of a one-pair call, taken by value: a launch instead
// of a host-to-device copy, so that the call's sequence reads no host memory
// and can be replayed from a graph.
__global__ void store_pair_kernel(PairDesc* dst, PairDesc v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}

__global__ void diag_setup_kernel(Work w, int32_t i0, int32_t j0, int32_t i1, int32_t j1, int32_t dir,
                                  int32_t kstop) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Ctl c = {};
  PassDesc P;
  P.i0 = i0; P.j0 = j0; P.i1 = i1; P.j1 = j1;
  P.Mb = i1 - i0 + 1; P.Nb = j1 - j0 + 1;
  P.dir = dir;
  P.kstop = kstop;
  P.kf = kstop;
  P.raw = 1;
  P.tie = 0;
  P.f0 = __builtin_nan("");
  P.n_rows = min(P.Mb - 1, kstop) + 1;
  P.n_stripes = (P.n_rows + kWave - 1) / kWave;
  P.L = P.Mb;
  P.band_off = 0;
  P.ring_off = 0;
  w.passes[0] = P;
  for (int s = 0; s < P.n_stripes; ++s) w.tickets[s] = make_int2(0, s);
  c.n_tickets = P.n_stripes;
  c.n_pass = 1;
  *w.ctl = c;
}

// ----------------------------------------------------------------- launchers
}  // namespace dtw

#include "dtw_launch.h"

namespace dtw {

hipError_t launch_pass(const Work& w, int level, int grid, hipStream_t st);

hipError_t launch_store_pair(PairDesc* dst, const PairDesc& v, hipStream_t st) {
  return launch_checked(&store_pair_kernel, 1, 64, 0, st, dst, v);
}
hipError_t launch_init(const Work& w, hipStream_t st) {
  return launch_checked(&init_kernel, 256, 256, 0, st, w);
}
hipError_t launch_plan(const Work& w, int level, int final_level, int64_t lds_leaf_bytes, hipStream_t st) {
  return launch_checked(&plan_kernel, 1, 1024, 0, st, w, level, final_level, lds_leaf_bytes);
}
hipError_t launch_combine(const Work& w, int grid, hipStream_t st) {
  const hipError_t e = launch_checked(&combine_min_kernel, grid, kBandChunk, 0, st, w);
  if (e != hipSuccess) return e;
  return launch_checked(&combine_argmin_kernel, grid, kBandChunk, 0, st, w);
}
hipError_t launch_assemble(const Work& w, int32_t* poff, int32_t* lidx, double* costs, int64_t* lens,
                           int32_t* paths, int grid, hipStream_t st) {
  hipError_t e = launch_checked(&leaf_index_kernel, 64, 256, 0, st, w, lidx);
  if (e == hipSuccess) e = launch_checked(&scan_kernel, w.n_pairs, 1024, 0, st, w, poff, lidx, costs, lens);
  if (e == hipSuccess) e = launch_checked(&copy_kernel, grid, 256, 0, st, w, static_cast<const int32_t*>(poff), paths);
  return e;
}
hipError_t launch_pad_convert(const void* in, int in_f64, void* out, int out_f64, int64_t rows, int d, int D,
                              hipStream_t st) {
  const int64_t n = rows * D;
  const int grid = (int)min((int64_t)2048, (n + 255) / 256 + 1);
  if (in_f64 && out_f64)
    return launch_checked(&pad_convert_kernel<double, double>, grid, 256, 0, st, static_cast<const double*>(in),
                          static_cast<double*>(out), rows, d, D);
  if (in_f64)
    return launch_checked(&pad_convert_kernel<float, double>, grid, 256, 0, st, static_cast<const double*>(in),
                          static_cast<float*>(out), rows, d, D);
  if (out_f64)
    return launch_checked(&pad_convert_kernel<double, float>, grid, 256, 0, st, static_cast<const float*>(in),
                          static_cast<double*>(out), rows, d, D);
  return launch_checked(&pad_convert_kernel<float, float>, grid, 256, 0, st, static_cast<const float*>(in),
                        static_cast<float*>(out), rows, d, D);
}
hipError_t launch_normalize(const void* in, int in_f64, void* out, int out_f64, int64_t rows, int d, int D,
                            hipStream_t st) {
  const int grid = (int)min((int64_t)2048, (rows + 255) / 256 + 1);
  if (in_f64 && out_f64)
    return launch_checked(&normalize_kernel<double, double>, grid, 256, 0, st, static_cast<const double*>(in),
                          static_cast<double*>(out), rows, d, D);
  if (in_f64)
    return launch_checked(&normalize_kernel<float, double>, grid, 256, 0, st, static_cast<const double*>(in),
                          static_cast<float*>(out), rows, d, D);
  if (out_f64)
    return launch_checked(&normalize_kernel<double, float>, grid, 256, 0, st, static_cast<const float*>(in),
                          static_cast<double*>(out), rows, d, D);
  return launch_checked(&normalize_kernel<float, float>, grid, 256, 0, st, static_cast<const float*>(in),
                        static_cast<float*>(out), rows, d, D);
}
template <bool kCos>
hipError_t launch_gram_stage_t(const void* in, int in_f64, int64_t rows, int d, int D, int bf16, uint16_t* out,
                               float* norms, hipStream_t st) {
  const int grid = (int)min((int64_t)2048, (rows + 3) / 4 + 1);
  const double* id = static_cast<const double*>(in);
  const float* is = static_cast<const float*>(in);
  if (in_f64 && bf16)
    return launch_checked(&gram_stage_kernel<double, true, kCos>, grid, 256, 0, st, id, rows, d, D, out, norms);
  if (bf16) return launch_checked(&gram_stage_kernel<float, true, kCos>, grid, 256, 0, st, is, rows, d, D, out, norms);
  if (in_f64)
    return launch_checked(&gram_stage_kernel<double, false, kCos>, grid, 256, 0, st, id, rows, d, D, out, norms);
  return launch_checked(&gram_stage_kernel<float, false, kCos>, grid, 256, 0, st, is, rows, d, D, out, norms);
}
hipError_t launch_gram_stage(const void* in, int in_f64, int64_t rows, int d, int D, int bf16, int cos,
                             uint16_t* out, float* norms, hipStream_t st) {
  return cos ? launch_gram_stage_t<true>(in, in_f64, rows, d, D, bf16, out, norms, st)
             : launch_gram_stage_t<false>(in, in_f64, rows, d, D, bf16, out, norms, st);
}
hipError_t launch_nonfinite(const void* in, int in_f64, int64_t n, int32_t* flag, hipStream_t st) {
  const int grid = (int)min((int64_t)1024, (n + 255) / 256 + 1);
  if (in_f64) return launch_checked(&nonfinite_kernel<double>, grid, 256, 0, st, static_cast<const double*>(in), n, flag);
  return launch_checked(&nonfinite_kernel<float>, grid, 256, 0, st, static_cast<const float*>(in), n, flag);
}
hipError_t launch_diag(const Work& w, int32_t i0, int32_t j0, int32_t i1, int32_t j1, int32_t dir,
                       int32_t kstop, int grid, double* out, hipStream_t st) {
  hipError_t e = launch_checked(&init_kernel, 256, 256, 0, st, w);
  if (e == hipSuccess) e = launch_checked(&diag_setup_kernel, 1, 1, 0, st, w, i0, j0, i1, j1, dir, kstop);
  if (e == hipSuccess) e = launch_pass(w, 0, grid, st);
  if (e == hipSuccess) e = launch_checked(&diag_out_kernel, 64, 256, 0, st, w, out);
  return e;
}

}  // namespace dtw
