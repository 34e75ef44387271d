/*
 * dtw.h -- C-ABI of the MI355X (gfx950) linear-memory exact DTW library
 * (libdtw_hip.so).
 *
 * The library computes an optimal dynamic-time-warping alignment between two
 * multivariate series with the divide-and-conquer method of Tralie & Dempsey,
 * "Exact, Parallelizable Dynamic Time Warping Alignment with Linear Memory"
 * (arXiv 2008.02734), Algorithm 2: forward and backward anti-diagonal
 * wavefront sweeps (Algorithm 1, "DiagDTW") to the three central diagonals,
 * the split cost F + B - C on them (Lemma 2), an argmin pivot that lies on an
 * optimal path, recursion on the two sub-rectangles, and a full-table solve
 * with backtrace for blocks whose shorter side is below the cutoff m
 * (Sec. 3.2).  Working memory is O(M + N) plus the leaf tables.
 *
 * Conventions for every entry point:
 *   - X is M x d and Y is N x d, row-major, one frame per row, contiguous, in
 *     device memory.  Element type is given by dtw_dtype.
 *   - The frame cost is the Euclidean distance (Sec. 4.1), or on request the
 *     cosine cost that passage discusses (dtw_opts.cost).
 *   - The warping path (Sec. 2.1) is written as int32 pairs (i, j) from (0,0)
 *     to (M-1, N-1); its length lies in [max(M,N), M+N-1].
 *   - Ownership: the caller owns X, Y, the outputs and the workspace; the
 *     library allocates no device memory in dtw_align / dtw_align_batched /
 *     dtw_diag.  Buffers must stay valid until the stream has completed.
 *   - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).
 *     Calls are stream-ordered and return before the work completes, unless
 *     a host-visible result is requested (stats != NULL or
 *     opts->validate_finite != 0), in which case the call synchronises the
 *     stream before returning.
 *   - Errors: a negative dtw_status.  Argument errors are detected before any
 *     work is enqueued.  No partial output is promised after an error.
 *     DTW_ERR_HIP carries the HIP error code, readable with
 *     dtw_last_hip_error().
 *   - Floating point: in DTW_PREC_FP64 the frame cost is the sum over the
 *     dimensions in index order of fma(e, e, s) with e = x - y, followed by a
 *     correctly rounded square root; every accumulated cost is one rounded
 *     addition of the exact minimum of its three predecessors.
 */
#ifndef DTW_H
#define DTW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DTW_OK = 0,
  DTW_ERR_INVALID_ARG = -1, /* null pointer, size < 1, unsupported combination */
  DTW_ERR_CAPACITY = -2,    /* path capacity below M + N - 1                    */
  DTW_ERR_WORKSPACE = -3,   /* workspace smaller than dtw_workspace_size()      */
  DTW_ERR_NONFINITE = -4,   /* NaN/Inf in X or Y (only with validate_finite)    */
  DTW_ERR_HIP = -5,         /* a HIP runtime call failed                        */
  DTW_ERR_BUSY = -6,        /* serving: result not ready yet                     */
  DTW_ERR_NOT_FOUND = -7,   /* serving: unknown ticket                          */
  DTW_ERR_UNSUPPORTED = -8, /* feature dimension or mode not built              */
  DTW_ERR_INTERNAL = -9     /* device-side consistency check failed             */
} dtw_status;

/* Element type of X and Y. */
typedef enum { DTW_F64 = 0, DTW_F32 = 1 } dtw_dtype;

/* Arithmetic of the sweeps.  The split cost F + B - C, the argmin that picks
 * the pivot, and the reported path cost are FP64 in every mode. */
typedef enum {
  DTW_PREC_FP64 = 0,     /* exact method: frame cost and accumulation in FP64          */
  DTW_PREC_FP32 = 1,     /* frame cost and accumulation in FP32 on the vector ALUs     */
  DTW_PREC_BF16_COST = 2, /* frame cost from a BF16 Gram tile on MFMA, FP32 accumulation */
  DTW_PREC_FP16_COST = 3  /* the same Gram tile from FP16 frames (finer rounding, same rate) */
} dtw_precision;

/* Frame cost C(i,j) (Sec. 4.1): the Euclidean distance the paper uses, or the
 * cosine cost it discusses for chroma-type features, 1 - x.y / (|x| |y|) with
 * a zero frame kept zero, raised to 0 where rounding takes it below.  In
 * DTW_PREC_FP64 the cosine cost is: each frame divided by its norm (the
 * correctly rounded square root of the fma chain of its squares in dimension
 * order; IEEE division), the dot product of the normalised frames as an fma
 * chain in dimension order, then 1 - dot.  In DTW_PREC_FP32 the normalised
 * frames are rounded to FP32 and the dot product is an FP32 fma chain.  In
 * the Gram forms the normalised frames are rounded to FP32 and then to bf16
 * or fp16, and the cost is max(0, 1 - dot) with the dot product from the
 * matrix-core tile (FP32 accumulation). */
typedef enum { DTW_COST_EUCLIDEAN = 0, DTW_COST_COSINE = 1 } dtw_cost;

typedef struct dtw_opts {
  int32_t precision;       /* dtw_precision, default DTW_PREC_FP64                       */
  int32_t min_block;       /* m of Algorithm 2: a block is solved with the full table when
                              its shorter side is below m.  Default 500 (Sec. 3.2);
                              valid range [3, 1024]: below 3 the recursion would not
                              terminate, above 1024 a leaf no longer fits one workgroup */
  int32_t validate_finite; /* nonzero: scan X and Y for NaN/Inf first (synchronises)    */
  int32_t profile;         /* with stats: 1 = time each kernel class with HIP events
                              recorded on `stream` and report the sums in dtw_stats;
                              2 = time the sweep launches only (ms_sweep; fewer events
                              in the stream); 0 = no timing                              */
  int32_t wait_limit_us;   /* bound on one boundary-row wait of a sweep, in microseconds of
                              the device wall clock; 0 = the default of 20 s.  When a wait
                              runs out, the call fails with DTW_ERR_INTERNAL and device
                              error 9, and every other wait of the call ends at once       */
  int32_t cost;            /* dtw_cost, default DTW_COST_EUCLIDEAN; every precision
                              takes either                                               */
  int32_t tie_exact;       /* 1: tie-exact splits (DTW_PREC_FP64 only, else
                              DTW_ERR_UNSUPPORTED; not in the paper, whose split ties are
                              broken arbitrarily, Sec. 3.2).  Each split is read from labels
                              that a forward sweep over the whole block carries, and each
                              block's table starts from its origin's value in the whole
                              table, so the path equals the textbook backtrace (Sec. 2.1,
                              ties DIAG, UP, LEFT) on every input, exact ties included; the
                              sweep of a split covers the whole block in one chain of
                              stripes instead of two half chains.  0: the split of
                              Algorithm 2 (default)                                       */
  int32_t reserved[1];     /* must be zero                                                */
} dtw_opts;

typedef struct dtw_stats {
  double s_min;            /* min of F + B - C at the top split (the optimal cost up to
                              rounding), or the full-table cost when the whole problem is
                              one leaf                                                     */
  double cost_lowp;        /* reduced-precision modes: s_min as the low-precision sweeps
                              see it (their accumulated costs widened to FP64), i.e. the
                              internal optimum before the FP64 re-evaluation of the path;
                              0 in FP64 mode                                              */
  int64_t cells_processed; /* cells evaluated by both half sweeps of every split plus the
                              cells of every leaf table (progress measure of Sec. 3.2)     */
  int64_t path_len;        /* number of (i,j) pairs written                               */
  int64_t workspace_bytes; /* bytes of the workspace this problem needs                  */
  int64_t sweep_cells;     /* cells evaluated by the wavefront sweeps                     */
  int64_t leaf_cells;      /* cells of the leaf tables                                    */
  int32_t levels;          /* split levels executed                                       */
  int32_t leaves;          /* leaf blocks solved with the full table                      */
  int32_t device_error;    /* 0, or a device-side consistency code                        */
  int32_t reserved[3];
  double ms_sweep;         /* with opts->profile: summed GPU time of the sweep launches   */
  double ms_split;         /* split cost + argmin launches                                */
  double ms_plan;          /* recursion planning launches                                 */
  double ms_leaf;          /* leaf solve launches                                         */
  double ms_other;         /* input staging, initialisation and path assembly             */
} dtw_stats;

/* Fill *opts with the defaults (FP64, m = 500, no validation). */
void dtw_default_opts(dtw_opts* opts);

/* Human-readable name of a status code (static string). */
const char* dtw_status_string(int32_t status);

/* HIP error code of the most recent DTW_ERR_HIP on the calling thread. */
int32_t dtw_last_hip_error(void);

/* Workspace bytes needed by dtw_align for an M x N problem of dimension d.
 * opts may be NULL (defaults).  Returns DTW_OK and writes *bytes, or
 * DTW_ERR_INVALID_ARG (M, N < 1, bytes NULL, bad opts) / DTW_ERR_UNSUPPORTED.
 * The size is linear in M + N, as the memory bound of the divide-and-conquer
 * recursion (Sec. 3.2) and the memory comparison of Sec. 4.3 require: the three
 * split-diagonal bands F, B and C of every block of one recursion level
 * (Eq. "splitcost"; about 4.5 (M + N) doubles summed over a level), the
 * boundary rows handed from one wavefront stripe to the next (Algorithm 1),
 * the leaf tables of side < m (two bits per cell: the traceback choice), the path, the
 * block and pass descriptors, and a converted copy of X and Y when the sweep
 * arithmetic, the frame padding or the cosine cost needs one.  Never the
 * M x N table.  The size depends only on M, N, d, in_dtype, opts->precision,
 * opts->min_block and opts->cost. */
dtw_status dtw_workspace_size(int64_t M, int64_t N, int32_t d, int32_t in_dtype,
                              const dtw_opts* opts, size_t* bytes);

/* Optimal warping path and its cost (Algorithm 2 of arXiv 2008.02734).
 *   X, Y        device, M x d and N x d, element type in_dtype
 *   workspace   device, at least dtw_workspace_size() bytes, any contents
 *   cost_out    device, 1 double: FP64 sum of the FP64 frame costs along the path
 *   path_out    device, 2 * path_cap int32: the (i, j) pairs
 *   path_cap    capacity in pairs, must be >= M + N - 1
 *   path_len_out device, 1 int64
 *   stats       host, may be NULL; when set the call synchronises `stream`
 *   stream      hipStream_t or NULL
 * Supported feature dimensions: 1 <= d <= 128 for DTW_PREC_FP64 / FP32 (frames
 * zero-padded to 4, 8, 12, 16, 24, 32, 64 or 128),
 * 1 <= d <= 128 for DTW_PREC_BF16_COST / FP16_COST (frames zero-padded to 32,
 * 64 or 128);
 * other d give DTW_ERR_UNSUPPORTED. */
dtw_status dtw_align(const void* X, int64_t M, const void* Y, int64_t N, int32_t d,
                     int32_t in_dtype, const dtw_opts* opts, void* workspace,
                     size_t ws_bytes, double* cost_out, int32_t* path_out,
                     int64_t path_cap, int64_t* path_len_out, dtw_stats* stats,
                     void* stream);

/* No-allocation form of dtw_align, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as dtw_align, except:
 *   - there is no workspace argument: the library's own fixed device array of
 *     DTW_NOALLOC_SCRATCH_BYTES (one per GPU, held from the library's load
 *     until the process ends) serves as the workspace;
 *   - a problem whose dtw_workspace_size() exceeds DTW_NOALLOC_SCRATCH_BYTES
 *     is rejected with DTW_ERR_WORKSPACE before any work is enqueued (64 MiB
 *     holds, e.g., 20000 x 16000 at d = 12 in FP64, about 10.4 MiB);
 *   - opts->profile must be 0 (DTW_ERR_INVALID_ARG otherwise).
 * The call allocates no device or pinned host memory.  Every call on one GPU
 * shares that GPU's array, and each call re-initialises what it reads there,
 * so successive calls on one stream are independent; calls that overlap in
 * time on one GPU (different streams or host threads) race and give undefined
 * results.  A device-side error shows as a NaN cost and path length 0, and in
 * stats->device_error when stats is given. */
#define DTW_NOALLOC_SCRATCH_BYTES (64u << 20)
dtw_status dtw_align_noalloc(const void* X, int64_t M, const void* Y, int64_t N, int32_t d,
                             int32_t in_dtype, const dtw_opts* opts, double* cost_out,
                             int32_t* path_out, int64_t path_cap, int64_t* path_len_out,
                             dtw_stats* stats, void* stream);

/* DiagDTW (Algorithm 1): one wavefront sweep over the block rows i0..i1,
 * columns j0..j1 of X, Y, stopping at local diagonal kstop
 * (2 <= kstop <= Mb + Nb - 2, Mb = i1-i0+1, Nb = j1-j0+1).
 *   reverse = 0: the sweep starts at (i0, j0); local cell (a, b) = (i0+a, j0+b).
 *   reverse = 1: the sweep runs on the reversed series from (i1, j1); local cell
 *                (a, b) = (i1-a, j1-b).
 *   out (device, 3 * Mb doubles): out[q*Mb + a] = accumulated cost of local cell
 *   (a, kstop-2+q-a), q = 0,1,2, or NaN where that cell is outside the block.
 * X holds at least i1+1 frames and Y at least j1+1.  Uses the same wavefront
 * kernel as dtw_align; needs dtw_workspace_size(i1+1, j1+1, d, in_dtype, opts)
 * bytes of workspace, opts->precision = precision. */
dtw_status dtw_diag(const void* X, const void* Y, int32_t d, int32_t in_dtype,
                    int64_t i0, int64_t j0, int64_t i1, int64_t j1, int32_t reverse,
                    int64_t kstop, int32_t precision, void* workspace, size_t ws_bytes,
                    double* out, void* stream);

/* Replay of repeated calls.  A dtw_align call whose arguments (device,
 * pointers, sizes, options) all equal an earlier call's is recorded once into
 * a HIP graph (recording runs nothing) and from then on replayed with one
 * graph launch on `stream`; the first sighting of a set of arguments runs
 * launch by launch, so one-off calls never pay the recording.  Calls with
 * opts->profile and stats, dtw_align_noalloc, the batched and the serving
 * forms always run launch by launch.  Results are those of the launch-by-
 * launch sequence (the same kernels with the same arguments); the inputs are
 * read when the replay runs.  Up to 16 graphs are kept (least recently used
 * first out); DTW_GRAPHS=0 in the environment turns replay off.
 * dtw_graph_count: graphs currently kept (a diagnostic). */
int32_t dtw_graph_count(void);

/* Device-side consistency code of the latest dtw_align, dtw_align_batched or
 * dtw_diag call that ran in `workspace` (device pointer).  The call's kernels
 * write the code, so it is valid once `stream` has completed that call: this
 * function synchronises `stream`, then reads it into *code (host).
 *   0      no error
 *   9      a boundary-row wait of a sweep ran past opts->wait_limit_us; every
 *          other wait of the call then ends at once
 *   other  a planner, queue or descriptor check failed (1..8, 10..14)
 * A nonzero code also shows in the outputs without this query: the cost is
 * NaN and the path length 0 (dtw_align, dtw_align_batched), every value NaN
 * (dtw_diag).  With stats != NULL, dtw_align / dtw_align_batched report it in
 * stats->device_error and return DTW_ERR_INTERNAL. */
dtw_status dtw_device_error(const void* workspace, int32_t* code, void* stream);

/* Batched form: B independent pairs packed back to back, each solved by
 * Algorithm 2 exactly as dtw_align solves it (the paper aligns one pair per
 * call; batching is this library's, for many short pairs).
 *   x_offsets, y_offsets  host, B+1 frame offsets (pair b uses frames
 *                         x_offsets[b] .. x_offsets[b+1]-1 of X_packed)
 *   path_offsets          host, B+1 pair offsets into paths_out; pair b needs
 *                         capacity >= M_b + N_b - 1
 *   costs_out             device, B doubles; paths_out device int32 pairs;
 *   path_lens_out         device, B int64
 * All pairs share one launch per recursion level.  Results are identical to
 * calling dtw_align on each pair.  Errors: as dtw_align, checked for every
 * pair before any work is enqueued (B < 1, offsets not increasing, a pair's
 * path capacity too small).  Workspace: dtw_workspace_size_batched(), the sum
 * of the per-pair linear terms above (one level's bands, rings and leaf
 * tables over all pairs) plus one copy of the shared descriptors. */
dtw_status dtw_workspace_size_batched(int32_t B, const int64_t* x_offsets,
                                      const int64_t* y_offsets, int32_t d, int32_t in_dtype,
                                      const dtw_opts* opts, size_t* bytes);
dtw_status dtw_align_batched(int32_t B, const void* X_packed, const int64_t* x_offsets,
                             const void* Y_packed, const int64_t* y_offsets, int32_t d,
                             int32_t in_dtype, const dtw_opts* opts, void* workspace,
                             size_t ws_bytes, double* costs_out, int32_t* paths_out,
                             const int64_t* path_offsets, int64_t* path_lens_out,
                             dtw_stats* stats, void* stream);

/* ------------------------------------------------------------------------
 * Serving form (continuous batching; the paper has no serving layer).
 *
 * A server owns one device memory pool, allocated once by dtw_server_create;
 * no other call of the server allocates device memory.  Requests queue in
 * submission order.  A scheduler thread admits requests from the head of the
 * queue into a batch as long as the batch's whole footprint (workspace,
 * packed inputs, packed outputs) fits in free pool memory, the batch holds at
 * most max_batch requests and all of them share precision, d, input type and
 * min_block (the head of the queue first, then later requests of its class
 * in submission order); it then runs the batch as dtw_align_batched would (one launch per
 * recursion level for all of its pairs, the recursion state on the device) on
 * a stream of its own.  Up to max_slots batches are in flight at once, so
 * requests that arrive while others run are admitted as slots and memory free
 * up, and their work overlaps on the device.  Each result is identical to a
 * dtw_align call on the same request.
 *
 * Ownership: the caller owns every request's inputs and outputs (device
 * pointers) and keeps them valid until the request has finished (poll or
 * wait returned DTW_OK for it).  Errors: DTW_ERR_INVALID_ARG for a bad
 * argument, DTW_ERR_WORKSPACE when a request alone cannot fit in the pool,
 * DTW_ERR_UNSUPPORTED for a d the precision does not support,
 * DTW_ERR_NOT_FOUND for an unknown or already collected ticket, DTW_ERR_BUSY
 * from dtw_server_poll while the request is queued or running.  A result
 * whose device-side consistency check failed has status DTW_ERR_INTERNAL. */
typedef struct dtw_server dtw_server;

typedef struct dtw_server_opts {
  size_t pool_bytes;  /* device memory pool, default 8 GiB                      */
  int32_t max_slots;  /* batches in flight at once, 1..16, default 4            */
  int32_t max_batch;  /* requests per batch, >= 1, default 64                   */
  int32_t device;     /* HIP device ordinal, default 0                          */
  int32_t reserved[5];
} dtw_server_opts;

typedef struct dtw_request {
  const void* X;          /* device, M x d                                      */
  int64_t M;
  const void* Y;          /* device, N x d                                      */
  int64_t N;
  int32_t d;
  int32_t in_dtype;       /* dtw_dtype                                          */
  dtw_opts opts;          /* precision and min_block as for dtw_align           */
  double* cost_out;       /* device, 1 double                                   */
  int32_t* path_out;      /* device, 2 * path_cap int32                         */
  int64_t path_cap;       /* >= M + N - 1                                       */
  int64_t* path_len_out;  /* device, 1 int64                                    */
} dtw_request;

typedef struct dtw_result {
  int32_t status;         /* DTW_OK, or the error of the request's batch        */
  int32_t device_error;   /* device-side consistency code of the batch, 0 ok   */
  int32_t batch_size;     /* requests in the batch this request ran in          */
  int32_t reserved;
  int64_t t_submit_ns;    /* host steady-clock times: submission, admission     */
  int64_t t_admit_ns;     /* into a batch, and completion observed by the       */
  int64_t t_done_ns;      /* scheduler                                          */
} dtw_result;

void dtw_server_default_opts(dtw_server_opts* opts);
dtw_status dtw_server_create(const dtw_server_opts* opts, dtw_server** server);
/* Queue one request; returns at once with a ticket. */
dtw_status dtw_server_submit(dtw_server* server, const dtw_request* request, uint64_t* ticket);
/* DTW_ERR_BUSY while the request is queued or running; once it has finished,
 * fills `result`, releases the ticket and returns DTW_OK. */
dtw_status dtw_server_poll(dtw_server* server, uint64_t ticket, dtw_result* result);
/* As dtw_server_poll, but blocks until the request has finished. */
dtw_status dtw_server_wait(dtw_server* server, uint64_t ticket, dtw_result* result);
/* Waits for every submitted request, then releases the pool and the streams. */
dtw_status dtw_server_destroy(dtw_server* server);

/* ------------------------------------------------------------------------
 * Weighted edit distance in linear memory.  Sec. 6 names edit distance as a
 * problem with the DTW dynamic-programming structure that alignment under
 * memory limits would serve; the method of Sec. 3 is carried over to it:
 *   - lattice: nodes (i, j), 0 <= i <= M, 0 <= j <= N, for byte strings a
 *     (length M) and b (length N); a DIAG move into (i, j) costs 0 when
 *     a[i-1] == b[j-1] and `sub` otherwise, UP and LEFT moves cost `gap`;
 *     the distance is the least total cost of a path (0,0) -> (M, N);
 *   - split on a node row (every path crosses it): with F the least cost
 *     from a block's origin to each node of row mid and B the least cost
 *     from there to the block's end, the smallest column minimising F + B
 *     lies on an optimal path (the counterpart of Lemma 2, with nothing to
 *     subtract because the costs sit on the moves);
 *   - rows follow a fixed dyadic partition: block k of level L spans node
 *     rows floor(k M / 2^L) .. floor((k+1) M / 2^L) and splits at
 *     floor((2k+1) M / 2^(L+1)); levels split while ceil(M / 2^L) exceeds
 *     leaf_rows, and the blocks of the first level that does not are solved
 *     with a full table and a backtrace (ties DIAG, then UP, then LEFT).
 * Working memory is O(M + N) (no M x N table).
 *
 * dtw_edit_workspace_size: bytes of device workspace for M x N and
 * leaf_rows.  DTW_ERR_INVALID_ARG for bytes == NULL or sizes outside the
 * limits of dtw_edit_align. */
dtw_status dtw_edit_workspace_size(int64_t M, int64_t N, int32_t leaf_rows, size_t* bytes);

/* Optional host-side measurements of one dtw_edit_align call. */
typedef struct dtw_edit_stats {
  int32_t levels;        /* split levels (sweep launches)                          */
  int32_t device_error;  /* 0, or the device-side code (see dist_out)              */
  int64_t sweep_cells;   /* cells evaluated by the half sweeps of every level      */
  int64_t leaf_cells;    /* cells of the leaf tables                               */
  double sweep_ms;       /* summed duration of the sweep launches (HIP events)     */
  double total_ms;       /* first launch of the call to its last (HIP events)      */
} dtw_edit_stats;

/* Edit distance and an optimal alignment path.
 *   a, b          device, M and N bytes (may be NULL when the length is 0)
 *   sub, gap      move costs, 0 <= sub, gap <= 2^20, and
 *                 (M + N + 1) * max(sub, gap) < 2^30
 *   leaf_rows     2 .. 64: rows of the blocks solved with a full table
 *   workspace     device, at least dtw_edit_workspace_size() bytes, any contents
 *   dist_out      device, 1 int64: the distance, which is also the cost of the
 *                 returned path; a negative value -code after a device-side
 *                 error (1: a boundary wait expired, 2: an inconsistent block,
 *                 3: the path's cost differs from the top split's minimum)
 *   path_out      device, 2 * path_cap int32: the nodes (i, j) from (0, 0) to
 *                 (M, N) in path order
 *   path_cap      capacity in nodes, >= M + N + 1
 *   path_len_out  device, 1 int64: node count (0 after a device-side error)
 *   stats         host, may be NULL; when set, HIP events bracket every sweep
 *                 launch and the call, and the call synchronises `stream`
 *   stream        hipStream_t or NULL
 * 0 <= M, N <= 2^30.  Stream-ordered: returns before the work completes
 * (unless stats is set).
 * The caller owns every buffer; the call allocates no device memory.  Errors
 * before any work is enqueued: DTW_ERR_INVALID_ARG (sizes, costs, leaf_rows,
 * null pointers), DTW_ERR_CAPACITY, DTW_ERR_WORKSPACE; DTW_ERR_HIP when a
 * launch fails.  Calls that share a workspace must not overlap in time. */
dtw_status dtw_edit_align(const uint8_t* a, int64_t M, const uint8_t* b, int64_t N, int32_t sub,
                          int32_t gap, int32_t leaf_rows, void* workspace, size_t ws_bytes,
                          int64_t* dist_out, int32_t* path_out, int64_t path_cap,
                          int64_t* path_len_out, dtw_edit_stats* stats, void* stream);

/* Local alignment score (Smith-Waterman), the other problem Sec. 6 names:
 * the best score over all pairs of substrings, H[0][j] = H[i][0] = 0,
 * H[i][j] = max(0, H[i-1][j-1] + s, H[i-1][j] - gap, H[i][j-1] - gap) with
 * s = +match on equal letters and -mismatch otherwise, and the end of a best
 * local alignment: the first cell holding the maximum in row-major order,
 * (0, 0) when the maximum is 0.  Working memory O(N) (two boundary rows and
 * one record per 256 rows of a).
 *   a, b        device, M and N bytes (may be NULL when the length is 0)
 *   match       1 .. 2^20 and (min(M, N) + 1) * match < 2^30
 *   mismatch, gap  0 .. 2^20 (penalties)
 *   workspace   device, at least dtw_local_workspace_size() bytes, any contents
 *   out         device, 3 int64: score, i_end, j_end (the end cell is the node
 *               after the last aligned letters: a[i_end - 1] and b[j_end - 1]);
 *               a negative score -1 after a boundary wait expired
 *   stream      hipStream_t or NULL; stream-ordered, allocates nothing
 * Errors before any work: DTW_ERR_INVALID_ARG, DTW_ERR_WORKSPACE; DTW_ERR_HIP
 * when a launch fails.  Calls that share a workspace must not overlap.
 * In this build dtw_local_score returns DTW_ERR_UNSUPPORTED after checking its
 * arguments: the device launch is switched off (its first launch did not
 * finish on the device; the cause is not yet found). */
dtw_status dtw_local_workspace_size(int64_t M, int64_t N, size_t* bytes);
dtw_status dtw_local_score(const uint8_t* a, int64_t M, const uint8_t* b, int64_t N, int32_t match,
                           int32_t mismatch, int32_t gap, void* workspace, size_t ws_bytes,
                           int64_t* out, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DTW_H */
