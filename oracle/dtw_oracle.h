/*
 * CPU oracle for exact dynamic time warping (test infrastructure only).
 *
 * This library is the checker, not the product: only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It is
 * plain, single-threaded, FP64 C with no blocking or fusion, written from the
 * definitions in Tralie & Dempsey, "Exact, Parallelizable Dynamic Time
 * Warping Alignment with Linear Memory" (arXiv 2008.02734):
 *
 *   - frame cost C(i,j): Euclidean distance between frame i of X and frame j
 *     of Y (Sec. 4.1, "Features": Euclidean chosen over cosine), or on
 *     request the cosine cost that passage discusses;
 *   - warping path: starts at (0,0), ends at (M-1,N-1), steps (0,1),(1,0),
 *     (1,1) (Sec. 2.1);
 *   - textbook table: boundary equation (prefix sums along row 0 and column
 *     0) and the LEFT/UP/DIAG recurrence (Sec. 2.1, Eqs. 2-3), backpointers
 *     and backtrace (Sec. 2.1, last paragraph);
 *   - DiagDTW: anti-diagonal sweep with three diagonal buffers that stops at
 *     a given diagonal (Sec. 3.1, Algorithm 1);
 *   - linmdtw: the divide-and-conquer recursion (Sec. 3.2, Algorithm 2,
 *     Lemmas 1-2, the four-step pivot selection, the cutoff of Sec. 3.2's
 *     last paragraph).
 *
 * Conventions (shared with nothing else; restated here so a reader can check
 * them against the paper):
 *   - X is M x d, Y is N x d, row-major FP64, frame-major.
 *   - C(i,j) = sqrt(s) with s accumulated as s <- fma(e,e,s), e = X[i,t]-Y[j,t],
 *     t = 0..d-1, s starting at +0; sqrt is the IEEE correctly rounded one.
 *   - Tie-break of the backpointers: DIAG, then UP, then LEFT, where
 *     UP = (i-1,j) and LEFT = (i,j-1) as labelled in the recurrence.
 *   - Paths are written as int32 pairs (i,j), from (0,0) to (M-1,N-1).
 *
 * Return values: 0 on success, -1 on invalid arguments, -2 when an output
 * capacity is too small, -3 when memory cannot be allocated.
 */
#ifndef DTW_ORACLE_H
#define DTW_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Frame cost kinds (Sec. 4.1): the Euclidean distance the paper uses, and
 * the cosine cost it discusses for chroma-type features (1 - cos of the
 * angle between the frames; each frame divided by its norm, a zero frame
 * kept zero; dot product of the normalised frames as an fma chain in
 * dimension order; negative rounding results raised to 0). */
enum { DTWO_COST_EUCLIDEAN = 0, DTWO_COST_COSINE = 1 };

/* Select the frame cost of every later call (default Euclidean); -1 for an
 * unknown kind.  Process-wide state: the oracle is single-threaded. */
int dtwo_set_cost(int32_t kind);

/* C(i,j) for one pair of frames under the selected cost. */
double dtwo_frame_cost(const double* x, const double* y, int32_t d);

/* Textbook DTW on the whole M x N grid (Sec. 2.1).
 * cost      : out, D(M-1,N-1) = accumulated cost of the optimal path.
 * path      : out, path_cap pairs (i,j); path_cap >= M+N-1 is always enough.
 * path_len  : out, number of pairs written.
 * F         : optional out (may be NULL), the full M x N accumulated table. */
int dtwo_full(const double* X, int64_t M, const double* Y, int64_t N, int32_t d,
              double* cost, int32_t* path, int64_t path_cap, int64_t* path_len,
              double* F);

/* The references of Sec. 4.2 (numerical precision and tie breaking):
 * dtwo_full_f32        textbook DTW entirely in binary32 (frames rounded to
 *                      float, fmaf/sqrtf frame cost, float accumulation),
 *                      backpointers DIAG, UP, LEFT; *cost is the float
 *                      optimum widened to double;
 * dtwo_full_left_first textbook DTW in FP64 with the reversed tie rule:
 *                      LEFT, then UP, then DIAG.
 * Arguments and return values as for dtwo_full (no table output). */
int dtwo_full_f32(const double* X, int64_t M, const double* Y, int64_t N, int32_t d,
                  double* cost, int32_t* path, int64_t path_cap, int64_t* path_len);
int dtwo_full_left_first(const double* X, int64_t M, const double* Y, int64_t N, int32_t d,
                         double* cost, int32_t* path, int64_t path_cap, int64_t* path_len);

/* DiagDTW (Algorithm 1) on the block of rows i0..i1 and columns j0..j1.
 * reverse = 0: the sweep starts at (i0,j0); local cell (a,b) is (i0+a, j0+b).
 * reverse = 1: the sweep starts at (i1,j1); local cell (a,b) is (i1-a, j1-b),
 *              i.e. the block of the reversed series X_R, Y_R.
 * The sweep covers local diagonals 0..kstop and returns diagonals
 * kstop-2, kstop-1, kstop in out[0..3*Mb): out[q*Mb + a] holds the value of
 * local cell (a, kstop-2+q-a), or NaN where that cell is outside the block.
 * Mb = i1-i0+1.  Requires 2 <= kstop <= Mb+Nb-2. */
int dtwo_diag(const double* X, const double* Y, int32_t d,
              int64_t i0, int64_t j0, int64_t i1, int64_t j1,
              int32_t reverse, int64_t kstop, double* out);

/* linmdtw (Algorithm 2) with the readings stated in the source file.
 * min_block  : m of Algorithm 2 (the paper uses 500); values below 3 are
 *              rejected (-1) because the recursion would not terminate.
 * cost       : out, sequential FP64 sum of C along the returned path.
 * s_min      : out (may be NULL), the minimum of F+B-C at the top level, or
 *              the full-table cost when the top level is already a leaf.
 * cells      : out (may be NULL), cells evaluated: both half sweeps of every
 *              split plus every leaf table.
 * pivots     : optional out (may be NULL), pivot cells (i,j) in the order of a
 *              depth-first, left-first recursion; n_pivots receives the count.
 */
int dtwo_linmdtw(const double* X, int64_t M, const double* Y, int64_t N, int32_t d,
                 int32_t min_block, double* cost, int32_t* path, int64_t path_cap,
                 int64_t* path_len, double* s_min, int64_t* cells,
                 int32_t* pivots, int64_t pivots_cap, int64_t* n_pivots);

/* Tie-exact divide and conquer (not in the paper, whose split ties are
 * broken arbitrarily): the recursion of Algorithm 2 with the split taken from
 * a forward table that carries, per cell, the last cell of its backtrace
 * (ties DIAG, UP, LEFT) on local diagonal kf-1 or kf, kf = ceil(K/2); each
 * block's table starts from the accumulated cost its origin holds in the
 * whole problem's table.  The returned path equals dtwo_full's on every input.
 * dtwo_tie_pivot: one split of the block rows i0..i1, columns j0..j1 whose
 *   origin holds f0: pivot local row *piv_a on local diagonal *piv_k, and its
 *   accumulated cost *piv_f.  Requires Mb + Nb - 1 >= 4.
 * dtwo_linmdtw_tie: the whole recursion (cutoff as dtwo_linmdtw); cells
 *   counts every full block table and leaf table; pivots as dtwo_linmdtw. */
int dtwo_tie_pivot(const double* X, const double* Y, int32_t d, int64_t i0, int64_t j0, int64_t i1,
                   int64_t j1, double f0, int64_t* piv_a, int64_t* piv_k, double* piv_f);
int dtwo_linmdtw_tie(const double* X, int64_t M, const double* Y, int64_t N, int32_t d, int32_t min_block,
                     double* cost, int32_t* path, int64_t path_cap, int64_t* path_len, int64_t* cells,
                     int32_t* pivots, int64_t pivots_cap, int64_t* n_pivots);

/* Sequential FP64 sum of C along a given path, in path order (the cost that
 * Eq. 1 assigns to a warping path).  Returns NaN when the path is not a valid
 * warping path for M x N (Sec. 2.1 definition). */
double dtwo_path_cost(const double* X, int64_t M, const double* Y, int64_t N, int32_t d,
                      const int32_t* path, int64_t path_len);

#ifdef __cplusplus
}
#endif
#endif
