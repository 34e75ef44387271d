/*
 * CPU oracle for exact DTW -- test infrastructure only (see dtw_oracle.h).
 *
 * Plain single-threaded FP64.  Every function follows one passage of
 * Tralie & Dempsey, arXiv 2008.02734, cited at the function.  Build with
 * floating-point contraction off (-ffp-contract=off) so that the only fused
 * operation is the explicit fma() of the frame cost.
 *
 * Readings taken where the paper is silent, garbled or ambiguous (each is
 * restated where it is used):
 *   R1  Indexing is 0-based everywhere; the boundary equation covers row 0
 *       and column 0 (Sec. 2.1 mixes 0- and 1-based indices).
 *   R2  The three backpointers are LEFT, UP and DIAG as labelled in the
 *       recurrence (Sec. 2.1 lists "LEFT, RIGHT, and UP").
 *   R3  Lemma 2's split cost reads D(i,j) + D_{X_R,Y_R}(...) - C(i,j), i.e.
 *       S = F + B - C (the printed equation has C and D swapped; the prose
 *       after it and Algorithm 2 give this form).
 *   R4  DiagDTW(kstop) returns diagonals kstop-2, kstop-1, kstop, oldest
 *       first; Algorithm 2 pairs forward diagonal q with reversed diagonal
 *       (kb - q'), which with kf = ceil(K/2) and kb = kf + [K even] is the
 *       same cell set (kf + kb = K + 1).
 *   R5  Pivot ties ("breaking ties arbitrarily", Sec. 3.2) go to the smallest
 *       diagonal, then the smallest row.
 *   R6  The cutoff m must be >= 3: for M',N' >= 3 the band excludes both
 *       corner diagonals, so each child is strictly smaller.
 *   R7  Both children include the pivot; the right child's first cell is
 *       dropped on concatenation (Algorithm 2's return statement).
 *   R8  The reported cost is the sequential FP64 sum of C along the returned
 *       path (Eq. 1).
 */
#include "dtw_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Euclidean frame cost, Sec. 4.1. */
static double euclidean_cost(const double* x, const double* y, int32_t d) {
  double s = 0.0;
  for (int32_t t = 0; t < d; ++t) {
    double e = x[t] - y[t];
    s = fma(e, e, s);
  }
  return sqrt(s);
}

/* Cosine frame cost, the alternative Sec. 4.1 discusses for the chroma-type
 * features: one minus the cosine of the angle between the two frames.  Each
 * frame is divided by its Euclidean norm (sqrt of the fma chain of its
 * squares, in dimension order; a zero frame stays zero), the normalised
 * frames' dot product is an fma chain in dimension order, and the cost is
 * 1 - dot, raised to 0 where rounding takes it below (so that no cost is
 * negative). */
static double cosine_cost(const double* x, const double* y, int32_t d) {
  double nx = 0.0, ny = 0.0;
  for (int32_t t = 0; t < d; ++t) nx = fma(x[t], x[t], nx);
  for (int32_t t = 0; t < d; ++t) ny = fma(y[t], y[t], ny);
  nx = sqrt(nx);
  ny = sqrt(ny);
  double s = 0.0;
  for (int32_t t = 0; t < d; ++t) {
    double xt = nx > 0.0 ? x[t] / nx : 0.0;
    double yt = ny > 0.0 ? y[t] / ny : 0.0;
    s = fma(xt, yt, s);
  }
  double c = 1.0 - s;
  return c < 0.0 ? 0.0 : c;
}

/* The frame cost every table and sweep below uses: Euclidean unless
 * dtwo_set_cost selected the cosine cost. */
static int32_t g_cost_kind = DTWO_COST_EUCLIDEAN;

int dtwo_set_cost(int32_t kind) {
  if (kind != DTWO_COST_EUCLIDEAN && kind != DTWO_COST_COSINE) return -1;
  g_cost_kind = kind;
  return 0;
}

double dtwo_frame_cost(const double* x, const double* y, int32_t d) {
  return g_cost_kind == DTWO_COST_COSINE ? cosine_cost(x, y, d) : euclidean_cost(x, y, d);
}

enum { MOVE_DIAG = 0, MOVE_UP = 1, MOVE_LEFT = 2 };

/* Textbook DTW, Sec. 2.1: boundary equation, recurrence, backpointers,
 * backtrace from (M-1,N-1) to (0,0). */
int dtwo_full(const double* X, int64_t M, const double* Y, int64_t N, int32_t d,
              double* cost, int32_t* path, int64_t path_cap, int64_t* path_len,
              double* F_out) {
  if (!X || !Y || M < 1 || N < 1 || d < 1 || !cost || !path_len) return -1;
  double* F = F_out ? F_out : (double*)malloc(sizeof(double) * (size_t)(M * N));
  unsigned char* P = (unsigned char*)malloc((size_t)(M * N));
  if (!F || !P) {
    if (!F_out) free(F);
    free(P);
    return -3;
  }
  for (int64_t i = 0; i < M; ++i) {
    for (int64_t j = 0; j < N; ++j) {
      double c = dtwo_frame_cost(X + i * d, Y + j * d, d);
      double f;
      unsigned char p;
      if (i == 0 && j == 0) {
        f = c;
        p = MOVE_DIAG; /* unused */
      } else if (i == 0) { /* boundary: prefix sum along row 0 */
        f = F[j - 1] + c;
        p = MOVE_LEFT;
      } else if (j == 0) { /* boundary: prefix sum along column 0 */
        f = F[(i - 1) * N] + c;
        p = MOVE_UP;
      } else {
        double dg = F[(i - 1) * N + (j - 1)];
        double up = F[(i - 1) * N + j];
        double lf = F[i * N + (j - 1)];
        double best;
        if (dg <= up && dg <= lf) {
          best = dg;
          p = MOVE_DIAG;
        } else if (up <= lf) {
          best = up;
          p = MOVE_UP;
        } else {
          best = lf;
          p = MOVE_LEFT;
        }
        f = best + c;
      }
      F[i * N + j] = f;
      P[i * N + j] = p;
    }
  }
  *cost = F[(M - 1) * N + (N - 1)];
  /* Backtrace into a reversed list, then flip it. */
  int64_t len = 0;
  int64_t i = M - 1, j = N - 1;
  int rc = 0;
  for (;;) {
    if (len >= path_cap) { rc = -2; break; }
    if (path) {
      path[2 * len] = (int32_t)i;
      path[2 * len + 1] = (int32_t)j;
    }
    ++len;
    if (i == 0 && j == 0) break;
    unsigned char p = P[i * N + j];
    if (p == MOVE_DIAG) { --i; --j; }
    else if (p == MOVE_UP) { --i; }
    else { --j; }
  }
  if (rc == 0 && path) {
    for (int64_t a = 0, b = len - 1; a < b; ++a, --b) {
      int32_t ti = path[2 * a], tj = path[2 * a + 1];
      path[2 * a] = path[2 * b];
      path[2 * a + 1] = path[2 * b + 1];
      path[2 * b] = ti;
      path[2 * b + 1] = tj;
    }
  }
  *path_len = len;
  if (!F_out) free(F);
  free(P);
  return rc;
}

/* Sec. 4.2 ("Numerical Precision / Tie Breaking"): the paper checks its
 * 32-bit GPU result against a brute-force 32-bit CPU textbook solve, and two
 * 64-bit textbook solves that differ only in whether DIAG or LEFT wins a tie.
 * The two functions below are those two references, written as separate
 * plain copies of the textbook table so that each can be read on its own. */

/* Textbook DTW (Sec. 2.1) entirely in binary32: the frames are rounded to
 * float, the frame cost is s <- fmaf(e,e,s), e = x-y in float, then sqrtf,
 * and every accumulated cost is one float addition; backpointers DIAG, then
 * UP, then LEFT.  *cost is the float optimum widened to double. */
int dtwo_full_f32(const double* X, int64_t M, const double* Y, int64_t N, int32_t d,
                  double* cost, int32_t* path, int64_t path_cap, int64_t* path_len) {
  if (!X || !Y || M < 1 || N < 1 || d < 1 || !cost || !path_len) return -1;
  float* F = (float*)malloc(sizeof(float) * (size_t)(M * N));
  unsigned char* P = (unsigned char*)malloc((size_t)(M * N));
  if (!F || !P) {
    free(F);
    free(P);
    return -3;
  }
  for (int64_t i = 0; i < M; ++i) {
    for (int64_t j = 0; j < N; ++j) {
      float sc = 0.0f;
      for (int32_t t = 0; t < d; ++t) {
        float e = (float)X[i * d + t] - (float)Y[j * d + t];
        sc = fmaf(e, e, sc);
      }
      float c = sqrtf(sc);
      float f;
      unsigned char p;
      if (i == 0 && j == 0) {
        f = c;
        p = MOVE_DIAG;
      } else if (i == 0) {
        f = F[j - 1] + c;
        p = MOVE_LEFT;
      } else if (j == 0) {
        f = F[(i - 1) * N] + c;
        p = MOVE_UP;
      } else {
        float dg = F[(i - 1) * N + (j - 1)];
        float up = F[(i - 1) * N + j];
        float lf = F[i * N + (j - 1)];
        float best;
        if (dg <= up && dg <= lf) {
          best = dg;
          p = MOVE_DIAG;
        } else if (up <= lf) {
          best = up;
          p = MOVE_UP;
        } else {
          best = lf;
          p = MOVE_LEFT;
        }
        f = best + c;
      }
      F[i * N + j] = f;
      P[i * N + j] = p;
    }
  }
  *cost = (double)F[(M - 1) * N + (N - 1)];
  int64_t len = 0, i = M - 1, j = N - 1;
  int rc = 0;
  for (;;) {
    if (len >= path_cap) { rc = -2; break; }
    if (path) {
      path[2 * len] = (int32_t)i;
      path[2 * len + 1] = (int32_t)j;
    }
    ++len;
    if (i == 0 && j == 0) break;
    unsigned char p = P[i * N + j];
    if (p == MOVE_DIAG) { --i; --j; }
    else if (p == MOVE_UP) { --i; }
    else { --j; }
  }
  if (rc == 0 && path) {
    for (int64_t a = 0, b = len - 1; a < b; ++a, --b) {
      int32_t ti = path[2 * a], tj = path[2 * a + 1];
      path[2 * a] = path[2 * b];
      path[2 * a + 1] = path[2 * b + 1];
      path[2 * b] = ti;
      path[2 * b + 1] = tj;
    }
  }
  *path_len = len;
  free(F);
  free(P);
  return rc;
}

/* Textbook DTW in FP64 with the opposite tie rule: LEFT wins over DIAG.  The
 * whole preference order is reversed, LEFT, then UP, then DIAG (the paper
 * names only the DIAG/LEFT pair; UP keeps its middle place).  Same table,
 * frame cost and backtrace as dtwo_full otherwise. */
int dtwo_full_left_first(const double* X, int64_t M, const double* Y, int64_t N, int32_t d,
                         double* cost, int32_t* path, int64_t path_cap, int64_t* path_len) {
  if (!X || !Y || M < 1 || N < 1 || d < 1 || !cost || !path_len) return -1;
  double* F = (double*)malloc(sizeof(double) * (size_t)(M * N));
  unsigned char* P = (unsigned char*)malloc((size_t)(M * N));
  if (!F || !P) {
    free(F);
    free(P);
    return -3;
  }
  for (int64_t i = 0; i < M; ++i) {
    for (int64_t j = 0; j < N; ++j) {
      double c = dtwo_frame_cost(X + i * d, Y + j * d, d);
      double f;
      unsigned char p;
      if (i == 0 && j == 0) {
        f = c;
        p = MOVE_DIAG;
      } else if (i == 0) {
        f = F[j - 1] + c;
        p = MOVE_LEFT;
      } else if (j == 0) {
        f = F[(i - 1) * N] + c;
        p = MOVE_UP;
      } else {
        double dg = F[(i - 1) * N + (j - 1)];
        double up = F[(i - 1) * N + j];
        double lf = F[i * N + (j - 1)];
        double best;
        if (lf <= up && lf <= dg) {
          best = lf;
          p = MOVE_LEFT;
        } else if (up <= dg) {
          best = up;
          p = MOVE_UP;
        } else {
          best = dg;
          p = MOVE_DIAG;
        }
        f = best + c;
      }
      F[i * N + j] = f;
      P[i * N + j] = p;
    }
  }
  *cost = F[(M - 1) * N + (N - 1)];
  int64_t len = 0, i = M - 1, j = N - 1;
  int rc = 0;
  for (;;) {
    if (len >= path_cap) { rc = -2; break; }
    if (path) {
      path[2 * len] = (int32_t)i;
      path[2 * len + 1] = (int32_t)j;
    }
    ++len;
    if (i == 0 && j == 0) break;
    unsigned char p = P[i * N + j];
    if (p == MOVE_DIAG) { --i; --j; }
    else if (p == MOVE_UP) { --i; }
    else { --j; }
  }
  if (rc == 0 && path) {
    for (int64_t a = 0, b = len - 1; a < b; ++a, --b) {
      int32_t ti = path[2 * a], tj = path[2 * a + 1];
      path[2 * a] = path[2 * b];
      path[2 * a + 1] = path[2 * b + 1];
      path[2 * b] = ti;
      path[2 * b + 1] = tj;
    }
  }
  *path_len = len;
  free(F);
  free(P);
  return rc;
}

/* Number of cells of an Mb x Nb block on local diagonal k (cells (a,k-a)). */
static int64_t diag_len(int64_t Mb, int64_t Nb, int64_t k) {
  int64_t lo = k - (Nb - 1) > 0 ? k - (Nb - 1) : 0;
  int64_t hi = k < Mb - 1 ? k : Mb - 1;
  return hi >= lo ? hi - lo + 1 : 0;
}

/* DiagDTW, Algorithm 1 (Sec. 3.1): the accumulated cost is filled one
 * anti-diagonal at a time; diagonal k needs only diagonals k-1 and k-2, kept
 * in three buffers that rotate after each diagonal.  Buffers are indexed by
 * local row a (length Mb) so the neighbour lookups read as in the
 * recurrence: (a-1,b-1) on k-2, (a-1,b) and (a,b-1) on k-1. */
int dtwo_diag(const double* X, const double* Y, int32_t d,
              int64_t i0, int64_t j0, int64_t i1, int64_t j1,
              int32_t reverse, int64_t kstop, double* out) {
  if (!X || !Y || !out || d < 1 || i1 < i0 || j1 < j0) return -1;
  const int64_t Mb = i1 - i0 + 1, Nb = j1 - j0 + 1;
  if (kstop < 2 || kstop > Mb + Nb - 2) return -1;
  double* buf = (double*)malloc(sizeof(double) * (size_t)(3 * Mb));
  if (!buf) return -3;
  double* dm2 = buf;          /* diagonal k-2 */
  double* dm1 = buf + Mb;     /* diagonal k-1 */
  double* dk = buf + 2 * Mb;  /* diagonal k   */
  for (int64_t a = 0; a < 3 * Mb; ++a) buf[a] = NAN;
  for (int64_t k = 0; k <= kstop; ++k) {
    int64_t lo = k - (Nb - 1) > 0 ? k - (Nb - 1) : 0;
    int64_t hi = k < Mb - 1 ? k : Mb - 1;
    for (int64_t a = 0; a < Mb; ++a) dk[a] = NAN;
    for (int64_t a = lo; a <= hi; ++a) {
      int64_t b = k - a;
      int64_t gi = reverse ? i1 - a : i0 + a;
      int64_t gj = reverse ? j1 - b : j0 + b;
      double c = dtwo_frame_cost(X + gi * d, Y + gj * d, d);
      double f;
      if (a == 0 && b == 0) f = c;
      else if (a == 0) f = dm1[0] + c;          /* F(0,b-1) + C */
      else if (b == 0) f = dm1[a - 1] + c;      /* F(a-1,0) + C */
      else {
        double dg = dm2[a - 1], up = dm1[a - 1], lf = dm1[a];
        double best = dg;
        if (up < best) best = up;
        if (lf < best) best = lf;
        f = best + c;
      }
      dk[a] = f;
    }
    if (k == kstop) break;
    /* circular shift of the three buffers */
    double* t = dm2;
    dm2 = dm1;
    dm1 = dk;
    dk = t;
  }
  memcpy(out, dm2, sizeof(double) * (size_t)Mb);
  memcpy(out + Mb, dm1, sizeof(double) * (size_t)Mb);
  memcpy(out + 2 * Mb, dk, sizeof(double) * (size_t)Mb);
  free(buf);
  return 0;
}

typedef struct {
  const double* X;
  const double* Y;
  int32_t d;
  int32_t m;
  int32_t* path;
  int64_t cap;
  int64_t len;
  int64_t cells;
  int32_t* piv;
  int64_t piv_cap;
  int64_t n_piv;
  int depth;
  double s_min;
  int err;
} rec_state;

/* Append a segment; when the accumulated path already ends at the segment's
 * first cell, that cell is not repeated (R7). */
static void append_segment(rec_state* st, const int32_t* seg, int64_t n) {
  int64_t start = 0;
  if (st->len > 0 && n > 0 && st->path[2 * (st->len - 1)] == seg[0] &&
      st->path[2 * (st->len - 1) + 1] == seg[1])
    start = 1;
  for (int64_t q = start; q < n; ++q) {
    if (st->len >= st->cap) { st->err = -2; return; }
    st->path[2 * st->len] = seg[2 * q];
    st->path[2 * st->len + 1] = seg[2 * q + 1];
    ++st->len;
  }
}

/* One call of Algorithm 2 on the block rows i0..i1, columns j0..j1. */
static void linm_rec(rec_state* st, int64_t i0, int64_t j0, int64_t i1, int64_t j1) {
  if (st->err) return;
  const int64_t Mb = i1 - i0 + 1, Nb = j1 - j0 + 1;
  const int32_t d = st->d;
  if (Mb < st->m || Nb < st->m) {
    /* Cutoff: brute-force (textbook) path on the sub-block. */
    int32_t* seg = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(Mb + Nb - 1));
    if (!seg) { st->err = -3; return; }
    double c;
    int64_t n = 0;
    int rc = dtwo_full(st->X + i0 * d, Mb, st->Y + j0 * d, Nb, d, &c, seg, Mb + Nb - 1, &n, NULL);
    if (rc) { free(seg); st->err = rc; return; }
    if (st->depth == 0) st->s_min = c;
    for (int64_t q = 0; q < n; ++q) {
      seg[2 * q] += (int32_t)i0;
      seg[2 * q + 1] += (int32_t)j0;
    }
    st->cells += Mb * Nb;
    append_segment(st, seg, n);
    free(seg);
    return;
  }
  const int64_t K = Mb + Nb - 1;        /* number of diagonals */
  const int64_t kf = (K + 1) / 2;       /* ceil(K/2) */
  const int64_t kb = kf + (K % 2 == 0); /* one more when K is even */
  double* fw = (double*)malloc(sizeof(double) * 3 * (size_t)Mb);
  double* bw = (double*)malloc(sizeof(double) * 3 * (size_t)Mb);
  if (!fw || !bw) { free(fw); free(bw); st->err = -3; return; }
  int rc = dtwo_diag(st->X, st->Y, d, i0, j0, i1, j1, 0, kf, fw);
  if (!rc) rc = dtwo_diag(st->X, st->Y, d, i0, j0, i1, j1, 1, kb, bw);
  if (rc) { free(fw); free(bw); st->err = rc; return; }
  for (int64_t k = 0; k <= kf; ++k) st->cells += diag_len(Mb, Nb, k);
  for (int64_t k = 0; k <= kb; ++k) st->cells += diag_len(Mb, Nb, k);
  /* Split cost on the three central diagonals (Lemma 2, R3, R4), argmin (R5). */
  double best = INFINITY;
  int64_t ba = -1, bk = -1;
  for (int64_t k = kf - 2; k <= kf; ++k) {
    int64_t kr = K - 1 - k; /* the same cells on the reversed sweep */
    int64_t lo = k - (Nb - 1) > 0 ? k - (Nb - 1) : 0;
    int64_t hi = k < Mb - 1 ? k : Mb - 1;
    for (int64_t a = lo; a <= hi; ++a) {
      int64_t ar = Mb - 1 - a;
      double f = fw[(k - (kf - 2)) * Mb + a];
      double b = bw[(kr - (kb - 2)) * Mb + ar];
      double c = dtwo_frame_cost(st->X + (i0 + a) * d, st->Y + (j0 + k - a) * d, d);
      double s = (f + b) - c;
      if (s < best) { best = s; ba = a; bk = k; }
    }
  }
  free(fw);
  free(bw);
  if (ba < 0) { st->err = -1; return; }
  if (st->depth == 0) st->s_min = best;
  const int64_t pi = i0 + ba, pj = j0 + (bk - ba);
  if (st->piv) {
    if (st->n_piv < st->piv_cap) {
      st->piv[2 * st->n_piv] = (int32_t)pi;
      st->piv[2 * st->n_piv + 1] = (int32_t)pj;
    }
  }
  ++st->n_piv;
  st->depth++;
  linm_rec(st, i0, j0, pi, pj); /* left: X(0..i), Y(0..j) */
  linm_rec(st, pi, pj, i1, j1); /* right: X(i..), Y(j..), pivot included */
  st->depth--;
}

int dtwo_linmdtw(const double* X, int64_t M, const double* Y, int64_t N, int32_t d,
                 int32_t min_block, double* cost, int32_t* path, int64_t path_cap,
                 int64_t* path_len, double* s_min, int64_t* cells,
                 int32_t* pivots, int64_t pivots_cap, int64_t* n_pivots) {
  if (!X || !Y || M < 1 || N < 1 || d < 1 || min_block < 3 || !cost || !path || !path_len)
    return -1;
  if (path_cap < M + N - 1) return -2;
  rec_state st;
  memset(&st, 0, sizeof(st));
  st.X = X;
  st.Y = Y;
  st.d = d;
  st.m = min_block;
  st.path = path;
  st.cap = path_cap;
  st.piv = pivots;
  st.piv_cap = pivots ? pivots_cap : 0;
  st.s_min = NAN;
  linm_rec(&st, 0, 0, M - 1, N - 1);
  if (st.err) return st.err;
  *path_len = st.len;
  *cost = dtwo_path_cost(X, M, Y, N, d, path, st.len);
  if (s_min) *s_min = st.s_min;
  if (cells) *cells = st.cells;
  if (n_pivots) *n_pivots = st.n_piv;
  if (pivots && st.n_piv > pivots_cap) return -2;
  return 0;
}

/* ------------------------------------------------------------------------
 * Tie-exact divide and conquer (an addition to the paper's method; the
 * paper breaks split ties arbitrarily, Sec. 3.2).  A split is chosen so that
 * the concatenated path equals the textbook backtrace (Sec. 2.1, ties DIAG,
 * UP, LEFT) on every input:
 *  - the block's table is filled forward from its origin, whose accumulated
 *    cost f0 is given (the value the whole problem's table holds there), so
 *    every cell on the textbook path holds exactly its value in the whole
 *    table;
 *  - each cell carries a label: on local diagonals kf-1 and kf (kf = ceil(K/2),
 *    K diagonals) the cell itself, past them the label of the predecessor
 *    its backpointer names.  The end cell's label is the last cell of the
 *    backtrace with a + b <= kf: the pivot;
 *  - the left child keeps f0, the right child starts from the pivot's value.
 * A cell off the textbook path can hold a larger value in a child's table
 * than in the whole table, never a smaller one, so no backpointer on the path
 * changes (the tie order is the same everywhere). */

/* Forward table of the block rows i0..i1, columns j0..j1 with F(origin) =
 * f0, labels as above; returns the pivot (local row a, local diagonal k) and
 * its accumulated cost.  Requires Mb + Nb - 1 >= 4. */
int dtwo_tie_pivot(const double* X, const double* Y, int32_t d, int64_t i0, int64_t j0, int64_t i1,
                   int64_t j1, double f0, int64_t* piv_a, int64_t* piv_k, double* piv_f) {
  const int64_t Mb = i1 - i0 + 1, Nb = j1 - j0 + 1;
  if (!X || !Y || d < 1 || Mb < 1 || Nb < 1 || Mb + Nb - 1 < 4 || !piv_a || !piv_k || !piv_f) return -1;
  const int64_t K = Mb + Nb - 1, kf = (K + 1) / 2;
  double* F = (double*)malloc(sizeof(double) * (size_t)(Mb * Nb));
  int64_t* lab = (int64_t*)malloc(sizeof(int64_t) * (size_t)(Mb * Nb));
  if (!F || !lab) { free(F); free(lab); return -3; }
  for (int64_t a = 0; a < Mb; ++a) {
    for (int64_t b = 0; b < Nb; ++b) {
      const double c = dtwo_frame_cost(X + (i0 + a) * d, Y + (j0 + b) * d, d);
      double f;
      int64_t from; /* index of the predecessor the backpointer names */
      if (a == 0 && b == 0) {
        f = f0;
        from = -1;
      } else if (a == 0) {
        f = F[b - 1] + c;
        from = b - 1;
      } else if (b == 0) {
        f = F[(a - 1) * Nb] + c;
        from = (a - 1) * Nb;
      } else {
        const double dg = F[(a - 1) * Nb + (b - 1)], up = F[(a - 1) * Nb + b], lf = F[a * Nb + (b - 1)];
        if (dg <= up && dg <= lf) { f = dg + c; from = (a - 1) * Nb + (b - 1); }
        else if (up <= lf) { f = up + c; from = (a - 1) * Nb + b; }
        else { f = lf + c; from = a * Nb + (b - 1); }
      }
      F[a * Nb + b] = f;
      /* label: a cell on diagonal kf-1 or kf names itself (2a + [on kf]) */
      if (a + b == kf - 1 || a + b == kf) lab[a * Nb + b] = 2 * a + (a + b == kf);
      else lab[a * Nb + b] = from >= 0 ? lab[from] : -1;
    }
  }
  const int64_t L = lab[Mb * Nb - 1];
  int rc = 0;
  if (L < 0) rc = -1;
  else {
    *piv_a = L / 2;
    *piv_k = kf - 1 + (L % 2);
    *piv_f = F[*piv_a * Nb + (*piv_k - *piv_a)];
  }
  free(F);
  free(lab);
  return rc;
}

/* Textbook table and backtrace of a block whose origin holds f0 (the segment
 * of the whole problem's textbook path through that block). */
static int full_block_from(const double* X, const double* Y, int32_t d, int64_t i0, int64_t j0, int64_t Mb,
                           int64_t Nb, double f0, int32_t* seg, int64_t* n) {
  double* F = (double*)malloc(sizeof(double) * (size_t)(Mb * Nb));
  unsigned char* P = (unsigned char*)malloc((size_t)(Mb * Nb));
  if (!F || !P) { free(F); free(P); return -3; }
  for (int64_t a = 0; a < Mb; ++a)
    for (int64_t b = 0; b < Nb; ++b) {
      const double c = dtwo_frame_cost(X + (i0 + a) * d, Y + (j0 + b) * d, d);
      double f;
      unsigned char p = MOVE_DIAG;
      if (a == 0 && b == 0) f = f0;
      else if (a == 0) { f = F[b - 1] + c; p = MOVE_LEFT; }
      else if (b == 0) { f = F[(a - 1) * Nb] + c; p = MOVE_UP; }
      else {
        const double dg = F[(a - 1) * Nb + (b - 1)], up = F[(a - 1) * Nb + b], lf = F[a * Nb + (b - 1)];
        if (dg <= up && dg <= lf) { f = dg + c; p = MOVE_DIAG; }
        else if (up <= lf) { f = up + c; p = MOVE_UP; }
        else { f = lf + c; p = MOVE_LEFT; }
      }
      F[a * Nb + b] = f;
      P[a * Nb + b] = p;
    }
  int64_t len = 0, a = Mb - 1, b = Nb - 1;
  for (;;) {
    seg[2 * len] = (int32_t)(i0 + a);
    seg[2 * len + 1] = (int32_t)(j0 + b);
    ++len;
    if (a == 0 && b == 0) break;
    const unsigned char p = P[a * Nb + b];
    if (p == MOVE_DIAG) { --a; --b; }
    else if (p == MOVE_UP) --a;
    else --b;
  }
  for (int64_t u = 0, v = len - 1; u < v; ++u, --v) {
    const int32_t ti = seg[2 * u], tj = seg[2 * u + 1];
    seg[2 * u] = seg[2 * v];
    seg[2 * u + 1] = seg[2 * v + 1];
    seg[2 * v] = ti;
    seg[2 * v + 1] = tj;
  }
  *n = len;
  free(F);
  free(P);
  return 0;
}

static void tie_rec(rec_state* st, int64_t i0, int64_t j0, int64_t i1, int64_t j1, double f0) {
  if (st->err) return;
  const int64_t Mb = i1 - i0 + 1, Nb = j1 - j0 + 1;
  if (Mb < st->m || Nb < st->m) {
    int32_t* seg = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(Mb + Nb - 1));
    if (!seg) { st->err = -3; return; }
    int64_t n = 0;
    const int rc = full_block_from(st->X, st->Y, st->d, i0, j0, Mb, Nb, f0, seg, &n);
    if (rc) { free(seg); st->err = rc; return; }
    st->cells += Mb * Nb;
    append_segment(st, seg, n);
    free(seg);
    return;
  }
  int64_t pa = 0, pk = 0;
  double pf = 0.0;
  const int rc = dtwo_tie_pivot(st->X, st->Y, st->d, i0, j0, i1, j1, f0, &pa, &pk, &pf);
  if (rc) { st->err = rc; return; }
  st->cells += Mb * Nb;
  const int64_t pi = i0 + pa, pj = j0 + (pk - pa);
  if (st->piv && st->n_piv < st->piv_cap) {
    st->piv[2 * st->n_piv] = (int32_t)pi;
    st->piv[2 * st->n_piv + 1] = (int32_t)pj;
  }
  ++st->n_piv;
  tie_rec(st, i0, j0, pi, pj, f0);
  tie_rec(st, pi, pj, i1, j1, pf);
}

int dtwo_linmdtw_tie(const double* X, int64_t M, const double* Y, int64_t N, int32_t d, int32_t min_block,
                     double* cost, int32_t* path, int64_t path_cap, int64_t* path_len, int64_t* cells,
                     int32_t* pivots, int64_t pivots_cap, int64_t* n_pivots) {
  if (!X || !Y || M < 1 || N < 1 || d < 1 || min_block < 3 || !cost || !path || !path_len) return -1;
  if (path_cap < M + N - 1) return -2;
  rec_state st;
  memset(&st, 0, sizeof(st));
  st.X = X;
  st.Y = Y;
  st.d = d;
  st.m = min_block;
  st.path = path;
  st.cap = path_cap;
  st.piv = pivots;
  st.piv_cap = pivots ? pivots_cap : 0;
  tie_rec(&st, 0, 0, M - 1, N - 1, dtwo_frame_cost(X, Y, d));
  if (st.err) return st.err;
  *path_len = st.len;
  *cost = dtwo_path_cost(X, M, Y, N, d, path, st.len);
  if (cells) *cells = st.cells;
  if (n_pivots) *n_pivots = st.n_piv;
  if (pivots && st.n_piv > pivots_cap) return -2;
  return 0;
}

/* Eq. 1 evaluated along a path, after checking the path definition of
 * Sec. 2.1 (start, end, allowed steps). */
double dtwo_path_cost(const double* X, int64_t M, const double* Y, int64_t N, int32_t d,
                      const int32_t* path, int64_t path_len) {
  if (!X || !Y || !path || path_len < 1) return NAN;
  if (path[0] != 0 || path[1] != 0) return NAN;
  if (path[2 * (path_len - 1)] != M - 1 || path[2 * (path_len - 1) + 1] != N - 1) return NAN;
  double s = 0.0;
  for (int64_t q = 0; q < path_len; ++q) {
    int32_t i = path[2 * q], j = path[2 * q + 1];
    if (i < 0 || j < 0 || i >= M || j >= N) return NAN;
    if (q > 0) {
      int32_t di = i - path[2 * (q - 1)], dj = j - path[2 * (q - 1) + 1];
      if (!((di == 0 && dj == 1) || (di == 1 && dj == 0) || (di == 1 && dj == 1))) return NAN;
    }
    s += dtwo_frame_cost(X + (int64_t)i * d, Y + (int64_t)j * d, d);
  }
  return s;
}
