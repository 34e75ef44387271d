/*
 * edit_oracle.c -- CPU oracle for the weighted edit distance and its
 * linear-memory alignment.  Test infrastructure only: the GPU library never
 * calls it and shares no source with it.
 *
 * The paper (Tralie & Dempsey, arXiv 2008.02734) closes (Sec. 6) by naming
 * edit distance as a problem with the same dynamic-programming structure that
 * would benefit from alignment in linear memory; it defines no algorithm for
 * it.  What is computed here:
 *
 *  - Lattice: nodes (i, j), 0 <= i <= M, 0 <= j <= N, for byte strings a
 *    (length M) and b (length N).  Moves: DIAG (i-1,j-1) -> (i,j), cost 0 when
 *    a[i-1] == b[j-1] and `sub` otherwise; UP (i-1,j) -> (i,j), cost `gap`
 *    (a[i-1] deleted); LEFT (i,j-1) -> (i,j), cost `gap` (b[j-1] inserted).
 *    The distance is the least total move cost of a path (0,0) -> (M,N).
 *  - Textbook table E with E[0][j] = j gap, E[i][0] = i gap and
 *    E[i][j] = min(E[i-1][j-1] + s, E[i-1][j] + gap, E[i][j-1] + gap); the
 *    backtrace from (M,N) takes the first of DIAG, UP, LEFT whose predecessor
 *    plus move cost equals E[i][j] (the tie rule of the DTW backtrace).
 *  - Linear memory (the divide and conquer of Sec. 3 with the split placed on
 *    a row, as in Hirschberg's linear-space alignment): every path from
 *    (i0,j0) to (i1,j1) crosses node row mid, so with F[j] the least cost
 *    (i0,j0) -> (mid,j) and B[j] the least cost (mid,j) -> (i1,j1), the
 *    smallest j minimising F[j] + B[j] is a node of an optimal path.  The rows
 *    follow a fixed dyadic partition: block k of level L spans node rows
 *    floor(k M / 2^L) .. floor((k+1) M / 2^L) and splits at
 *    floor((2k+1) M / 2^(L+1)); levels split while ceil(M / 2^L) exceeds the
 *    leaf height, and the blocks of the first level that does not are solved
 *    by the textbook table and backtrace on the block.  B comes from the
 *    same row recurrence on the reversed block.
 *
 * Integers: every cost is an int64 sum of nonnegative int32 move costs.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int64_t move_sub(uint8_t x, uint8_t y, int32_t sub) { return x == y ? 0 : sub; }

/* Textbook table on the block a[i0..i1) x b[j0..j1) (node rows i0..i1,
 * columns j0..j1), written to E ((i1-i0+1) x (j1-j0+1), row-major). */
static void table_block(const uint8_t* a, const uint8_t* b, int64_t i0, int64_t j0, int64_t i1,
                        int64_t j1, int32_t sub, int32_t gap, int64_t* E) {
  const int64_t H = i1 - i0, W = j1 - j0, ld = W + 1;
  for (int64_t j = 0; j <= W; ++j) E[j] = j * (int64_t)gap;
  for (int64_t i = 1; i <= H; ++i) {
    E[i * ld] = i * (int64_t)gap;
    for (int64_t j = 1; j <= W; ++j) {
      int64_t dg = E[(i - 1) * ld + j - 1] + move_sub(a[i0 + i - 1], b[j0 + j - 1], sub);
      int64_t up = E[(i - 1) * ld + j] + gap;
      int64_t lf = E[i * ld + j - 1] + gap;
      int64_t m = dg < up ? dg : up;
      E[i * ld + j] = m < lf ? m : lf;
    }
  }
}

/* Backtrace of a block table from its last node; writes the nodes (global
 * coordinates) in path order to out (2 int32 each) and returns their count. */
static int64_t backtrace_block(const uint8_t* a, const uint8_t* b, int64_t i0, int64_t j0, int64_t i1,
                               int64_t j1, int32_t sub, int32_t gap, const int64_t* E, int32_t* out) {
  const int64_t ld = j1 - j0 + 1;
  int64_t i = i1 - i0, j = j1 - j0, n = 0;
  int32_t* rev = out;  /* written backwards first, then reversed in place */
  for (;;) {
    rev[2 * n] = (int32_t)(i0 + i);
    rev[2 * n + 1] = (int32_t)(j0 + j);
    ++n;
    if (i == 0 && j == 0) break;
    const int64_t e = E[i * ld + j];
    if (i > 0 && j > 0 && e == E[(i - 1) * ld + j - 1] + move_sub(a[i0 + i - 1], b[j0 + j - 1], sub)) {
      --i;
      --j;
    } else if (i > 0 && e == E[(i - 1) * ld + j] + gap) {
      --i;
    } else {
      --j;
    }
  }
  for (int64_t p = 0, q = n - 1; p < q; ++p, --q) {
    int32_t ti = rev[2 * p], tj = rev[2 * p + 1];
    rev[2 * p] = rev[2 * q];
    rev[2 * p + 1] = rev[2 * q + 1];
    rev[2 * q] = ti;
    rev[2 * q + 1] = tj;
  }
  return n;
}

/* Distance and textbook path of the whole problem.  path needs 2 (M+N+1)
 * int32; *path_len receives the node count.  table (may be NULL) receives
 * the (M+1) x (N+1) table.  Returns 0, or -1 when memory runs out. */
int edo_full(const uint8_t* a, int64_t M, const uint8_t* b, int64_t N, int32_t sub, int32_t gap,
             int64_t* dist, int32_t* path, int64_t* path_len, int64_t* table) {
  int64_t* E = table ? table : (int64_t*)malloc(sizeof(int64_t) * (size_t)((M + 1) * (N + 1)));
  if (!E) return -1;
  table_block(a, b, 0, 0, M, N, sub, gap, E);
  *dist = E[M * (N + 1) + N];
  if (path) *path_len = backtrace_block(a, b, 0, 0, M, N, sub, gap, E, path);
  if (!table) free(E);
  return 0;
}

/* Least cost from (i0, j0) to every node of row i1, columns j0..j1, one row
 * buffer at a time (rev = 0); with rev = 1 the same on the reversed block:
 * out[j - j0] = least cost from (i0, j) to (i1, j1), where the row of the
 * reversed table that is computed last is node row i0.  out has j1-j0+1
 * entries; work has as many.  Returns 0. */
int edo_row(const uint8_t* a, const uint8_t* b, int64_t i0, int64_t j0, int64_t i1, int64_t j1,
            int32_t sub, int32_t gap, int rev, int64_t* out) {
  const int64_t H = i1 - i0, W = j1 - j0;
  /* x(r) / y(c): the r-th row / c-th column character of the swept table */
  int64_t* row = out;
  for (int64_t c = 0; c <= W; ++c) row[c] = c * (int64_t)gap;
  for (int64_t r = 1; r <= H; ++r) {
    const uint8_t x = rev ? a[i1 - r] : a[i0 + r - 1];
    int64_t diag = row[0];
    row[0] = r * (int64_t)gap;
    for (int64_t c = 1; c <= W; ++c) {
      const uint8_t y = rev ? b[j1 - c] : b[j0 + c - 1];
      int64_t dg = diag + move_sub(x, y, sub);
      int64_t up = row[c] + gap;
      int64_t lf = row[c - 1] + gap;
      diag = row[c];
      int64_t m = dg < up ? dg : up;
      row[c] = m < lf ? m : lf;
    }
  }
  if (rev) {
    /* entry c of the reversed row belongs to column j1 - c */
    for (int64_t p = 0, q = W; p < q; ++p, --q) {
      int64_t t = row[p];
      row[p] = row[q];
      row[q] = t;
    }
  }
  return 0;
}

typedef struct {
  const uint8_t* a;
  const uint8_t* b;
  int64_t M, N;
  int32_t sub, gap;
  int32_t levels;   /* split levels */
  int32_t* path;    /* output nodes */
  int64_t n;        /* nodes written */
  int64_t* F;       /* row buffers, N + 1 each */
  int64_t* B;
  int64_t* E;       /* leaf table */
  int64_t leaf_cells;
  int64_t* pivots;  /* optional: (level, k, mid, j) per split, in recursion order */
  int64_t n_piv, piv_cap;
} rec_ctx;

static int64_t row_at(int64_t k, int64_t M, int L) { return (k * M) >> L; }

static int solve(rec_ctx* c, int L, int64_t k, int64_t j0, int64_t j1) {
  const int64_t i0 = row_at(k, c->M, L), i1 = row_at(k + 1, c->M, L);
  if (L == c->levels) {
    const int64_t cells = (i1 - i0 + 1) * (j1 - j0 + 1);
    if (cells > c->leaf_cells) {
      free(c->E);
      c->E = (int64_t*)malloc(sizeof(int64_t) * (size_t)cells);
      if (!c->E) return -1;
      c->leaf_cells = cells;
    }
    table_block(c->a, c->b, i0, j0, i1, j1, c->sub, c->gap, c->E);
    int32_t* seg = c->path + 2 * (c->n > 0 ? c->n - 1 : 0);
    int64_t m = backtrace_block(c->a, c->b, i0, j0, i1, j1, c->sub, c->gap, c->E, seg);
    /* the first node repeats the previous leaf's last one */
    c->n += c->n > 0 ? m - 1 : m;
    return 0;
  }
  const int64_t mid = row_at(2 * k + 1, c->M, L + 1);
  edo_row(c->a, c->b, i0, j0, mid, j1, c->sub, c->gap, 0, c->F);
  edo_row(c->a, c->b, mid, j0, i1, j1, c->sub, c->gap, 1, c->B);
  int64_t best = -1, bj = j0;
  for (int64_t j = j0; j <= j1; ++j) {
    const int64_t s = c->F[j - j0] + c->B[j - j0];
    if (best < 0 || s < best) {
      best = s;
      bj = j;
    }
  }
  if (c->pivots && c->n_piv < c->piv_cap) {
    int64_t* p = c->pivots + 4 * c->n_piv;
    p[0] = L;
    p[1] = k;
    p[2] = mid;
    p[3] = bj;
  }
  c->n_piv++;
  if (solve(c, L + 1, 2 * k, j0, bj)) return -1;
  return solve(c, L + 1, 2 * k + 1, bj, j1);
}

/* Split levels for M rows and leaf height leaf_rows (>= 2): the smallest L
 * with ceil(M / 2^L) <= leaf_rows. */
int32_t edo_levels(int64_t M, int32_t leaf_rows) {
  int32_t L = 0;
  while (((M + ((int64_t)1 << L) - 1) >> L) > leaf_rows) ++L;
  return L;
}

/* Linear-memory alignment.  path needs 2 (M+N+1) int32.  pivots (may be
 * NULL) receives up to piv_cap (level, k, mid, j) quadruples; *n_piv the
 * number of splits.  Returns 0, -1 (memory) or -2 (leaf_rows < 2). */
int edo_linear(const uint8_t* a, int64_t M, const uint8_t* b, int64_t N, int32_t sub, int32_t gap,
               int32_t leaf_rows, int64_t* dist, int32_t* path, int64_t* path_len, int64_t* pivots,
               int64_t piv_cap, int64_t* n_piv) {
  if (leaf_rows < 2) return -2;
  rec_ctx c;
  memset(&c, 0, sizeof c);
  c.a = a;
  c.b = b;
  c.M = M;
  c.N = N;
  c.sub = sub;
  c.gap = gap;
  c.levels = edo_levels(M, leaf_rows);
  c.path = path;
  c.F = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N + 1));
  c.B = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N + 1));
  c.pivots = pivots;
  c.piv_cap = pivots ? piv_cap : 0;
  int rc = (c.F && c.B) ? solve(&c, 0, 0, 0, N) : -1;
  free(c.F);
  free(c.B);
  free(c.E);
  if (rc) return rc;
  *path_len = c.n;
  if (n_piv) *n_piv = c.n_piv;
  /* the path's cost, move by move */
  int64_t s = 0;
  for (int64_t q = 1; q < c.n; ++q) {
    const int32_t di = path[2 * q] - path[2 * q - 2], dj = path[2 * q + 1] - path[2 * q - 1];
    s += (di == 1 && dj == 1) ? move_sub(a[path[2 * q] - 1], b[path[2 * q + 1] - 1], sub) : gap;
  }
  *dist = s;
  return 0;
}

/* Cost of a node path under the move costs; -1 when a step is not a move or
 * the path does not run from (0,0) to (M,N). */
int64_t edo_path_cost(const uint8_t* a, int64_t M, const uint8_t* b, int64_t N, int32_t sub, int32_t gap,
                      const int32_t* path, int64_t n) {
  if (n < 1 || path[0] != 0 || path[1] != 0 || path[2 * n - 2] != M || path[2 * n - 1] != N) return -1;
  int64_t s = 0;
  for (int64_t q = 1; q < n; ++q) {
    const int32_t di = path[2 * q] - path[2 * q - 2], dj = path[2 * q + 1] - path[2 * q - 1];
    if (di == 1 && dj == 1)
      s += move_sub(a[path[2 * q] - 1], b[path[2 * q + 1] - 1], sub);
    else if ((di == 1 && dj == 0) || (di == 0 && dj == 1))
      s += gap;
    else
      return -1;
  }
  return s;
}

/*
 * Local alignment (Smith-Waterman), the other problem Sec. 6 names: the best
 * score over all pairs of substrings, a match scoring +match, a mismatch
 * -mismatch, every gap letter -gap.  Table H[0][j] = H[i][0] = 0,
 * H[i][j] = max(0, H[i-1][j-1] + s, H[i-1][j] - gap, H[i][j-1] - gap).  The
 * end cell is the first cell holding the maximum in row-major order ((0,0)
 * when the maximum is 0).  Returns 0, or -1 when memory runs out.
 */
int edo_local_score(const uint8_t* a, int64_t M, const uint8_t* b, int64_t N, int32_t match, int32_t mismatch,
                    int32_t gap, int64_t* score, int64_t* i_end, int64_t* j_end) {
  int64_t* row = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N + 1));
  if (!row) return -1;
  for (int64_t j = 0; j <= N; ++j) row[j] = 0;
  int64_t best = 0, bi = 0, bj = 0;
  for (int64_t i = 1; i <= M; ++i) {
    int64_t diag = row[0];
    row[0] = 0;
    for (int64_t j = 1; j <= N; ++j) {
      const int64_t s = a[i - 1] == b[j - 1] ? match : -(int64_t)mismatch;
      int64_t h = diag + s;
      const int64_t up = row[j] - gap, lf = row[j - 1] - gap;
      if (up > h) h = up;
      if (lf > h) h = lf;
      if (h < 0) h = 0;
      diag = row[j];
      row[j] = h;
      if (h > best) {
        best = h;
        bi = i;
        bj = j;
      }
    }
  }
  free(row);
  *score = best;
  *i_end = bi;
  *j_end = bj;
  return 0;
}
