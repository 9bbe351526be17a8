/*
 * Serial FP64 CPU oracle for level-scheduled SpTRSV with equation rewriting.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the checker: only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it. It shares no
 * code, header, table or helper with the HIP library, and the HIP library never
 * calls it. It is deliberately plain: one thread, no blocking, no fusion, each
 * step written in the order the paper states it. Build with
 *   gcc -O2 -ffp-contract=off -fPIC -shared oracle.c -o liboracle.so
 * (no FMA contraction, so every product and sum is rounded on its own).
 *
 * Paper: "A Graph Transformation Strategy for Optimizing SpTRSV"
 * (Yilmaz and Yildiz, arXiv 2206.05843).
 *
 *   O1 orc_validate        CSR well-formedness, diagonal last   (Sec. II.A, Algorithm 1)
 *   O2 orc_solve           serial forward substitution          (Sec. II.A, Algorithm 1)
 *      orc_solve_upper     serial backward substitution for an upper-triangular
 *                          matrix (the same recurrence from the last row up)
 *   O3 orc_levels          level sets by longest path in DAG_L  (Sec. II.A)
 *   O4 orc_level_costs     row/level cost, avgLevelCost         (Sec. III, cost model)
 *   O5 orc_rewrite_*       thin/target/source scan + explicit
 *                          substitution and rearrangement       (Sec. II.B, Sec. III)
 *      orc_spmv            b' = T b for the rewritten system    (Sec. II.B, rearrangement)
 *      orc_level_features  per-level features for the learned policy (no paper passage;
 *                          built from the cost model and a distance-1 substitution)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Status names are mapped to strings on the Python side; the numbering is the
 * oracle's own. */
enum {
  ORC_OK = 0,
  ORC_ERR_ARG = 1,
  ORC_ERR_NOT_LOWER = 2,
  ORC_ERR_UNSORTED = 3,
  ORC_ERR_MISSING_DIAG = 4,
  ORC_ERR_ZERO_PIVOT = 5,
  ORC_ERR_NONFINITE = 6,
  ORC_ERR_ALLOC = 7,
  ORC_ERR_OVERFLOW = 8
};

/* per-level features of the learned policy */
enum { ORC_NFEAT = 20 };

/* ---------------------------------------------------------------------------
 * O1. Validation. Algorithm 1 reads the diagonal of row i at the last slot of
 * the row, so a usable row has its columns in ascending order, every column at
 * most i, the last column equal to i and a nonzero diagonal. All problems are
 * collected; the one reported is the first in the priority order
 * ARG > NOT_LOWER > UNSORTED > MISSING_DIAG > ZERO_PIVOT > NONFINITE.
 * ------------------------------------------------------------------------- */
int orc_validate(int32_t n, int32_t nnz, const int32_t *rp, const int32_t *ci, const double *v) {
  if (n < 0 || nnz < 0 || rp[0] != 0 || rp[n] != nnz) return ORC_ERR_ARG;
  for (int32_t r = 0; r < n; ++r)
    if (rp[r + 1] < rp[r]) return ORC_ERR_ARG;
  int seen[7] = {0};
  for (int32_t r = 0; r < n; ++r) {
    int32_t b = rp[r], e = rp[r + 1];
    for (int32_t p = b; p < e; ++p) {
      if (ci[p] < 0 || ci[p] > r) seen[ORC_ERR_NOT_LOWER] = 1;
      if (p + 1 < e && ci[p] >= ci[p + 1]) seen[ORC_ERR_UNSORTED] = 1;
      if (!isfinite(v[p])) seen[ORC_ERR_NONFINITE] = 1;
    }
    if (e == b || ci[e - 1] != r)
      seen[ORC_ERR_MISSING_DIAG] = 1;
    else if (v[e - 1] == 0.0)
      seen[ORC_ERR_ZERO_PIVOT] = 1;
  }
  for (int k = ORC_ERR_NOT_LOWER; k <= ORC_ERR_NONFINITE; ++k)
    if (seen[k]) return k;
  return ORC_OK;
}

/* ---------------------------------------------------------------------------
 * O2. Serial forward substitution, Algorithm 1 (Sec. II.A). For each row in
 * order: accumulate the off-diagonal products in ascending column order into
 * one scalar, subtract from b, divide by the diagonal (the last entry of the
 * row). The printed listing indexes its accumulator by column; a single scalar
 * per row is the reading that computes x = L^{-1} b. Column-major b and x.
 * ------------------------------------------------------------------------- */
/* Backward substitution, U x = b, U upper-triangular in CSR with the diagonal
 * first in each row: x_i = (b_i - sum_{j > i} U_ij x_j) / U_ii for i from n-1
 * down to 0, the off-diagonals in ascending column order. */
void orc_solve_upper(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nrhs,
                     const double *b, int64_t ldb, double *x, int64_t ldx) {
  for (int32_t c = 0; c < nrhs; ++c) {
    const double *bc = b + (int64_t)c * ldb;
    double *xc = x + (int64_t)c * ldx;
    for (int32_t i = n - 1; i >= 0; --i) {
      double sum = 0.0;
      for (int32_t p = rp[i] + 1; p < rp[i + 1]; ++p) sum = sum + v[p] * xc[ci[p]];
      xc[i] = (bc[i] - sum) / v[rp[i]];
    }
  }
}

void orc_solve(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nrhs,
               const double *b, int64_t ldb, double *x, int64_t ldx) {
  for (int32_t c = 0; c < nrhs; ++c) {
    const double *bc = b + (int64_t)c * ldb;
    double *xc = x + (int64_t)c * ldx;
    for (int32_t i = 0; i < n; ++i) {
      double sum = 0.0;
      for (int32_t p = rp[i]; p < rp[i + 1] - 1; ++p) sum = sum + v[p] * xc[ci[p]];
      xc[i] = (bc[i] - sum) / v[rp[i + 1] - 1];
    }
  }
}

/* y = A b for a CSR matrix (ascending column order per row), column-major. */
void orc_spmv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nrhs,
              const double *b, int64_t ldb, double *y, int64_t ldy) {
  for (int32_t c = 0; c < nrhs; ++c)
    for (int32_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int32_t p = rp[i]; p < rp[i + 1]; ++p) s = s + v[p] * b[(int64_t)c * ldb + ci[p]];
      y[(int64_t)c * ldy + i] = s;
    }
}

/* ---------------------------------------------------------------------------
 * O3. Level sets (Sec. II.A): rows in one level never depend on each other and
 * levels run in order. The level of a row is the length of the longest
 * dependency path ending at it: 0 for a row with no off-diagonal, else one more
 * than the largest level among the rows it reads. level_ptr is a count and an
 * exclusive prefix sum; level_rows lists the rows of each level in ascending
 * row order. Returns the number of levels.
 * ------------------------------------------------------------------------- */
int32_t orc_levels(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *lev, int32_t *level_ptr,
                   int32_t *level_rows) {
  int32_t nlev = 0;
  for (int32_t r = 0; r < n; ++r) {
    int32_t l = 0;
    for (int32_t p = rp[r]; p < rp[r + 1] - 1; ++p)
      if (lev[ci[p]] + 1 > l) l = lev[ci[p]] + 1;
    lev[r] = l;
    if (l + 1 > nlev) nlev = l + 1;
  }
  for (int32_t l = 0; l <= nlev; ++l) level_ptr[l] = 0;
  for (int32_t r = 0; r < n; ++r) level_ptr[lev[r] + 1] += 1;
  for (int32_t l = 0; l < nlev; ++l) level_ptr[l + 1] += level_ptr[l];
  int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nlev > 0 ? nlev : 1));
  for (int32_t l = 0; l < nlev; ++l) fill[l] = level_ptr[l];
  for (int32_t r = 0; r < n; ++r) level_rows[fill[lev[r]]++] = r;
  free(fill);
  return nlev;
}

/* ---------------------------------------------------------------------------
 * O4. Cost model (Sec. III): a row with nnz nonzeros (diagonal included) costs
 * 2*nnz - 1 flops; a level costs the sum over its rows, i.e. 2*sum(nnz) - rows.
 * avgLevelCost is the total cost divided by the number of levels, computed once.
 * Outputs per level: rows, sum of nnz, cost. Returns avgLevelCost.
 * ------------------------------------------------------------------------- */
double orc_level_costs(int32_t n, const int32_t *rp, int32_t nlev, const int32_t *level_ptr,
                       const int32_t *level_rows, int64_t *rows_out, int64_t *nnz_out, int64_t *cost_out,
                       int64_t *total_out) {
  int64_t total = 0;
  (void)n;
  for (int32_t l = 0; l < nlev; ++l) {
    int64_t rows = 0, nz = 0, cost = 0;
    for (int32_t q = level_ptr[l]; q < level_ptr[l + 1]; ++q) {
      int32_t r = level_rows[q];
      int64_t k = rp[r + 1] - rp[r];
      rows += 1;
      nz += k;
      cost += 2 * k - 1;
    }
    rows_out[l] = rows;
    nnz_out[l] = nz;
    cost_out[l] = cost;
    total += cost;
  }
  *total_out = total;
  return nlev > 0 ? (double)total / (double)nlev : 0.0;
}

/* ---------------------------------------------------------------------------
 * Explicit substitution (Sec. II.B, Fig. 2) with rearrangement into Lx=b form.
 *
 * Row r is rewritten toward target level t: every unknown x[j] of the row whose
 * row currently sits at level >= t (cur[j] >= t) is replaced by row j's own
 * equation, x[j] = (b[j] - sum_k L[j][k] x[k]) / L[j][j]. Collecting the
 * coefficients of each remaining unknown gives the rewritten row L'[r]
 * (diagonal unchanged) and collecting the b terms gives row T[r] of the
 * b-transform, so that L'[r] x = T[r] b.
 *
 * Unknowns are eliminated largest column first; each elimination can only add
 * columns smaller than the eliminated one, so a column is eliminated at most
 * once. A column that enters the row by fill-in stays in the pattern even if its
 * coefficient later cancels to zero (the pattern is structural).
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t n;
  int32_t *pos;     /* column -> slot in w, or -1 */
  int32_t *wcol;    /* slot -> column */
  double *wval;     /* slot -> coefficient */
  uint8_t *alive;   /* slot still in the row (0 once eliminated) */
  int32_t wlen, wcap;
  int32_t *heap;    /* max-heap of columns still to eliminate */
  int32_t hlen, hcap;
  int32_t *tcol;    /* eliminated columns */
  double *tval;     /* their T coefficients */
  int32_t tlen, tcap;
} subst_ws;

static int ws_grow_i32(int32_t **a, int32_t *cap, int32_t need) {
  if (need <= *cap) return 1;
  int32_t nc = *cap ? *cap : 64;
  while (nc < need) nc *= 2;
  int32_t *p = (int32_t *)realloc(*a, sizeof(int32_t) * (size_t)nc);
  if (!p) return 0;
  *a = p;
  *cap = nc;
  return 1;
}

static int ws_grow_w(subst_ws *s, int32_t need) {
  if (need <= s->wcap) return 1;
  int32_t nc = s->wcap ? s->wcap : 64;
  while (nc < need) nc *= 2;
  int32_t *c = (int32_t *)realloc(s->wcol, sizeof(int32_t) * (size_t)nc);
  if (!c) return 0;
  s->wcol = c;
  double *v = (double *)realloc(s->wval, sizeof(double) * (size_t)nc);
  if (!v) return 0;
  s->wval = v;
  uint8_t *a = (uint8_t *)realloc(s->alive, (size_t)nc);
  if (!a) return 0;
  s->alive = a;
  s->wcap = nc;
  return 1;
}

static int ws_grow_t(subst_ws *s, int32_t need) {
  if (need <= s->tcap) return 1;
  int32_t nc = s->tcap ? s->tcap : 64;
  while (nc < need) nc *= 2;
  int32_t *c = (int32_t *)realloc(s->tcol, sizeof(int32_t) * (size_t)nc);
  if (!c) return 0;
  s->tcol = c;
  double *v = (double *)realloc(s->tval, sizeof(double) * (size_t)nc);
  if (!v) return 0;
  s->tval = v;
  s->tcap = nc;
  return 1;
}

static void heap_push(subst_ws *s, int32_t c) {
  int32_t i = s->hlen++;
  s->heap[i] = c;
  while (i > 0) {
    int32_t p = (i - 1) / 2;
    if (s->heap[p] >= s->heap[i]) break;
    int32_t t = s->heap[p];
    s->heap[p] = s->heap[i];
    s->heap[i] = t;
    i = p;
  }
}

static int32_t heap_pop(subst_ws *s) {
  int32_t top = s->heap[0];
  s->heap[0] = s->heap[--s->hlen];
  int32_t i = 0;
  for (;;) {
    int32_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < s->hlen && s->heap[l] > s->heap[m]) m = l;
    if (r < s->hlen && s->heap[r] > s->heap[m]) m = r;
    if (m == i) break;
    int32_t t = s->heap[m];
    s->heap[m] = s->heap[i];
    s->heap[i] = t;
    i = m;
  }
  return top;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* Substitute row r toward target t. On return the rewritten row's surviving
 * off-diagonal columns are the alive slots of w and the eliminated columns are
 * tcol/tval (unsorted). Returns 0 on allocation failure. */
static int substitute(subst_ws *s, const int32_t *rp, const int32_t *ci, const double *v, const int32_t *cur,
                      int32_t r, int32_t t) {
  s->wlen = 0;
  s->hlen = 0;
  s->tlen = 0;
  int32_t b = rp[r], e = rp[r + 1] - 1;
  if (!ws_grow_w(s, e - b) || !ws_grow_i32(&s->heap, &s->hcap, e - b)) return 0;
  for (int32_t p = b; p < e; ++p) {
    int32_t k = ci[p];
    s->pos[k] = s->wlen;
    s->wcol[s->wlen] = k;
    s->wval[s->wlen] = v[p];
    s->alive[s->wlen] = 1;
    s->wlen++;
    if (cur[k] >= t) heap_push(s, k);
  }
  while (s->hlen > 0) {
    int32_t j = heap_pop(s);
    int32_t sj = s->pos[j];
    double m = s->wval[sj] / v[rp[j + 1] - 1];
    s->alive[sj] = 0;
    if (!ws_grow_t(s, s->tlen + 1)) return 0;
    s->tcol[s->tlen] = j;
    s->tval[s->tlen] = -m;
    s->tlen++;
    int32_t jb = rp[j], je = rp[j + 1] - 1;
    if (!ws_grow_w(s, s->wlen + (je - jb)) || !ws_grow_i32(&s->heap, &s->hcap, s->hlen + (je - jb))) return 0;
    for (int32_t p = jb; p < je; ++p) {
      int32_t k = ci[p];
      int32_t sk = s->pos[k];
      if (sk < 0) {
        sk = s->wlen++;
        s->pos[k] = sk;
        s->wcol[sk] = k;
        s->wval[sk] = 0.0;
        s->alive[sk] = 1;
        if (cur[k] >= t) heap_push(s, k);
      }
      s->wval[sk] = s->wval[sk] - m * v[p];
    }
  }
  return 1;
}

static void ws_reset_pos(subst_ws *s) {
  for (int32_t q = 0; q < s->wlen; ++q) s->pos[s->wcol[q]] = -1;
}

static int32_t alive_count(const subst_ws *s) {
  int32_t a = 0;
  for (int32_t q = 0; q < s->wlen; ++q) a += s->alive[q];
  return a;
}

/* ---------------------------------------------------------------------------
 * O5. The decision scan of the naive strategy (Sec. III) plus the rewriting.
 *
 * Thin levels are the sources. With THIN_COST (metric 1) a level is thin when
 * its cost is below the threshold (avgLevelCost when threshold <= 0) and the
 * same number is the budget a target may reach; with THIN_ROWS (metric 0) a
 * level is thin when it has fewer than W rows and a target may hold W rows. A
 * level mask, when given, replaces the thin test. Level 0 is never a source.
 *
 * The scan starts with level 0 as the target. A non-source level becomes the
 * new target. The rows of a source level are taken in ascending order and each
 * is rewritten toward the current target; it is accepted while the target stays
 * within budget (and, optionally, the rewritten row stays within fill_cap times
 * its original nnz and the move is at most max_distance levels). The first row
 * that is refused stops the run and its level becomes the new target, with
 * every row of that level not moved; rows moved before it stay moved.
 *
 * Row constraints (Sec. III.A lists them as refinements of the level-wise
 * strategy): a row that passes the tests above is still left where it is,
 * without stopping the run, when its rewritten form has max_indeg or more
 * dependencies (indegree < alpha), when the columns of its rewritten form span
 * max_spread or more (distance between dependencies < beta, the locality
 * limit), or, with crit_only, when it is not on a longest path of the original
 * DAG (level + height = nlev - 1, height = longest path to a row nothing
 * depends on). Zero disables a limit.
 *
 * Per-level budgets and caps (the learned policy's actions, not in the
 * paper): lv_budget[l] > 0 replaces the row budget W for the rows of source
 * level l (THIN_ROWS: such a row is accepted while the target holds at most
 * lv_budget[l] rows after it), and lv_cap[l] > 0 replaces fill_cap for them.
 *
 * Outputs per row: tgt[r] = target level if the row was rewritten, else -1.
 * The rewritten rows are kept inside the returned context until collected.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t n;
  int32_t *lp_ptr, *lp_col;  /* L' CSR */
  double *lp_val;
  int32_t *t_ptr, *t_col;    /* T CSR */
  double *t_val;
  int64_t nnz_lp, nnz_t;
  int32_t rows_rewritten, max_distance;
  int32_t steps;             /* number of target steps */
  int32_t rows_skipped;      /* rows left in place by a row constraint */
} orc_rewrite_ctx;

typedef struct {
  int32_t *col;
  double *val;
  int32_t len;
} rowbuf;

void orc_rewrite_free(orc_rewrite_ctx *c) {
  if (!c) return;
  free(c->lp_ptr);
  free(c->lp_col);
  free(c->lp_val);
  free(c->t_ptr);
  free(c->t_col);
  free(c->t_val);
  free(c);
}

/* Sort (col, val) pairs of a row by column (insertion order is arbitrary). */
static void sort_pairs(int32_t *col, double *val, int32_t len) {
  for (int32_t i = 1; i < len; ++i) {
    int32_t c = col[i];
    double x = val[i];
    int32_t j = i - 1;
    while (j >= 0 && col[j] > c) {
      col[j + 1] = col[j];
      val[j + 1] = val[j];
      --j;
    }
    col[j + 1] = c;
    val[j + 1] = x;
  }
}

orc_rewrite_ctx *orc_rewrite_lv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nlev,
                                const int32_t *lev, const int32_t *level_ptr, const int32_t *level_rows,
                                int32_t thin_metric, double thin_threshold, double fill_cap, int32_t max_distance,
                                const uint8_t *mask, int32_t max_indeg, int64_t max_spread, int32_t crit_only,
                                int32_t both_ends, const int32_t *lv_budget, const float *lv_cap, int32_t *tgt,
                                int32_t *status) {
  *status = ORC_OK;
  int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nlev + 1));
  int64_t *nzl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nlev + 1));
  int64_t *cost = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nlev + 1));
  int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  rowbuf *lrow = (rowbuf *)calloc((size_t)(n + 1), sizeof(rowbuf));
  rowbuf *trow = (rowbuf *)calloc((size_t)(n + 1), sizeof(rowbuf));
  orc_rewrite_ctx *ctx = (orc_rewrite_ctx *)calloc(1, sizeof(orc_rewrite_ctx));
  subst_ws s;
  memset(&s, 0, sizeof(s));
  s.n = n;
  s.pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!rows || !nzl || !cost || !cur || !lrow || !trow || !ctx || !s.pos) {
    *status = ORC_ERR_ALLOC;
    return NULL;
  }
  for (int32_t k = 0; k < n; ++k) s.pos[k] = -1;
  int64_t total = 0;
  double avg = orc_level_costs(n, rp, nlev, level_ptr, level_rows, rows, nzl, cost, &total);
  double W = thin_threshold;
  if (thin_metric == 1 && W <= 0.0) W = avg;
  for (int32_t r = 0; r < n; ++r) {
    cur[r] = lev[r];
    tgt[r] = -1;
  }
  /* critical-path membership: heights by a sweep from the last row back (a
     row's dependents all come after it) */
  uint8_t *oncrit = NULL;
  if (crit_only) {
    int32_t *height = (int32_t *)calloc((size_t)(n + 1), sizeof(int32_t));
    oncrit = (uint8_t *)malloc((size_t)(n + 1));
    if (!height || !oncrit) {
      *status = ORC_ERR_ALLOC;
      return NULL;
    }
    for (int32_t r = n - 1; r >= 0; --r)
      for (int32_t p = rp[r]; p < rp[r + 1] - 1; ++p)
        if (height[ci[p]] < height[r] + 1) height[ci[p]] = height[r] + 1;
    for (int32_t r = 0; r < n; ++r) oncrit[r] = (uint8_t)(lev[r] + height[r] == nlev - 1);
    free(height);
  }
  int32_t skipped = 0;

  /* Segments: level 0 and every level that is not a source start one, and the
   * scan above runs inside each. A segment's scan neither reads nor changes
   * anything another one decides: its rows only move to levels inside it, and
   * a substitution expands only unknowns at or below the current target, while
   * every row of an earlier segment sits (moved or not) below the segment's
   * first level. So the segments may be taken in any order with the same
   * result; both_ends takes them alternately from the first and from the last
   * (first, last, second, second to last, ...), the scan started at the
   * beginning and at the end of the graph at once (Sec. III, the parallel
   * sketch; empty levels are only removed afterwards, so level numbers hold). */
  int32_t *seg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nlev + 1));
  if (!seg) {
    *status = ORC_ERR_ALLOC;
    return NULL;
  }
  int32_t nseg = 0;
  for (int32_t l = 0; l < nlev; ++l) {
    int src;
    if (l == 0)
      src = 0;
    else if (mask)
      src = mask[l] != 0;
    else if (thin_metric == 0)
      src = (double)rows[l] < W;
    else
      src = (double)cost[l] < W;
    if (!src) seg[nseg++] = l;
  }
  seg[nseg] = nlev;
  int32_t dist_max = 0, moved = 0, steps = 0;
  for (int32_t k = 0; k < nseg; ++k) {
    const int32_t sk = both_ends ? (k % 2 == 0 ? k / 2 : nseg - 1 - k / 2) : k;
    int32_t t = seg[sk];
    int64_t size_t_ = rows[t];
    int64_t cost_t = cost[t];
    steps++;
    for (int32_t l = seg[sk] + 1; l < seg[sk + 1]; ++l) {
      for (int32_t q = level_ptr[l]; q < level_ptr[l + 1]; ++q) {
        int32_t r = level_rows[q];
        if (!substitute(&s, rp, ci, v, cur, r, t)) {
          *status = ORC_ERR_ALLOC;
          return NULL;
        }
        int64_t nnz_new = (int64_t)alive_count(&s) + 1;
        int64_t nnz_old = rp[r + 1] - rp[r];
        /* a source level may carry its own budget (rows, THIN_ROWS) and fill
           cap; the budget bounds the target's size for the rows coming from
           that level */
        const double Wl = (thin_metric == 0 && lv_budget && lv_budget[l] > 0) ? (double)lv_budget[l] : W;
        const double capl = (lv_cap && lv_cap[l] > 0.0f) ? (double)lv_cap[l] : fill_cap;
        int ok;
        if (thin_metric == 0)
          ok = (double)(size_t_ + 1) <= Wl;
        else
          ok = (double)(cost_t + 2 * nnz_new - 1) <= W;
        if (capl > 0.0) ok = ok && (double)nnz_new <= capl * (double)nnz_old;
        if (max_distance > 0) ok = ok && (l - t) <= max_distance;
        if (ok) {
          int skip = 0;
          if (max_indeg > 0 && (int64_t)alive_count(&s) >= max_indeg) skip = 1;
          if (!skip && max_spread > 0) {
            int32_t lo = INT32_MAX, hi = -1;
            for (int32_t p = 0; p < s.wlen; ++p)
              if (s.alive[p]) {
                if (s.wcol[p] < lo) lo = s.wcol[p];
                if (s.wcol[p] > hi) hi = s.wcol[p];
              }
            if (hi >= 0 && (int64_t)hi - lo >= max_spread) skip = 1;
          }
          if (!skip && crit_only && !oncrit[r]) skip = 1;
          if (skip) { /* the row stays in its level; the run goes on */
            ws_reset_pos(&s);
            skipped += 1;
            continue;
          }
        }
        if (ok) {
          /* commit: L'[r] = surviving columns + diagonal, T[r] = eliminated + 1 */
          int32_t la = alive_count(&s);
          lrow[r].col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(la + 1));
          lrow[r].val = (double *)malloc(sizeof(double) * (size_t)(la + 1));
          trow[r].col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(s.tlen + 1));
          trow[r].val = (double *)malloc(sizeof(double) * (size_t)(s.tlen + 1));
          if (!lrow[r].col || !lrow[r].val || !trow[r].col || !trow[r].val) {
            *status = ORC_ERR_ALLOC;
            return NULL;
          }
          int32_t k = 0;
          for (int32_t p = 0; p < s.wlen; ++p)
            if (s.alive[p]) {
              lrow[r].col[k] = s.wcol[p];
              lrow[r].val[k] = s.wval[p];
              ++k;
            }
          sort_pairs(lrow[r].col, lrow[r].val, la);
          lrow[r].col[la] = r;
          lrow[r].val[la] = v[rp[r + 1] - 1];
          lrow[r].len = la + 1;
          memcpy(trow[r].col, s.tcol, sizeof(int32_t) * (size_t)s.tlen);
          memcpy(trow[r].val, s.tval, sizeof(double) * (size_t)s.tlen);
          sort_pairs(trow[r].col, trow[r].val, s.tlen);
          trow[r].col[s.tlen] = r;
          trow[r].val[s.tlen] = 1.0;
          trow[r].len = s.tlen + 1;
          ws_reset_pos(&s);
          cur[r] = t;
          tgt[r] = t;
          size_t_ += 1;
          cost_t += 2 * nnz_new - 1;
          moved += 1;
          if (l - t > dist_max) dist_max = l - t;
        } else {
          ws_reset_pos(&s);
          t = l;
          steps++;
          size_t_ = 0;
          cost_t = 0;
          for (int32_t q2 = level_ptr[l]; q2 < level_ptr[l + 1]; ++q2) {
            int32_t r2 = level_rows[q2];
            if (cur[r2] != l) continue; /* moved before the refusal */
            int64_t k2 = rp[r2 + 1] - rp[r2];
            size_t_ += 1;
            cost_t += 2 * k2 - 1;
          }
          break;
        }
      }
    }
  }
  free(seg);

  /* Assemble L' and T; rows never rewritten are copied (T row = unit). */
  ctx->n = n;
  ctx->lp_ptr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  ctx->t_ptr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!ctx->lp_ptr || !ctx->t_ptr) {
    *status = ORC_ERR_ALLOC;
    return NULL;
  }
  int64_t a = 0, bsum = 0;
  ctx->lp_ptr[0] = 0;
  ctx->t_ptr[0] = 0;
  for (int32_t r = 0; r < n; ++r) {
    a += lrow[r].col ? lrow[r].len : (rp[r + 1] - rp[r]);
    bsum += trow[r].col ? trow[r].len : 1;
    if (a > INT32_MAX || bsum > INT32_MAX) {
      *status = ORC_ERR_OVERFLOW;
      return NULL;
    }
    ctx->lp_ptr[r + 1] = (int32_t)a;
    ctx->t_ptr[r + 1] = (int32_t)bsum;
  }
  ctx->nnz_lp = a;
  ctx->nnz_t = bsum;
  ctx->lp_col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(a + 1));
  ctx->lp_val = (double *)malloc(sizeof(double) * (size_t)(a + 1));
  ctx->t_col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(bsum + 1));
  ctx->t_val = (double *)malloc(sizeof(double) * (size_t)(bsum + 1));
  if (!ctx->lp_col || !ctx->lp_val || !ctx->t_col || !ctx->t_val) {
    *status = ORC_ERR_ALLOC;
    return NULL;
  }
  for (int32_t r = 0; r < n; ++r) {
    int32_t o = ctx->lp_ptr[r];
    if (lrow[r].col) {
      memcpy(ctx->lp_col + o, lrow[r].col, sizeof(int32_t) * (size_t)lrow[r].len);
      memcpy(ctx->lp_val + o, lrow[r].val, sizeof(double) * (size_t)lrow[r].len);
    } else {
      memcpy(ctx->lp_col + o, ci + rp[r], sizeof(int32_t) * (size_t)(rp[r + 1] - rp[r]));
      memcpy(ctx->lp_val + o, v + rp[r], sizeof(double) * (size_t)(rp[r + 1] - rp[r]));
    }
    int32_t ot = ctx->t_ptr[r];
    if (trow[r].col) {
      memcpy(ctx->t_col + ot, trow[r].col, sizeof(int32_t) * (size_t)trow[r].len);
      memcpy(ctx->t_val + ot, trow[r].val, sizeof(double) * (size_t)trow[r].len);
    } else {
      ctx->t_col[ot] = r;
      ctx->t_val[ot] = 1.0;
    }
    free(lrow[r].col);
    free(lrow[r].val);
    free(trow[r].col);
    free(trow[r].val);
  }
  ctx->rows_rewritten = moved;
  ctx->max_distance = dist_max;
  ctx->steps = steps;
  ctx->rows_skipped = skipped;
  free(oncrit);
  free(rows);
  free(nzl);
  free(cost);
  free(cur);
  free(lrow);
  free(trow);
  free(s.pos);
  free(s.wcol);
  free(s.wval);
  free(s.alive);
  free(s.heap);
  free(s.tcol);
  free(s.tval);
  return ctx;
}

orc_rewrite_ctx *orc_rewrite_rc(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nlev,
                                const int32_t *lev, const int32_t *level_ptr, const int32_t *level_rows,
                                int32_t thin_metric, double thin_threshold, double fill_cap, int32_t max_distance,
                                const uint8_t *mask, int32_t max_indeg, int64_t max_spread, int32_t crit_only,
                                int32_t both_ends, int32_t *tgt, int32_t *status) {
  return orc_rewrite_lv(n, rp, ci, v, nlev, lev, level_ptr, level_rows, thin_metric, thin_threshold, fill_cap,
                        max_distance, mask, max_indeg, max_spread, crit_only, both_ends, NULL, NULL, tgt, status);
}

orc_rewrite_ctx *orc_rewrite(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nlev,
                             const int32_t *lev, const int32_t *level_ptr, const int32_t *level_rows,
                             int32_t thin_metric, double thin_threshold, double fill_cap, int32_t max_distance,
                             const uint8_t *mask, int32_t *tgt, int32_t *status) {
  return orc_rewrite_rc(n, rp, ci, v, nlev, lev, level_ptr, level_rows, thin_metric, thin_threshold, fill_cap,
                        max_distance, mask, 0, 0, 0, 0, tgt, status);
}

int32_t orc_rewrite_skipped(const orc_rewrite_ctx *c) { return c->rows_skipped; }

void orc_rewrite_sizes(const orc_rewrite_ctx *c, int64_t *nnz_lp, int64_t *nnz_t, int32_t *rows_rewritten,
                       int32_t *max_distance, int32_t *steps) {
  *nnz_lp = c->nnz_lp;
  *nnz_t = c->nnz_t;
  *rows_rewritten = c->rows_rewritten;
  *max_distance = c->max_distance;
  *steps = c->steps;
}

void orc_rewrite_copy(const orc_rewrite_ctx *c, int32_t *lp_ptr, int32_t *lp_col, double *lp_val, int32_t *t_ptr,
                      int32_t *t_col, double *t_val) {
  memcpy(lp_ptr, c->lp_ptr, sizeof(int32_t) * (size_t)(c->n + 1));
  memcpy(lp_col, c->lp_col, sizeof(int32_t) * (size_t)c->nnz_lp);
  memcpy(lp_val, c->lp_val, sizeof(double) * (size_t)c->nnz_lp);
  memcpy(t_ptr, c->t_ptr, sizeof(int32_t) * (size_t)(c->n + 1));
  memcpy(t_col, c->t_col, sizeof(int32_t) * (size_t)c->nnz_t);
  memcpy(t_val, c->t_val, sizeof(double) * (size_t)c->nnz_t);
}

/* ---------------------------------------------------------------------------
 * Per-level features for the learned rewrite policy (20 per level, FP64 here).
 * None of these come from the paper; they summarise the quantities its strategy
 * discussion names as relevant (level cost against avgLevelCost, number of
 * dependencies, growth of a row when it is rewritten; Sec. III and Sec. III.A):
 *   0 log1p(rows)            1 log1p(sum nnz)        2 log1p(cost)
 *   3 cost / avgLevelCost    4 rows / 32             5 sum nnz / rows
 *   6..11 fraction of rows with 0, 1, 2, 3-4, 5-8, >=9 off-diagonals
 *   12 sum nnz(L'[r]) / sum nnz(L[r]) if the level were rewritten into the
 *      level before it (every other row in place)    13 log1p(sum nnz(T[r])) of that move
 *   14 level / nlev          15 log1p(rows of the level before)
 * and the row constraints of Sec. III.A, measured on the same move:
 *   16 fraction of rows whose moved form keeps fewer than 4 off-diagonals
 *      (indegree < alpha, alpha = 4)
 *   17 fraction of rows on a longest path of the DAG (level + height = nlev - 1,
 *      height = longest path from the row to a row nothing depends on)
 *   18 log1p(mean over rows of the moved form's off-diagonal column span,
 *      largest minus smallest column; 0 for a row with fewer than two)
 *   19 fraction of rows whose moved form spans fewer than 1024 columns
 *      (dependency spread < beta, beta = 1024: the x values a row reads lie
 *      within 8 KB)
 * For level 0 features 12..13 and 16..19 are those of an identity move (the
 * row as it is: 1 and log1p(rows) for 12..13) and feature 15 is 0.
 * ------------------------------------------------------------------------- */
int orc_level_features(int32_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t nlev,
                       const int32_t *lev, const int32_t *level_ptr, const int32_t *level_rows, double *feat) {
  int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nlev + 1));
  int64_t *nzl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nlev + 1));
  int64_t *cost = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nlev + 1));
  subst_ws s;
  memset(&s, 0, sizeof(s));
  s.n = n;
  s.pos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!rows || !nzl || !cost || !s.pos) return ORC_ERR_ALLOC;
  for (int32_t k = 0; k < n; ++k) s.pos[k] = -1;
  int32_t *height = (int32_t *)calloc((size_t)(n + 1), sizeof(int32_t));
  if (!height) return ORC_ERR_ALLOC;
  /* a row's dependents all come after it: one sweep from the last row back */
  for (int32_t r = n - 1; r >= 0; --r)
    for (int32_t p = rp[r]; p < rp[r + 1] - 1; ++p)
      if (height[ci[p]] < height[r] + 1) height[ci[p]] = height[r] + 1;
  int64_t total = 0;
  double avg = orc_level_costs(n, rp, nlev, level_ptr, level_rows, rows, nzl, cost, &total);
  for (int32_t l = 0; l < nlev; ++l) {
    double *f = feat + (int64_t)l * ORC_NFEAT;
    int64_t hist[6] = {0, 0, 0, 0, 0, 0};
    int64_t sum_lp = 0, sum_l = 0, sum_t = 0;
    int64_t n_alpha = 0, n_crit = 0, n_local = 0, sum_span = 0;
    for (int32_t q = level_ptr[l]; q < level_ptr[l + 1]; ++q) {
      int32_t r = level_rows[q];
      int32_t off = rp[r + 1] - rp[r] - 1;
      int bin = off == 0 ? 0 : off == 1 ? 1 : off == 2 ? 2 : off <= 4 ? 3 : off <= 8 ? 4 : 5;
      hist[bin] += 1;
      sum_l += off + 1;
      int32_t na, lo = INT32_MAX, hi = -1;
      if (l == 0) {
        sum_lp += off + 1;
        sum_t += 1;
        na = off;
        for (int32_t p = rp[r]; p < rp[r + 1] - 1; ++p) {
          if (ci[p] < lo) lo = ci[p];
          if (ci[p] > hi) hi = ci[p];
        }
      } else {
        if (!substitute(&s, rp, ci, v, lev, r, l - 1)) return ORC_ERR_ALLOC;
        na = alive_count(&s);
        sum_lp += na + 1;
        sum_t += s.tlen + 1;
        for (int32_t p = 0; p < s.wlen; ++p)
          if (s.alive[p]) {
            if (s.wcol[p] < lo) lo = s.wcol[p];
            if (s.wcol[p] > hi) hi = s.wcol[p];
          }
        ws_reset_pos(&s);
      }
      const int64_t span = hi >= 0 ? (int64_t)hi - lo : 0;
      n_alpha += na < 4;
      n_crit += lev[r] + height[r] == nlev - 1;
      sum_span += span;
      n_local += span < 1024;
    }
    double R = (double)rows[l];
    f[0] = log1p(R);
    f[1] = log1p((double)nzl[l]);
    f[2] = log1p((double)cost[l]);
    f[3] = avg > 0.0 ? (double)cost[l] / avg : 0.0;
    f[4] = R / 32.0;
    f[5] = R > 0.0 ? (double)nzl[l] / R : 0.0;
    for (int b = 0; b < 6; ++b) f[6 + b] = R > 0.0 ? (double)hist[b] / R : 0.0;
    f[12] = sum_l > 0 ? (double)sum_lp / (double)sum_l : 0.0;
    f[13] = log1p((double)sum_t);
    f[14] = (double)l / (double)nlev;
    f[15] = l > 0 ? log1p((double)rows[l - 1]) : 0.0;
    f[16] = R > 0.0 ? (double)n_alpha / R : 0.0;
    f[17] = R > 0.0 ? (double)n_crit / R : 0.0;
    f[18] = R > 0.0 ? log1p((double)sum_span / R) : 0.0;
    f[19] = R > 0.0 ? (double)n_local / R : 0.0;
  }
  free(height);
  free(rows);
  free(nzl);
  free(cost);
  free(s.pos);
  free(s.wcol);
  free(s.wval);
  free(s.alive);
  free(s.heap);
  free(s.tcol);
  free(s.tval);
  return ORC_OK;
}
