/* Test driver for a sanitizer build of the oracle (AddressSanitizer and
 * UndefinedBehaviorSanitizer, host code only): runs every oracle entry point
 * on small seeded matrices and on malformed inputs, and checks what the
 * mathematics fixes (x = 1 for b = L 1, the rewritten system's x equals the
 * original's, levels free of internal dependencies). Built and run by
 * tests/test_oracle_sanitize.py; prints "OK" and exits 0 when every check
 * passes and the sanitizers report nothing. */
#include "../oracle/oracle.c"

#include <stdio.h>

static uint64_t lcg_state = 0x9e3779b97f4a7c15ull;
static uint64_t lcg(void) {
  lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
  return lcg_state >> 11;
}
static double unif(void) { return (double)(lcg() >> 11) / 9007199254740992.0 * 2.0 - 1.0; }

typedef struct {
  int32_t n, nnz;
  int32_t *rp, *ci;
  double *v;
} csr;

/* Row i reads up to `draws` distinct columns from [max(0, i - window), i - 1];
 * diagonal 1 + sum |off| (strictly dominant). */
static csr window_matrix(int32_t n, int32_t window, int draws, uint64_t seed) {
  lcg_state = seed;
  csr m;
  m.n = n;
  m.rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  m.ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)(draws + 1));
  m.v = (double *)malloc(sizeof(double) * (size_t)n * (size_t)(draws + 1));
  int32_t nnz = 0;
  m.rp[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    int32_t cols[64];
    int k = 0;
    const int32_t lo = i - window > 0 ? i - window : 0;
    for (int d = 0; d < draws && i > 0; ++d) {
      const int32_t c = lo + (int32_t)(lcg() % (uint64_t)(i - lo));
      int dup = 0;
      for (int j = 0; j < k; ++j) dup |= cols[j] == c;
      if (!dup) cols[k++] = c;
    }
    for (int a = 1; a < k; ++a)
      for (int b = a; b > 0 && cols[b - 1] > cols[b]; --b) {
        const int32_t t = cols[b];
        cols[b] = cols[b - 1];
        cols[b - 1] = t;
      }
    double s = 0.0;
    for (int j = 0; j < k; ++j) {
      m.ci[nnz] = cols[j];
      m.v[nnz] = unif();
      s += fabs(m.v[nnz]);
      ++nnz;
    }
    m.ci[nnz] = i;
    m.v[nnz] = 1.0 + s;
    ++nnz;
    m.rp[i + 1] = nnz;
  }
  m.nnz = nnz;
  return m;
}

static int fails = 0;
#define CHECK(cond, ...)                    \
  do {                                      \
    if (!(cond)) {                          \
      fprintf(stderr, "FAIL: " __VA_ARGS__); \
      fputc('\n', stderr);                  \
      ++fails;                              \
    }                                       \
  } while (0)

static void exercise(const csr *m, const char *name) {
  const int32_t n = m->n;
  CHECK(orc_validate(n, m->nnz, m->rp, m->ci, m->v) == ORC_OK, "%s: validate", name);
  /* x = 1 for b = L 1 */
  double *one = (double *)malloc(sizeof(double) * (size_t)n * 2);
  double *b = (double *)malloc(sizeof(double) * (size_t)n * 2);
  double *x = (double *)malloc(sizeof(double) * (size_t)n * 2);
  double *x2 = (double *)malloc(sizeof(double) * (size_t)n * 2);
  double *bp = (double *)malloc(sizeof(double) * (size_t)n * 2);
  for (int32_t i = 0; i < 2 * n; ++i) one[i] = 1.0;
  orc_spmv(n, m->rp, m->ci, m->v, 2, one, n, b, n);
  orc_solve(n, m->rp, m->ci, m->v, 2, b, n, x, n);
  for (int32_t i = 0; i < 2 * n; ++i) CHECK(fabs(x[i] - 1.0) < 1e-12, "%s: x != 1 at %d", name, i);
  for (int32_t i = 0; i < 2 * n; ++i) b[i] = unif();
  orc_solve(n, m->rp, m->ci, m->v, 2, b, n, x, n);
  /* levels, costs */
  int32_t *lev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  int32_t *lp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 2));
  int32_t *lr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  const int32_t nlev = orc_levels(n, m->rp, m->ci, lev, lp, lr);
  for (int32_t r = 0; r < n; ++r)
    for (int32_t p = m->rp[r]; p < m->rp[r + 1] - 1; ++p)
      CHECK(lev[m->ci[p]] < lev[r], "%s: dependency inside or after a level at row %d", name, r);
  int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nlev + 1));
  int64_t *nzl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nlev + 1));
  int64_t *cost = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nlev + 1));
  int64_t total = 0;
  const double avg = orc_level_costs(n, m->rp, nlev, lp, lr, rows, nzl, cost, &total);
  CHECK(avg > 0.0 && total == 2 * (int64_t)m->nnz - n, "%s: cost model", name);
  /* features */
  double *feat = (double *)malloc(sizeof(double) * (size_t)nlev * ORC_NFEAT);
  CHECK(orc_level_features(n, m->rp, m->ci, m->v, nlev, lev, lp, lr, feat) == ORC_OK, "%s: features", name);
  /* rewrites under several option sets: x from (L', T b) equals x from (L, b) */
  struct {
    int32_t metric;
    double thr, cap;
    int32_t dist, indeg;
    int64_t spread;
    int32_t crit, both;
    int mask;
  } opts[] = {{0, 32.0, 4.0, 0, 0, 0, 0, 0, 0}, {1, 0.0, 0.0, 0, 0, 0, 0, 0, 0}, {1, 0.0, 0.0, 9, 0, 0, 0, 1, 0},
              {0, 1e9, 0.0, 0, 4, 0, 0, 0, 0},  {1, 0.0, 0.0, 0, 0, 64, 1, 0, 0}, {0, 16.0, 2.0, 3, 0, 0, 0, 1, 1}};
  uint8_t *mask = (uint8_t *)malloc((size_t)nlev + 1);
  for (int32_t l = 0; l < nlev; ++l) mask[l] = (uint8_t)(l > 0 && (lcg() & 1));
  int32_t *tgt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  for (size_t k = 0; k < sizeof(opts) / sizeof(opts[0]); ++k) {
    int32_t st = 0;
    orc_rewrite_ctx *c = orc_rewrite_rc(n, m->rp, m->ci, m->v, nlev, lev, lp, lr, opts[k].metric, opts[k].thr,
                                        opts[k].cap, opts[k].dist, opts[k].mask ? mask : NULL, opts[k].indeg,
                                        opts[k].spread, opts[k].crit, opts[k].both, tgt, &st);
    CHECK(c && st == ORC_OK, "%s: rewrite %zu status %d", name, k, st);
    if (!c) continue;
    int64_t a = 0, t = 0;
    int32_t rr = 0, md = 0, steps = 0;
    orc_rewrite_sizes(c, &a, &t, &rr, &md, &steps);
    int32_t *lpp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *lpc = (int32_t *)malloc(sizeof(int32_t) * (size_t)a);
    double *lpv = (double *)malloc(sizeof(double) * (size_t)a);
    int32_t *tp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *tc = (int32_t *)malloc(sizeof(int32_t) * (size_t)t);
    double *tv = (double *)malloc(sizeof(double) * (size_t)t);
    orc_rewrite_copy(c, lpp, lpc, lpv, tp, tc, tv);
    CHECK(orc_validate(n, (int32_t)a, lpp, lpc, lpv) == ORC_OK, "%s: rewrite %zu gives an invalid L'", name, k);
    orc_spmv(n, tp, tc, tv, 2, b, n, bp, n);
    orc_solve(n, lpp, lpc, lpv, 2, bp, n, x2, n);
    double num = 0.0, den = 0.0;
    for (int32_t i = 0; i < 2 * n; ++i) {
      num = fmax(num, fabs(x2[i] - x[i]));
      den = fmax(den, fabs(x[i]));
    }
    CHECK(num <= 1e-10 * den, "%s: rewrite %zu changes x (%g)", name, k, num / den);
    free(lpp);
    free(lpc);
    free(lpv);
    free(tp);
    free(tc);
    free(tv);
    orc_rewrite_free(c);
  }
  free(one);
  free(b);
  free(x);
  free(x2);
  free(bp);
  free(lev);
  free(lp);
  free(lr);
  free(rows);
  free(nzl);
  free(cost);
  free(feat);
  free(mask);
  free(tgt);
}

int main(void) {
  const struct {
    int32_t n, window;
    int draws;
    uint64_t seed;
  } cases[] = {{1, 1, 1, 1}, {2, 1, 1, 2}, {300, 64, 5, 3}, {500, 6, 3, 4}, {800, 1, 1, 5}, {400, 400, 8, 6}};
  for (size_t k = 0; k < sizeof(cases) / sizeof(cases[0]); ++k) {
    csr m = window_matrix(cases[k].n, cases[k].window, cases[k].draws, cases[k].seed);
    char name[64];
    snprintf(name, sizeof(name), "window n=%d w=%d", cases[k].n, cases[k].window);
    exercise(&m, name);
    free(m.rp);
    free(m.ci);
    free(m.v);
  }
  /* malformed inputs are refused without reading out of bounds */
  {
    int32_t rp[4] = {0, 1, 3, 4};
    int32_t ci_bad[4] = {0, 1, 0, 2}; /* row 1 unsorted */
    double v[4] = {1.0, 2.0, 3.0, 4.0};
    CHECK(orc_validate(3, 4, rp, ci_bad, v) == ORC_ERR_UNSORTED, "unsorted row not refused");
    int32_t ci_up[4] = {0, 2, 1, 2}; /* column above the diagonal */
    CHECK(orc_validate(3, 4, rp, ci_up, v) == ORC_ERR_NOT_LOWER, "upper entry not refused");
    int32_t rp_bad[4] = {0, 2, 1, 4};
    int32_t ci_ok[4] = {0, 0, 1, 2};
    CHECK(orc_validate(3, 4, rp_bad, ci_ok, v) == ORC_ERR_ARG, "decreasing row pointer not refused");
    double vz[4] = {1.0, 2.0, 0.0, 4.0};
    CHECK(orc_validate(3, 4, rp, ci_ok, vz) == ORC_ERR_ZERO_PIVOT, "zero pivot not refused");
  }
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("OK\n");
  return 0;
}
