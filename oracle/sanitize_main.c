/*
 * Sanitizer driver for the FP64 oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Runs every entry point of the oracle on small seeded problems, including
 * an empty column, an empty matrix and one-row / one-column shapes, so that a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitized.py) sees every code path touch its buffers.
 * The oracle source is compiled into this translation unit.
 */
#include <stdio.h>

#include "gencd_oracle.c"

static uint64_t g_state;
static double urand(void) {
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return ((double)(g_state >> 11) + 0.5) * 0x1.0p-53;
}

typedef struct {
  orc_csc X;
  int64_t *cp;
  int32_t *ri;
  double *v, *y;
} problem;

/* Bernoulli(d) pattern, column 0 left empty; N(0,1)-like values. */
static problem make(int64_t n, int64_t k, double d, int loss, uint64_t seed) {
  problem P;
  g_state = seed;
  P.cp = (int64_t *)calloc((size_t)k + 1, sizeof(int64_t));
  int64_t cap = n * k + 1;
  P.ri = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
  P.v = (double *)malloc(sizeof(double) * (size_t)cap);
  P.y = (double *)malloc(sizeof(double) * (size_t)n);
  int64_t e = 0;
  for (int64_t j = 0; j < k; ++j) {
    for (int64_t i = 0; i < n && j > 0; ++i)
      if (urand() < d) {
        P.ri[e] = (int32_t)i;
        P.v[e] = (urand() - 0.5) * 3.0 + (urand() < 0.5 ? 0.25 : -0.25);
        ++e;
      }
    P.cp[j + 1] = e;
  }
  for (int64_t i = 0; i < n; ++i)
    P.y[i] = loss == ORC_LOGISTIC ? (urand() < 0.5 ? -1.0 : 1.0) : urand() * 2.0 - 1.0;
  P.X.n = n;
  P.X.k = k;
  P.X.nnz = e;
  P.X.col_ptr = P.cp;
  P.X.row_idx = P.ri;
  P.X.val = P.v;
  return P;
}

static void release(problem *P) {
  free(P->cp);
  free(P->ri);
  free(P->v);
  free(P->y);
}

static int run_case(int64_t n, int64_t k, double d, int loss, uint64_t seed) {
  problem P = make(n, k, d, loss, seed);
  const orc_csc *X = &P.X;
  double lmax = orc_lambda_max(X, P.y, loss);
  double lam = 0.2 * lmax;
  double *w = (double *)calloc((size_t)k, sizeof(double));
  double *z = (double *)calloc((size_t)n, sizeof(double));
  double *g = (double *)calloc((size_t)k, sizeof(double));
  int32_t *color = (int32_t *)calloc((size_t)k, sizeof(int32_t));
  int32_t *order = (int32_t *)calloc((size_t)k, sizeof(int32_t));
  int32_t *bal = (int32_t *)calloc((size_t)k, sizeof(int32_t));
  int32_t nc = 0;
  int bad = 0;
  if (orc_color(n, k, P.cp, P.ri, 0, color, &nc, order) != ORC_OK) bad |= 1;
  int32_t nb = orc_balance_colors(k, P.cp, color, nc > 0 ? nc : 1, 0, bal);
  if (nb < 1) bad |= 2;
  double hist[32];
  int64_t k_live = 0;
  double rho = orc_rho(X, 20, hist, &k_live);
  int64_t S = orc_pstar(k_live, rho, k_live > 0 ? k_live : 1);
  if (k_live > 0) {
    int64_t nblk = k_live < 3 ? k_live : 3;
    double brho[3];
    int64_t bp[3];
    if (orc_block_pstar(X, 7, nblk, 10, brho, bp) != ORC_OK) bad |= 4;
  }
  for (int rule = ORC_CYCLIC; rule <= ORC_BLOCK_SHOTGUN; ++rule) {
    for (int improve = 0; improve <= 3; improve += 3) {
      orc_params p;
      memset(&p, 0, sizeof(p));
      p.loss = loss;
      p.rule = rule;
      p.lambda = lam;
      p.select_size = S > 0 ? S : 1;
      p.block = rule == ORC_BLOCK_SHOTGUN ? 2 : (rule == ORC_TOP_GREEDY ? 3 : 2);
      p.seed = 11;
      p.tol = 1e-8;
      p.max_epochs = 2000;
      p.check_every = 1;
      p.color = color;
      p.num_colors = nc;
      p.improve = improve;
      orc_stats st;
      memset(w, 0, sizeof(double) * (size_t)k);
      int rc = orc_solve(X, P.y, &p, w, z, &st);
      if (rc != ORC_OK && rc != ORC_NOT_CONVERGED) bad |= 8;
      double kkt, obj;
      int64_t nz;
      orc_check(X, P.y, loss, lam, w, z, g, &kkt, &obj, &nz);
      double prim;
      (void)orc_duality_gap(X, P.y, loss, lam, w, &prim);
      if (!(obj == obj)) bad |= 16;
    }
  }
  /* one step with every output and a forced acceptance */
  if (k > 1) {
    double *c = (double *)calloc((size_t)k, sizeof(double));
    orc_curvature(X, loss, c);
    int32_t J[2] = {0, (int32_t)(k - 1)}, forced[2] = {0, 1}, acc[2];
    double go[2], dout[2], pout[2];
    int64_t nu = 0;
    if (orc_step(X, P.y, loss, lam, c, J, 2, 2, 0, 2, forced, w, z, go, dout, pout, acc, &nu) != ORC_OK)
      bad |= 32;
    free(c);
  }
  free(w);
  free(z);
  free(g);
  free(color);
  free(order);
  free(bal);
  release(&P);
  return bad;
}

int main(void) {
  int bad = 0;
  bad |= run_case(40, 30, 0.15, ORC_LOGISTIC, 1);
  bad |= run_case(25, 60, 0.1, ORC_SQUARED, 2);
  bad |= run_case(1, 5, 0.9, ORC_SQUARED, 3);   /* one row */
  bad |= run_case(12, 2, 0.5, ORC_LOGISTIC, 4); /* one live column */
  bad |= run_case(8, 6, 0.0, ORC_SQUARED, 5);   /* empty matrix */
  if (bad) {
    printf("failed: %d\n", bad);
    return 1;
  }
  printf("ok\n");
  return 0;
}
