/*
 * FP64 sequential oracle for GenCD (Scherrer, Halappanavar, Tewari, Haglin,
 * "Scaling Up Coordinate Descent Algorithms for Large l1 Regularization
 * Problems").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the HIP library: it is written
 * independently from the paper so that the two can be compared.
 *
 * Everything here is plain, sequential and double precision.  Matrices are
 * CSC (col_ptr int64[k+1], row_idx int32[nnz], val double[nnz]).  The caller
 * promotes the FP32 data to double exactly, so both sides solve the same
 * problem.
 *
 * Readings of the paper where it is silent (all documented in the design
 * notes of the repository):
 *   - l'(y,t) and l''(y,t) are derivatives in the fitted value t (section 3).
 *   - The per-coordinate curvature bound is c_j = beta * ||X_j||^2 / n
 *     (beta = 1 squared loss, 1/4 logistic; section 3.2).  It equals beta
 *     under the column normalisation of section 4.4 and H_jj exactly for
 *     squared loss (Eq. 4).  Empty columns (c_j = 0) propose 0.
 *   - Propose is synchronous (Jacobi): every proposal of an iteration reads
 *     the state at the start of that iteration.
 *   - Random subsets are windows of a per-epoch pseudo-random permutation of
 *     the non-empty columns: a keyed 4-round Feistel bijection on the next
 *     even power of two with cycle-walking (Black & Rogaway, 2002); the round
 *     function is the SplitMix64 finaliser (Steele, Lea & Flood, 2014).
 *   - Thread-Greedy accepts, in each block of B consecutive window positions,
 *     the first position with minimal phi (section 4.1, Table 2).
 *   - Coloring visits the colours of an epoch in the permuted order; within
 *     a colour the members are updated in column order.
 *   - The greedy colouring visits columns by decreasing nnz, ties by index,
 *     and gives each column the smallest colour not used by an already
 *     coloured column sharing a row (partial distance-2 colouring, 4.1).
 *   - Convergence: max_j KKT violation <= tol, evaluated in FP64 from a
 *     fresh z = Xw at the end of every check_every epochs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EDIVERGED (-3)

#define ORC_SQUARED 0
#define ORC_LOGISTIC 1

#define ORC_CYCLIC 0
#define ORC_STOCHASTIC 1
#define ORC_SHOTGUN 2
#define ORC_THREAD_GREEDY 3
#define ORC_GREEDY 4
#define ORC_COLORING 5
#define ORC_TOP_GREEDY 6 /* Thread-Greedy accepting the best |J'| of the window */
#define ORC_BLOCK_SHOTGUN 7 /* Shotgun inside preset blocks, |J| = P_b* per block */

typedef struct {
  int64_t n, k, nnz;
  const int64_t *col_ptr;
  const int32_t *row_idx;
  const double *val;
} orc_csc;

typedef struct {
  int32_t loss;
  int32_t rule;
  double lambda;
  int64_t select_size; /* |J| for Shotgun / Thread-Greedy */
  int64_t block;       /* Thread-Greedy block size B */
  uint64_t seed;
  double tol;
  int64_t max_epochs;
  int64_t check_every; /* epochs between convergence checks */
  const int32_t *color; /* Coloring: colour of every column */
  int32_t num_colors;
  int32_t improve;      /* extra quadratic-approximation steps per accepted proposal */
} orc_params;

typedef struct {
  int64_t iters, epochs, coord_updates, nnz_updates;
  double objective, kkt_max;
  int64_t nnz_w;
  int32_t converged;
} orc_stats;

/* ------------------------------------------------------------------------ */
/* Loss functions (section 1): squared 1/2 (y-t)^2, logistic log(1+e^{-yt}) */
/* ------------------------------------------------------------------------ */

double orc_loss(int loss, double y, double t) {
  if (loss == ORC_SQUARED) {
    double d = y - t;
    return 0.5 * d * d;
  }
  double m = y * t; /* log(1+exp(-m)) = max(-m,0) + log1p(exp(-|m|)) */
  return (m > 0.0 ? 0.0 : -m) + log1p(exp(-fabs(m)));
}

double orc_dloss(int loss, double y, double t) {
  if (loss == ORC_SQUARED) return t - y;
  double m = y * t; /* d/dt log(1+exp(-yt)) = -y / (1 + exp(yt)) */
  double s;
  if (m >= 0.0) {
    double e = exp(-m);
    s = e / (1.0 + e);
  } else {
    s = 1.0 / (1.0 + exp(m));
  }
  return -y * s;
}

double orc_beta(int loss) { return loss == ORC_SQUARED ? 1.0 : 0.25; }

/* ------------------------------------------------------------------------ */
/* Pseudo-random selection                                                   */
/* ------------------------------------------------------------------------ */

uint64_t orc_mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

/* One 4-round balanced Feistel encryption of x on 2*half bits. */
static uint64_t feistel(uint64_t x, int half, const uint64_t key[4]) {
  uint64_t mask = (half == 32) ? 0xFFFFFFFFull : ((1ull << half) - 1ull);
  uint64_t L = x >> half, R = x & mask;
  for (int r = 0; r < 4; ++r) {
    uint64_t F = orc_mix64(R ^ key[r]) & mask;
    uint64_t nl = R;
    R = L ^ F;
    L = nl;
  }
  return (L << half) | R;
}

/* pi_e(p) for p in [0, m): position p of epoch e's permutation of m items. */
int64_t orc_perm(int64_t m, uint64_t seed, int64_t epoch, int64_t p) {
  int bits = 2;
  while ((1ll << bits) < m) bits += 2;
  int half = bits / 2;
  uint64_t key[4];
  for (int r = 0; r < 4; ++r)
    key[r] = orc_mix64(seed + 0x9E3779B97F4A7C15ull * (uint64_t)(epoch * 8 + r + 1));
  uint64_t x = (uint64_t)p;
  do {
    x = feistel(x, half, key);
  } while (x >= (uint64_t)m);
  return (int64_t)x;
}

/* ------------------------------------------------------------------------ */
/* Building blocks of Algorithm 1                                            */
/* ------------------------------------------------------------------------ */

/* Curvature bound c_j = beta * ||X_j||^2 / n (section 3.2). */
void orc_curvature(const orc_csc *X, int loss, double *c) {
  double beta = orc_beta(loss);
  for (int64_t j = 0; j < X->k; ++j) {
    double s = 0.0;
    for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) s += X->val[p] * X->val[p];
    c[j] = beta * s / (double)X->n;
  }
}

/* lambda_max = max_j |X_j^T l'(y, 0)| / n: the smallest lambda for which
 * w = 0 satisfies the optimality conditions of Eq. 1. */
double orc_lambda_max(const orc_csc *X, const double *y, int loss) {
  double best = 0.0;
  for (int64_t j = 0; j < X->k; ++j) {
    double g = 0.0;
    for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p)
      g += X->val[p] * orc_dloss(loss, y[X->row_idx[p]], 0.0);
    g = fabs(g) / (double)X->n;
    if (g > best) best = g;
  }
  return best;
}

/* Proposal via the quadratic upper bound (Algorithm 4, Eq. 7 and Eq. 9) for
 * a coordinate with gradient g, curvature c and current weight w. */
void orc_propose(double g, double c, double w, double lambda, double *delta, double *phi) {
  if (!(c > 0.0)) {
    *delta = 0.0;
    *phi = 0.0;
    return;
  }
  double a = (g - lambda) / c; /* clip interval of Eq. 4 / Eq. 7 */
  double b = (g + lambda) / c;
  double psi = w < a ? a : (w > b ? b : w);
  double d = -psi;
  *delta = d;
  *phi = 0.5 * c * d * d + g * d + lambda * (fabs(w + d) - fabs(w));
}

/* One GenCD iteration (Algorithm 1) on the selected set J[0..nJ).
 *   Propose (Algorithm 2 / 4): g_j, delta_j, phi_j for every j in J, all from
 *     the state at entry.
 *   Accept (section 2.3): block == 0 accepts all; otherwise in each block of
 *     `block` consecutive positions the first position with minimal phi.  If
 *     `forced` is given, forced[b] (an absolute position, or -1 for none)
 *     replaces the choice of block b.
 *   Update (Algorithm 3): in ascending position, w_j += delta_j and
 *     z += delta_j X_j.
 * Optional outputs g/delta/phi (length nJ) and acc (0/1 per position). */
/* Order of window positions for the global accept: by proxy, ties to the
 * lower position. */
static const double *g_top_phi;
static int cmp_top(const void *a, const void *b) {
  int64_t ta = *(const int64_t *)a, tb = *(const int64_t *)b;
  if (g_top_phi[ta] < g_top_phi[tb]) return -1;
  if (g_top_phi[ta] > g_top_phi[tb]) return 1;
  return ta < tb ? -1 : (ta > tb ? 1 : 0);
}

/* One Jacobi iteration on the window J (Algorithm 1).  Accept:
 *   top > 0:   the `top` proposals with the smallest phi over the whole
 *              window (Thread-Greedy with global acceptance, section 4.1);
 *   block > 0: in each block of `block` consecutive positions the first
 *              position with minimal phi (Thread-Greedy, Greedy);
 *   otherwise every proposal (Shotgun, Coloring, CCD). */
/* "Improve delta_j" (Algorithm 3, section 4.1): up to `steps` further steps
 * of the quadratic approximation on the one-dimensional objective
 *   f_j(d) = (1/n) sum_i l(y_i, z_i + d x_ij) + lambda |w_j + d|
 * along column j, from d = delta and the state z of the iteration start:
 *   g = (1/n) sum_i x_ij l'(y_i, z_i + d x_ij),
 *   d <- d + (Eq. 7 increment at the point w_j + d with gradient g).
 * The loop stops once a step no longer changes d (in the arithmetic's own
 * precision): from there every further step would repeat it. */
static double improve_delta(const orc_csc *X, const double *y, int loss, double lambda, double c,
                            int64_t j, double wj, const double *z, double d, int32_t steps) {
  if (d == 0.0) return d;
  for (int32_t s = 0; s < steps; ++s) {
    double g = 0.0;
    for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) {
      int32_t i = X->row_idx[p];
      g += X->val[p] * orc_dloss(loss, y[i], z[i] + d * X->val[p]);
    }
    g /= (double)X->n;
    double inc, unused;
    orc_propose(g, c, wj + d, lambda, &inc, &unused);
    double dn = d + inc;
    if (dn == d) break; /* the step no longer changes the increment */
    d = dn;
  }
  return d;
}

int orc_step(const orc_csc *X, const double *y, int loss, double lambda, const double *c,
             const int32_t *J, int64_t nJ, int64_t block, int64_t top, int32_t improve,
             const int32_t *forced, double *w, double *z, double *g_out, double *d_out,
             double *p_out, int32_t *acc_out, int64_t *nnz_updates) {
  if (nJ < 0) return ORC_EINVAL;
  for (int64_t t = 0; t < nJ; ++t)
    if (J[t] < 0 || J[t] >= X->k) return ORC_EINVAL;
  double *d = (double *)malloc(sizeof(double) * (size_t)(nJ > 0 ? nJ : 1));
  double *ph = (double *)malloc(sizeof(double) * (size_t)(nJ > 0 ? nJ : 1));
  int32_t *acc = (int32_t *)calloc((size_t)(nJ > 0 ? nJ : 1), sizeof(int32_t));
  if (!d || !ph || !acc) {
    free(d);
    free(ph);
    free(acc);
    return ORC_ENOMEM;
  }
  /* Propose */
  for (int64_t t = 0; t < nJ; ++t) {
    int64_t j = J[t];
    double g = 0.0;
    for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) {
      int32_t i = X->row_idx[p];
      g += orc_dloss(loss, y[i], z[i]) * X->val[p];
    }
    g /= (double)X->n;
    orc_propose(g, c[j], w[j], lambda, &d[t], &ph[t]);
    if (g_out) g_out[t] = g;
  }
  /* Accept */
  if (top > 0) {
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nJ > 0 ? nJ : 1));
    if (!ord) {
      free(d);
      free(ph);
      free(acc);
      return ORC_ENOMEM;
    }
    for (int64_t t = 0; t < nJ; ++t) ord[t] = t;
    g_top_phi = ph;
    qsort(ord, (size_t)nJ, sizeof(int64_t), cmp_top);
    for (int64_t t = 0; t < nJ && t < top; ++t) acc[ord[t]] = 1;
    if (forced) { /* forced accept set: positions listed in forced[0..top) */
      for (int64_t t = 0; t < nJ; ++t) acc[t] = 0;
      for (int64_t t = 0; t < top && t < nJ; ++t)
        if (forced[t] >= 0 && forced[t] < nJ) acc[forced[t]] = 1;
    }
    free(ord);
  } else if (block <= 0) {
    for (int64_t t = 0; t < nJ; ++t) acc[t] = 1;
  } else {
    int64_t nb = (nJ + block - 1) / block;
    for (int64_t b = 0; b < nb; ++b) {
      int64_t lo = b * block, hi = lo + block < nJ ? lo + block : nJ;
      int64_t best = lo;
      for (int64_t t = lo + 1; t < hi; ++t)
        if (ph[t] < ph[best]) best = t;
      if (forced) best = forced[b];
      if (best >= lo && best < hi) acc[best] = 1;
    }
  }
  /* Update: every accepted proposal is improved against the iteration-start
   * state first (the loop of Algorithm 3 is parallel), then applied */
  if (improve > 0)
    for (int64_t t = 0; t < nJ; ++t)
      if (acc[t]) d[t] = improve_delta(X, y, loss, lambda, c[J[t]], J[t], w[J[t]], z, d[t], improve);
  int64_t nu = 0;
  for (int64_t t = 0; t < nJ; ++t) {
    if (!acc[t]) continue;
    int64_t j = J[t];
    nu += X->col_ptr[j + 1] - X->col_ptr[j];
    if (d[t] == 0.0) continue;
    w[j] += d[t];
    for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) z[X->row_idx[p]] += d[t] * X->val[p];
  }
  if (nnz_updates) *nnz_updates = nu;
  if (d_out) memcpy(d_out, d, sizeof(double) * (size_t)nJ);
  if (p_out) memcpy(p_out, ph, sizeof(double) * (size_t)nJ);
  if (acc_out) memcpy(acc_out, acc, sizeof(int32_t) * (size_t)nJ);
  free(d);
  free(ph);
  free(acc);
  return ORC_OK;
}

/* Objective of Eq. 1, gradient of F (section 3) and the KKT violation
 *   v_j = |g_j + lambda sign(w_j)|  (w_j != 0),  max(|g_j| - lambda, 0)  (w_j = 0)
 * evaluated from a fresh z = Xw.  z_out (n) and g_out (k) are optional. */
void orc_check(const orc_csc *X, const double *y, int loss, double lambda, const double *w,
               double *z_out, double *g_out, double *kkt_max, double *objective, int64_t *nnz_w) {
  double *z = (double *)calloc((size_t)(X->n > 0 ? X->n : 1), sizeof(double));
  for (int64_t j = 0; j < X->k; ++j) {
    if (w[j] == 0.0) continue;
    for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) z[X->row_idx[p]] += w[j] * X->val[p];
  }
  double lsum = 0.0;
  for (int64_t i = 0; i < X->n; ++i) lsum += orc_loss(loss, y[i], z[i]);
  double l1 = 0.0, vmax = 0.0;
  int64_t nz = 0;
  for (int64_t j = 0; j < X->k; ++j) {
    double g = 0.0;
    for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) {
      int32_t i = X->row_idx[p];
      g += orc_dloss(loss, y[i], z[i]) * X->val[p];
    }
    g /= (double)X->n;
    if (g_out) g_out[j] = g;
    double v;
    if (w[j] != 0.0) {
      v = fabs(g + (w[j] > 0 ? lambda : -lambda));
      l1 += fabs(w[j]);
      ++nz;
    } else {
      v = fabs(g) - lambda;
      if (v < 0.0) v = 0.0;
    }
    if (v > vmax) vmax = v;
  }
  if (objective) *objective = lsum / (double)X->n + lambda * l1;
  if (kkt_max) *kkt_max = vmax;
  if (nnz_w) *nnz_w = nz;
  if (z_out) memcpy(z_out, z, sizeof(double) * (size_t)X->n);
  free(z);
}

/* Duality gap of Eq. 1 at w (an upper bound on the suboptimality of w).
 * Fenchel dual of min f(Xw) + lambda |w|_1 with f(z) = (1/n) sum l(y_i, z_i):
 *   D(u) = -(1/n) sum_i l*(y_i, n u_i)  subject to  |X^T u|_inf <= lambda,
 * evaluated at the scaled residual u = s l'(y, Xw) / n with
 * s = min(1, lambda / |X^T l'(y, Xw) / n|_inf).  Conjugates:
 *   squared:   l*(y, v) = v y + v^2 / 2
 *   logistic:  l*(y, v) = p log p + (1 - p) log(1 - p),  p = -v y in [0, 1].
 * Returns P(w) - D(u); *primal receives P(w). */
double orc_duality_gap(const orc_csc *X, const double *y, int loss, double lambda, const double *w,
                       double *primal) {
  int64_t n = X->n;
  double *z = (double *)calloc((size_t)n, sizeof(double));
  double *r = (double *)malloc(sizeof(double) * (size_t)n);
  for (int64_t j = 0; j < X->k; ++j) {
    if (w[j] == 0.0) continue;
    for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) z[X->row_idx[p]] += w[j] * X->val[p];
  }
  double lsum = 0.0, l1 = 0.0, gmax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    lsum += orc_loss(loss, y[i], z[i]);
    r[i] = orc_dloss(loss, y[i], z[i]);
  }
  for (int64_t j = 0; j < X->k; ++j) {
    double g = 0.0;
    for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) g += X->val[p] * r[X->row_idx[p]];
    g = fabs(g) / (double)n;
    if (g > gmax) gmax = g;
    l1 += fabs(w[j]);
  }
  double s = (gmax > lambda) ? lambda / gmax : 1.0;
  double dsum = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double v = s * r[i]; /* n u_i */
    if (loss == ORC_SQUARED) {
      dsum -= v * y[i] + 0.5 * v * v;
    } else {
      double p = -v * y[i];
      double h = 0.0;
      if (p > 0.0) h -= p * log(p);
      if (p < 1.0) h -= (1.0 - p) * log1p(-p);
      dsum += h;
    }
  }
  double P = lsum / (double)n + lambda * l1;
  if (primal) *primal = P;
  free(z);
  free(r);
  return P - dsum / (double)n;
}

/* ------------------------------------------------------------------------ */
/* Spectral radius of the column-normalised Gram matrix (section 4.1)         */
/* ------------------------------------------------------------------------ */

/* Shotgun is guaranteed to converge when it selects at most P* = k/(2 rho)
 * coordinates, rho the largest eigenvalue of X^T X for columns scaled to unit
 * norm (section 4.1, after Bradley et al. 2011).  Here
 *   G = D^{-1/2} X^T X D^{-1/2},  D = diag(X^T X),
 * restricted to the non-empty columns, and rho is estimated by power
 * iteration from the unit vector with equal entries on those columns:
 *   u = G v,  rho_t = ||u||_2,  v <- u / rho_t,   t = 1..iters.
 * Returns rho_iters (0 if every column is empty); hist[t-1] = rho_t when hist
 * is non-null; *k_live receives the number of non-empty columns. */
/* The same restricted to the columns with in_set[j] != 0 (all when NULL). */
double orc_rho_subset(const orc_csc *X, const uint8_t *in_set, int32_t iters, double *hist,
                      int64_t *k_live) {
  int64_t n = X->n, k = X->k, kl = 0;
  double *dinv = (double *)calloc((size_t)k, sizeof(double)); /* D^{-1/2}, 0 on empty columns */
  double *v = (double *)calloc((size_t)k, sizeof(double));
  double *s = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int64_t j = 0; j < k; ++j) {
    if (in_set && !in_set[j]) continue;
    double q = 0.0;
    for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) q += X->val[p] * X->val[p];
    if (q > 0.0) {
      dinv[j] = 1.0 / sqrt(q);
      ++kl;
    }
  }
  if (k_live) *k_live = kl;
  double rho = 0.0;
  if (kl > 0) {
    for (int64_t j = 0; j < k; ++j) v[j] = dinv[j] > 0.0 ? 1.0 / sqrt((double)kl) : 0.0;
    for (int32_t t = 0; t < iters; ++t) {
      /* s = X D^{-1/2} v */
      for (int64_t i = 0; i < n; ++i) s[i] = 0.0;
      for (int64_t j = 0; j < k; ++j) {
        double xj = dinv[j] * v[j];
        for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) s[X->row_idx[p]] += X->val[p] * xj;
      }
      /* u = D^{-1/2} X^T s (stored in v), rho = ||u|| */
      double nrm = 0.0;
      for (int64_t j = 0; j < k; ++j) {
        double u = 0.0;
        for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) u += X->val[p] * s[X->row_idx[p]];
        v[j] = dinv[j] * u;
        nrm += v[j] * v[j];
      }
      rho = sqrt(nrm);
      if (hist) hist[t] = rho;
      if (rho == 0.0) break;
      for (int64_t j = 0; j < k; ++j) v[j] /= rho;
    }
  }
  free(dinv);
  free(v);
  free(s);
  return rho;
}

double orc_rho(const orc_csc *X, int32_t iters, double *hist, int64_t *k_live) {
  return orc_rho_subset(X, NULL, iters, hist, k_live);
}

/* Selection size from the estimate: floor(k_live / (2 rho)), clamped to
 * [1, cap]. */
int64_t orc_pstar(int64_t k_live, double rho, int64_t cap) {
  if (!(rho > 0.0)) return 1;
  double q = floor((double)k_live / (2.0 * rho));
  if (q < 1.0) return 1;
  if (q > (double)cap) return cap;
  return (int64_t)q;
}

/* ------------------------------------------------------------------------ */
/* Block Shotgun (section 7): preset random blocks with their own P_b*        */
/* ------------------------------------------------------------------------ */

/* Key of the preset partition and of the within-block orders. */
static uint64_t block_seed(uint64_t seed, int64_t b) {
  return orc_mix64(seed ^ orc_mix64(0x626c6f636b73ull + (uint64_t)(b + 1)));
}

/* Preset blocks: the non-empty columns in the order of the seeded
 * permutation (epoch 0 of block_seed(seed, -1)) are cut into nb contiguous
 * ranges [b k_live / nb, (b+1) k_live / nb).  base[q] is the column at
 * preset position q (k_live entries); returns k_live. */
int64_t orc_block_base(const orc_csc *X, uint64_t seed, int32_t *base) {
  int64_t kl = 0;
  int32_t *live = (int32_t *)malloc(sizeof(int32_t) * (size_t)(X->k > 0 ? X->k : 1));
  for (int64_t j = 0; j < X->k; ++j)
    if (X->col_ptr[j + 1] > X->col_ptr[j]) live[kl++] = (int32_t)j;
  for (int64_t q = 0; q < kl; ++q) base[q] = live[orc_perm(kl, block_seed(seed, -1), 0, q)];
  free(live);
  return kl;
}

static int64_t block_lo(int64_t b, int64_t kl, int64_t nb) { return b * kl / nb; }

/* rho_b (power iteration, `iters` steps) and P_b* = floor(k_b / (2 rho_b))
 * clamped to [1, k_b] for every preset block; nb in [1, k_live]. */
int orc_block_pstar(const orc_csc *X, uint64_t seed, int64_t nb, int32_t iters, double *rho_out,
                    int64_t *pstar_out) {
  int32_t *base = (int32_t *)malloc(sizeof(int32_t) * (size_t)(X->k > 0 ? X->k : 1));
  uint8_t *in_set = (uint8_t *)calloc((size_t)X->k, 1);
  int64_t kl = orc_block_base(X, seed, base);
  if (nb < 1 || nb > kl) {
    free(base);
    free(in_set);
    return ORC_EINVAL;
  }
  for (int64_t b = 0; b < nb; ++b) {
    int64_t lo = block_lo(b, kl, nb), hi = block_lo(b + 1, kl, nb);
    for (int64_t q = lo; q < hi; ++q) in_set[base[q]] = 1;
    int64_t kb = 0;
    double r = orc_rho_subset(X, in_set, iters, NULL, &kb);
    for (int64_t q = lo; q < hi; ++q) in_set[base[q]] = 0;
    int64_t p = 1;
    if (r > 0.0) {
      double f = floor((double)kb / (2.0 * r));
      p = f < 1.0 ? 1 : (f > (double)kb ? kb : (int64_t)f);
    }
    rho_out[b] = r;
    pstar_out[b] = p;
  }
  free(base);
  free(in_set);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Greedy partial distance-2 colouring of the column conflict graph           */
/* ------------------------------------------------------------------------ */

static const int64_t *g_sort_nnz;
static int cmp_priority(const void *a, const void *b) {
  int32_t ja = *(const int32_t *)a, jb = *(const int32_t *)b;
  int64_t na = g_sort_nnz[ja], nb = g_sort_nnz[jb];
  if (na != nb) return na > nb ? -1 : 1; /* more nonzeros first */
  return ja < jb ? -1 : (ja > jb ? 1 : 0);
}

/* order_mode 0: decreasing nnz, ties by column index; 1: column index.
 * color[k] receives colours 0..num_colors-1; order[k] (optional) the visit
 * order. */
int orc_color(int64_t n, int64_t k, const int64_t *col_ptr, const int32_t *row_idx, int order_mode,
              int32_t *color, int32_t *num_colors, int32_t *order_out) {
  if (n < 0 || k < 0) return ORC_EINVAL;
  int64_t nnz = col_ptr[k];
  int64_t *row_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *col_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
  int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k + 2));
  if (!row_ptr || !col_idx || !fill || !cnt || !order || !mark) {
    free(row_ptr); free(col_idx); free(fill); free(cnt); free(order); free(mark);
    return ORC_ENOMEM;
  }
  /* rows -> columns (the bipartite graph seen from the rows) */
  for (int64_t p = 0; p < nnz; ++p) row_ptr[row_idx[p] + 1]++;
  for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
  for (int64_t i = 0; i < n; ++i) fill[i] = row_ptr[i];
  for (int64_t j = 0; j < k; ++j)
    for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p) col_idx[fill[row_idx[p]]++] = (int32_t)j;
  for (int64_t j = 0; j < k; ++j) {
    cnt[j] = col_ptr[j + 1] - col_ptr[j];
    order[j] = (int32_t)j;
    color[j] = -1;
  }
  if (order_mode == 0) {
    g_sort_nnz = cnt;
    qsort(order, (size_t)k, sizeof(int32_t), cmp_priority);
  }
  for (int64_t c = 0; c < k + 2; ++c) mark[c] = -1;
  int32_t ncol = 0;
  for (int64_t t = 0; t < k; ++t) {
    int32_t j = order[t];
    /* colours of coloured columns that share a row with j */
    for (int64_t p = col_ptr[j]; p < col_ptr[j + 1]; ++p) {
      int32_t i = row_idx[p];
      for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
        int32_t c = color[col_idx[q]];
        if (c >= 0) mark[c] = j;
      }
    }
    int32_t c = 0;
    while (mark[c] == j) ++c;
    color[j] = c;
    if (c + 1 > ncol) ncol = c + 1;
  }
  *num_colors = ncol;
  if (order_out) memcpy(order_out, order, sizeof(int32_t) * (size_t)k);
  free(row_ptr); free(col_idx); free(fill); free(cnt); free(order); free(mark);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Full solve: Algorithm 1 with the rules of Table 2                         */
/* ------------------------------------------------------------------------ */

/* Selected set J for iteration t of epoch e.  Returns its size. */
/* Balanced colouring (section 4.1 Coloring, "more colours, even class
 * sizes"): every class of more than `cap` live columns is split into
 * parts = ceil(size / cap) parts; the member of rank r (column order) goes
 * to part floor(r * parts / size).  A part of an independent set is
 * independent, so the result is a valid colouring with classes of at most
 * cap columns.  New colours are numbered class by class, parts in order.
 * cap <= 0 takes the mean class size ceil(k_live / C).  Empty columns keep
 * their colour's first part.  Returns the number of colours. */
int32_t orc_balance_colors(int64_t k, const int64_t *col_ptr, const int32_t *color, int32_t C,
                           int64_t cap, int32_t *out) {
  int64_t *size = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
  int64_t *parts = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
  int64_t *first = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
  int64_t *seen = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
  int64_t kl = 0;
  for (int64_t j = 0; j < k; ++j)
    if (col_ptr[j + 1] > col_ptr[j]) {
      size[color[j]]++;
      kl++;
    }
  if (cap <= 0) cap = C > 0 ? (kl + C - 1) / C : 1;
  if (cap < 1) cap = 1;
  int64_t total = 0;
  for (int32_t c = 0; c < C; ++c) {
    parts[c] = size[c] > cap ? (size[c] + cap - 1) / cap : 1;
    first[c] = total;
    total += parts[c];
  }
  for (int64_t j = 0; j < k; ++j) {
    int32_t c = color[j];
    if (col_ptr[j + 1] > col_ptr[j]) {
      int64_t r = seen[c]++;
      out[j] = (int32_t)(first[c] + r * parts[c] / size[c]);
    } else {
      out[j] = (int32_t)first[c];
    }
  }
  free(size);
  free(parts);
  free(first);
  free(seen);
  return (int32_t)total;
}

static int64_t select_set(const orc_params *P, int64_t k_live, const int32_t *live,
                          const int64_t *cls_off, const int32_t *cls_mem, int32_t ncls, int64_t e,
                          int64_t t, int32_t *J) {
  if (P->rule == ORC_CYCLIC) {
    J[0] = live[t];
    return 1;
  }
  if (P->rule == ORC_COLORING) {
    int64_t c = orc_perm(ncls, P->seed, e, t);
    int64_t m = cls_off[c + 1] - cls_off[c];
    memcpy(J, cls_mem + cls_off[c], sizeof(int32_t) * (size_t)m);
    return m;
  }
  int64_t s = (P->rule == ORC_STOCHASTIC) ? 1 : (P->rule == ORC_GREEDY ? k_live : P->select_size);
  int64_t lo = t * s, hi = lo + s < k_live ? lo + s : k_live;
  for (int64_t p = lo; p < hi; ++p) J[p - lo] = live[orc_perm(k_live, P->seed, e, p)];
  return hi - lo;
}

int orc_solve(const orc_csc *X, const double *y, const orc_params *P, double *w, double *z_out,
              orc_stats *st) {
  memset(st, 0, sizeof(*st));
  if (X->n <= 0 || X->k <= 0 || P->lambda < 0) return ORC_EINVAL;
  int rule = P->rule;
  if (rule < ORC_CYCLIC || rule > ORC_BLOCK_SHOTGUN) return ORC_EINVAL;
  if (rule == ORC_BLOCK_SHOTGUN && P->block <= 0) return ORC_EINVAL;
  if ((rule == ORC_SHOTGUN || rule == ORC_THREAD_GREEDY || rule == ORC_TOP_GREEDY) &&
      P->select_size <= 0)
    return ORC_EINVAL;
  if ((rule == ORC_THREAD_GREEDY || rule == ORC_TOP_GREEDY) && P->block <= 0) return ORC_EINVAL;
  if (rule == ORC_COLORING && (!P->color || P->num_colors <= 0)) return ORC_EINVAL;

  int64_t n = X->n, k = X->k;
  double *c = (double *)malloc(sizeof(double) * (size_t)k);
  double *z = (double *)malloc(sizeof(double) * (size_t)n);
  int32_t *live = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
  int32_t *J = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
  int64_t *cls_off = NULL;
  int32_t *cls_mem = NULL;
  int32_t ncls = 0;
  if (!c || !z || !live || !J) {
    free(c); free(z); free(live); free(J);
    return ORC_ENOMEM;
  }
  orc_curvature(X, P->loss, c);
  int64_t k_live = 0;
  for (int64_t j = 0; j < k; ++j)
    if (X->col_ptr[j + 1] > X->col_ptr[j]) live[k_live++] = (int32_t)j;

  if (rule == ORC_COLORING) {
    /* colour classes: live members of each colour, in column order */
    ncls = P->num_colors;
    cls_off = (int64_t *)calloc((size_t)ncls + 1, sizeof(int64_t));
    cls_mem = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k_live > 0 ? k_live : 1));
    for (int64_t t = 0; t < k_live; ++t) cls_off[P->color[live[t]] + 1]++;
    for (int32_t q = 0; q < ncls; ++q) cls_off[q + 1] += cls_off[q];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncls);
    for (int32_t q = 0; q < ncls; ++q) fill[q] = cls_off[q];
    for (int64_t t = 0; t < k_live; ++t) cls_mem[fill[P->color[live[t]]]++] = live[t];
    free(fill);
  }

  /* z = Xw for the starting point (a warm start or zero) */
  memset(z, 0, sizeof(double) * (size_t)n);
  for (int64_t j = 0; j < k; ++j)
    if (w[j] != 0.0)
      for (int64_t p = X->col_ptr[j]; p < X->col_ptr[j + 1]; ++p) z[X->row_idx[p]] += w[j] * X->val[p];

  int64_t block = (rule == ORC_THREAD_GREEDY) ? P->block : (rule == ORC_GREEDY ? k_live : 0);
  int64_t top = (rule == ORC_TOP_GREEDY) ? P->block : 0;
  /* Block Shotgun: preset blocks and their P_b* (20 power iterations) */
  int64_t nblk = 0;
  int32_t *bbase = NULL;
  int64_t *bp = NULL;
  double *brho = NULL;
  if (rule == ORC_BLOCK_SHOTGUN && k_live > 0) {
    nblk = P->block < k_live ? P->block : k_live;
    bbase = (int32_t *)malloc(sizeof(int32_t) * (size_t)k_live);
    bp = (int64_t *)malloc(sizeof(int64_t) * (size_t)nblk);
    brho = (double *)malloc(sizeof(double) * (size_t)nblk);
    orc_block_base(X, P->seed, bbase);
    orc_block_pstar(X, P->seed, nblk, 20, brho, bp);
  }
  int64_t per_epoch;
  if (rule == ORC_CYCLIC || rule == ORC_STOCHASTIC) per_epoch = k_live;
  else if (rule == ORC_COLORING) per_epoch = ncls;
  else if (rule == ORC_GREEDY) per_epoch = 1;
  else if (rule == ORC_BLOCK_SHOTGUN) per_epoch = 0; /* windows come from the blocks */
  else per_epoch = (k_live + P->select_size - 1) / P->select_size;
  int64_t check_every = P->check_every > 0 ? P->check_every : 1;

  int status = ORC_NOT_CONVERGED;
  double last_obj = INFINITY;
  for (int64_t e = 0; e < P->max_epochs && k_live > 0; ++e) {
    /* Block Shotgun epoch: blocks in a per-epoch permuted order; inside
     * block b its members in a per-epoch permuted order, windows of P_b* */
    for (int64_t u = 0; u < nblk; ++u) {
      int64_t b = orc_perm(nblk, P->seed, e, u);
      int64_t lo = block_lo(b, k_live, nblk), kb = block_lo(b + 1, k_live, nblk) - lo;
      for (int64_t t0 = 0; t0 < kb; t0 += bp[b]) {
        int64_t m = kb - t0 < bp[b] ? kb - t0 : bp[b];
        for (int64_t i = 0; i < m; ++i)
          J[i] = bbase[lo + orc_perm(kb, block_seed(P->seed, b), e, t0 + i)];
        int64_t nu = 0;
        orc_step(X, y, P->loss, P->lambda, c, J, m, 0, 0, P->improve, NULL, w, z, NULL, NULL,
                 NULL, NULL, &nu);
        st->iters++;
        st->coord_updates += m;
        st->nnz_updates += nu;
      }
    }
    for (int64_t t = 0; t < per_epoch; ++t) {
      int64_t m = select_set(P, k_live, live, cls_off, cls_mem, ncls, e, t, J);
      if (m == 0) continue;
      int64_t nu = 0;
      orc_step(X, y, P->loss, P->lambda, c, J, m, block, top, P->improve, NULL, w, z, NULL, NULL,
               NULL, NULL, &nu);
      st->iters++;
      st->coord_updates += top > 0 ? (m < top ? m : top) : (block > 0 ? (m + block - 1) / block : m);
      st->nnz_updates += nu;
    }
    st->epochs = e + 1;
    if ((e + 1) % check_every == 0 || e + 1 == P->max_epochs) {
      double kkt, obj;
      int64_t nz;
      orc_check(X, y, P->loss, P->lambda, w, z, NULL, &kkt, &obj, &nz);
      st->objective = obj;
      st->kkt_max = kkt;
      st->nnz_w = nz;
      if (!isfinite(obj)) {
        status = ORC_EDIVERGED;
        break;
      }
      last_obj = obj;
      if (kkt <= P->tol) {
        status = ORC_OK;
        st->converged = 1;
        break;
      }
    }
  }
  (void)last_obj;
  if (k_live == 0) {
    double kkt, obj;
    int64_t nz;
    orc_check(X, y, P->loss, P->lambda, w, z, NULL, &kkt, &obj, &nz);
    st->objective = obj;
    st->kkt_max = kkt;
    st->nnz_w = nz;
    st->converged = kkt <= P->tol;
    status = st->converged ? ORC_OK : ORC_NOT_CONVERGED;
  }
  if (z_out) memcpy(z_out, z, sizeof(double) * (size_t)n);
  free(c); free(z); free(live); free(J); free(cls_off); free(cls_mem);
  free(bbase); free(bp); free(brho);
  return status;
}
