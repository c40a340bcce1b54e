// Internal declarations of the single-problem driver (gencd_solver.hip)
// shared with the server: set-up of one problem in a carved workspace and
// the FP64 check, also in an enqueue-then-fold form for callers that must
// not wait on the stream.
#pragma once

#include <vector>

#include "gencd_common.hpp"

namespace gencd {

// The check's reduction block as copied to the host (16 words).
struct Red {
  double loss_sum, l1;
  unsigned long long kkt_bits, nnz_w;
  unsigned long long gmax_bits;
  double dual_sum;
  unsigned long long pad[2];
  unsigned long long acc_nnz, acc_cnt, bad, spare;
  unsigned long long pad2[4];
};
static_assert(sizeof(Red) == 16 * 8, "reduction block layout");

struct Setup {
  Ws ws{};
  int piece = kDefaultPiece, group = kDefaultGroup;
  int32_t n_short = 0, n_lpieces = 0;
  int64_t k_live = 0;
  std::vector<double> rho_hist;  // spectral-radius estimate after each power iteration
  double rho = 0.0;
  std::vector<double> brho;      // Block Shotgun: rho_b of every preset block
  std::vector<int32_t> bp;       // Block Shotgun: P_b* of every preset block
};

struct CheckOut {
  double objective, kkt, gap;
  int64_t nnz_w;
  unsigned long long acc_nnz, acc_cnt;
  double drift_rel;  // re-syncing checks: max_i |z_i - z64_i| / rms(z64) (0 if z64 = 0)
};

bool csc_ok(const gencd_csc *X);
bool wants_rho(const gencd_params *p);
int params_ok(const gencd_params *p, bool need_rule);
int64_t pstar_of(int64_t k_live, double rho);
double bits_to_double(unsigned long long b);

// Preprocessing: validation, piece decomposition, live columns, curvature
// and (rho_iters > 0) the spectral-radius estimate.  Writes only the
// workspace; synchronises the stream.  y may be null only when need_y is
// false (no label check).
int setup(const gencd_csc *X, const float *y, int loss, const gencd_params *p, void *ws_base,
          size_t ws_bytes, bool validate_matrix, hipStream_t s, Setup *out, int rho_iters = 0,
          bool need_y = true, int64_t nblocks = 0, int block_iters = kRhoIters);

// FP64 check of w (z64 = Xw, objective, KKT, duality gap; resync: the FP32
// state from z64).  enqueue_check leaves the replica lines (kChkRep * 16
// doubles) and the reduction block in host memory once the stream reaches
// them; fold_check combines them.  run_check does both and waits.
int enqueue_check(const gencd_csc *X, const float *y, int loss, double lam, const float *w,
                  const Setup &su, bool resync, hipStream_t s, double *host_rep, Red *host_red);
void fold_check(const double *rep, const Red &red, int64_t n, double lam, CheckOut *out);
int run_check(const gencd_csc *X, const float *y, int loss, double lam, const float *w,
              const Setup &su, bool resync, hipStream_t s, CheckOut *out);

}  // namespace gencd
