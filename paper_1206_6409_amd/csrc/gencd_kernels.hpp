// Kernel argument blocks and launchers (implemented in gencd_kernels.hip).
#pragma once

#include "gencd_common.hpp"

namespace gencd {

// Everything one iteration's kernels read or write.  Passed by value.
struct IterArgs {
  const int64_t *col_ptr;
  const int32_t *row_idx;
  const float *val;
  const float *y;
  float n_f;
  int32_t loss;
  float lam;
  int32_t piece;
  const float *c;
  float *w;
  float *z_hi, *z_lo, *r;
  const int32_t *col_of_pos, *poff, *piece_pos;
  const int32_t *win_off;  // per-epoch window offsets, or null: [win_lo, win_hi)
  int32_t t, win_lo, win_hi;
  float *delta, *phi, *gacc, *gout;
  int32_t *tick, *acc;
  unsigned long long *counters;  // [0] accepted nnz, [1] accepted proposals, [3] fused-update nnz
};

int fill_f32(float *p, int64_t m, float v, hipStream_t s);
int fill_i32(int32_t *p, int64_t m, int32_t v, hipStream_t s);
int fill_f64(double *p, int64_t m, double v, hipStream_t s);
int copy_f32(float *d, const float *src, int64_t m, hipStream_t s);
int copy_i32(int32_t *d, const int32_t *src, int64_t m, hipStream_t s);

int launch_validate(const gencd_csc *X, const float *y, int loss, bool matrix,
                    unsigned long long *bad, hipStream_t s);
int launch_preprocess(const gencd_csc *X, int loss, int piece, const Ws &w, hipStream_t s);
int launch_curvature(const gencd_csc *X, int loss, int piece, int32_t total_pieces, const Ws &w,
                     hipStream_t s);
int launch_select_perm(int64_t m, uint64_t seed, int64_t epoch, int32_t *out, hipStream_t s);
int launch_epoch_order(const Ws &w, int64_t k_live, int rule, uint64_t seed, int64_t epoch,
                       int64_t num_colors, hipStream_t s);
int launch_list_order(const Ws &w, const int32_t *J, int64_t nJ, hipStream_t s);
int launch_refresh_all(int64_t n, int loss, const float *y, const float *z_hi, const float *z_lo,
                       float *r, hipStream_t s);
int launch_iteration(const IterArgs &a, int group, int mode, int64_t block, int64_t groups,
                     int64_t nblocks_accept, bool deferred_work, hipStream_t s,
                     hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
int launch_check(const gencd_csc *X, const float *y, int loss, double lam, const float *w,
                 int piece, int32_t total_pieces, const Ws &ws, bool resync, hipStream_t s);
int launch_round_f32(const double *src, float *dst, int64_t m, hipStream_t s);

}  // namespace gencd
