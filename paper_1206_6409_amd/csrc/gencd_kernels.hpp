// Kernel argument blocks and launchers (implemented in gencd_kernels.hip).
#pragma once

#include "gencd_common.hpp"

namespace gencd {

// Everything one iteration's kernels read or write.  Passed by value.
struct IterArgs {
  const int64_t *col_ptr;
  const int32_t *row_idx;
  const float *val;
  float n_f;
  int32_t loss;
  float lam;
  const float *c;
  float *w;
  float4 *zs;                      // {z_hi, z_lo, y, 0} per row
  float *rs;                       // non-null: refresh l'(y, z) into rs, Propose reads it
  int64_t nrows;
  const int32_t *col_of_pos;
  const int32_t *loff;             // long-piece offsets of the positions
  const int4 *desc_s;              // descriptor of every position (length 0: long column)
  const int4 *desc_l;              // long-piece descriptors of the current order
  const int32_t *wbl;              // window t: long pieces [wbl[t], wbl[t+1])
  int32_t nl;                      // waves walking long pieces (set by the launcher)
  int32_t piece;                   // nonzeros per long piece
  int64_t accept_top;              // > 0: deferred acceptance of the best accept_top of the window
  int32_t improve;                 // extra quadratic-approximation steps per accepted proposal
  const int32_t *win_off;  // per-epoch window offsets, or null: [win_lo, win_hi)
  int32_t t, win_lo, win_hi;
  float *delta, *phi, *gacc, *gout, *wsnap;
  int32_t *acc;
  int32_t *bw_pos, *bw_phi;  // per-chunk winners of a two-stage global accept (scratch)
  int32_t exact_accum;     // 1: TwoSum per update (returning atomics); 0: low-word accumulation
  unsigned long long *counters;  // [0] accepted nnz, [1] accepted proposals (greedy rules)
  unsigned long long *scat;      // non-null: Update adds the nonzeros it scatters here
                                 // (replica line b % kChkRep of workgroup b, 16 words each)
};

int fill_f32(float *p, int64_t m, float v, hipStream_t s);
int fill_i32(int32_t *p, int64_t m, int32_t v, hipStream_t s);
int fill_f64(double *p, int64_t m, double v, hipStream_t s);
int copy_f32(float *d, const float *src, int64_t m, hipStream_t s);
int copy_i32(int32_t *d, const int32_t *src, int64_t m, hipStream_t s);

int launch_validate(const gencd_csc *X, const float *y, int loss, bool matrix,
                    unsigned long long *bad, hipStream_t s);
int launch_preprocess(const gencd_csc *X, int loss, int piece, int short_max, const Ws &w,
                      hipStream_t s);
int launch_curvature(const gencd_csc *X, int loss, int32_t n_short, int32_t n_lpieces,
                     const Ws &w, hipStream_t s);
int launch_select_perm(int64_t m, uint64_t seed, int64_t epoch, int32_t *out, hipStream_t s);
// Writes the epoch order, its piece descriptors and, in w.wbounds[0..T], the
// first piece of every window (S positions per window; colour windows for
// COLORING).
int launch_epoch_order(const Ws &w, int64_t k_live, int rule, uint64_t seed,
                       const int64_t *epoch, int64_t num_colors, int64_t S, int64_t T,
                       hipStream_t s);
int launch_inc_epoch(int64_t *epoch, hipStream_t s);
int launch_list_order(const Ws &w, const int32_t *J, int64_t nJ, hipStream_t s);
// group: lanes per short column (4, 8, 16 or 32); short_bound / long_bound:
// expected short columns / long pieces of a window (they size the grid; the
// kernels stride over whatever the window holds).
// ev0/ev1 (optional) stamp the Propose dispatch, ev2/ev3 the Update dispatch.
int launch_iteration(const IterArgs &a, int group, int mode, int64_t block, int64_t short_bound,
                     int64_t long_bound, int64_t nblocks_accept, hipStream_t s,
                     hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                     hipEvent_t ev2 = nullptr, hipEvent_t ev3 = nullptr);
// Fused asynchronous Shotgun iteration (accept-all rules): window a.t, plus
// the split columns of window a.t - 1; `flush` applies only the latter
// (a.t = number of windows).
int launch_fused(const IterArgs &a, int group, int64_t short_bound, int64_t long_bound, bool flush,
                 hipStream_t s);
// Power-iteration estimate of the normalised Gram spectral radius; needs the
// column sums of squares in ws.g64 (left there by launch_curvature) and the
// rho arrays of the workspace.  Squared norms land in ws.rho_hist[0..iters).
int launch_rho(const gencd_csc *X, int32_t n_short, int32_t n_lpieces, const Ws &ws, int64_t k_live,
               int iters, hipStream_t s);
// Block Shotgun: preset blocks (base order, block of every column) and the
// per-block power iteration; needs the column sums of squares in ws.g64.
// Squared norms land in ws.bhist[t][b].
int launch_block_setup(const gencd_csc *X, int32_t n_short, int32_t n_lpieces, const Ws &ws,
                       int64_t k_live, uint64_t seed, int iters, hipStream_t s);
// Per-epoch order of Block Shotgun (col_of_pos, windows win_off[0..T]).
int launch_block_order(const Ws &w, int64_t k_live, uint64_t seed, const int64_t *epoch, int64_t T,
                       hipStream_t s);
int launch_check(const gencd_csc *X, const float *y, int loss, double lam, const float *w,
                 int32_t n_short, int32_t n_lpieces, const Ws &ws, bool resync, hipStream_t s);
int launch_renorm(int64_t n, float4 *zs, hipStream_t s);
// Copy caller-held (z_hi, z_lo) and the labels into the packed rows, and back.
int launch_pack_state(int64_t n, const float *z_hi, const float *z_lo, const float *y, float4 *zs,
                      hipStream_t s);
int launch_unpack_state(int64_t n, const float4 *zs, float *z_hi, float *z_lo, hipStream_t s);
int launch_round_f32(const double *src, float *dst, int64_t m, hipStream_t s);

}  // namespace gencd
