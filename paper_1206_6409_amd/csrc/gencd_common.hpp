// Internal declarations shared by the HIP translation units of libgencd.
// Device helpers (losses, the Propose formula, the selection permutation,
// group reductions), the workspace layout and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/gencd.h"

namespace gencd {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64)
constexpr int kWave = 64;
constexpr int kUnroll = 4;   // CSC entries a lane keeps in flight per round

#define GENCD_HIP(call)                                     \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return GENCD_ERR_HIP;             \
  } while (0)

// ---------------------------------------------------------------------------
// Losses of section 1, differentiated in the fitted value t.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float dloss_f32(int loss, float y, float t) {
  if (loss == GENCD_SQUARED) return t - y;
  float m = y * t;  // -y * sigma(-m), evaluated without overflow
  float s;
  if (m >= 0.0f) {
    float e = expf(-m);
    s = e / (1.0f + e);
  } else {
    s = 1.0f / (1.0f + expf(m));
  }
  return -y * s;
}

__device__ __forceinline__ double loss_f64(int loss, double y, double t) {
  if (loss == GENCD_SQUARED) {
    double d = y - t;
    return 0.5 * d * d;
  }
  double m = y * t;
  return (m > 0.0 ? 0.0 : -m) + log1p(exp(-fabs(m)));
}

__device__ __forceinline__ double dloss_f64(int loss, double y, double t) {
  if (loss == GENCD_SQUARED) return t - y;
  double m = y * t;
  double s;
  if (m >= 0.0) {
    double e = exp(-m);
    s = e / (1.0 + e);
  } else {
    s = 1.0 / (1.0 + exp(m));
  }
  return -y * s;
}

// Proposal from the quadratic upper bound (Algorithm 4: Eq. 7 for the step,
// Eq. 9 for the proxy), with the coordinate curvature c = beta ||X_j||^2 / n.
__device__ __forceinline__ void propose_f32(float g, float c, float w, float lam, float &d,
                                            float &phi) {
  if (!(c > 0.0f)) {
    d = 0.0f;
    phi = 0.0f;
    return;
  }
  float a = (g - lam) / c;
  float b = (g + lam) / c;
  float psi = w < a ? a : (w > b ? b : w);
  d = -psi;
  // Eq. 9.  When w and w + d have the same sign, lam (|w + d| - |w|) is
  // +-lam d exactly; factoring it out avoids the cancellation of two FP32
  // magnitudes when |d| << |w| (phi is then tiny and decides the Accept).
  const float wd = w + d;
  if (w > 0.0f && wd >= 0.0f)
    phi = d * (0.5f * c * d + (g + lam));
  else if (w < 0.0f && wd <= 0.0f)
    phi = d * (0.5f * c * d + (g - lam));
  else
    phi = 0.5f * c * d * d + g * d + lam * (fabsf(wd) - fabsf(w));
}

// ---------------------------------------------------------------------------
// Per-epoch selection permutation: 4-round balanced Feistel network on the
// smallest even power of two >= m, cycle-walked into [0, m); the round
// function is the SplitMix64 finaliser.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint64_t splitmix_fin(uint64_t x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBull;
  x ^= x >> 31;
  return x;
}

struct PermKey {
  uint64_t k[4];
  int half;
  uint64_t m;
};

__host__ __device__ inline PermKey make_perm_key(int64_t m, uint64_t seed, int64_t epoch) {
  PermKey pk;
  int bits = 2;
  while ((int64_t(1) << bits) < m) bits += 2;
  pk.half = bits / 2;
  pk.m = uint64_t(m);
  for (int r = 0; r < 4; ++r)
    pk.k[r] = splitmix_fin(seed + 0x9E3779B97F4A7C15ull * uint64_t(epoch * 8 + r + 1));
  return pk;
}

// Key of the preset block partition (b = -1) and of block b's per-epoch
// member order (Block Shotgun).
__host__ __device__ inline uint64_t block_seed(uint64_t seed, int64_t b) {
  return splitmix_fin(seed ^ splitmix_fin(0x626c6f636b73ull + uint64_t(b + 1)));
}

// Preset block b covers the preset positions [block_lo(b), block_lo(b + 1)).
__host__ __device__ inline int64_t block_lo(int64_t b, int64_t k_live, int64_t nb) {
  return b * k_live / nb;
}

__host__ __device__ __forceinline__ uint64_t perm_apply(const PermKey &pk, uint64_t x) {
  const uint64_t mask = pk.half >= 32 ? 0xFFFFFFFFull : ((uint64_t(1) << pk.half) - 1);
  do {
    uint64_t L = x >> pk.half, R = x & mask;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint64_t f = splitmix_fin(R ^ pk.k[r]) & mask;
      uint64_t t = R;
      R = L ^ f;
      L = t;
    }
    x = (L << pk.half) | R;
  } while (x >= pk.m);
  return x;
}

// ---------------------------------------------------------------------------
// Reductions inside an aligned group of G lanes of a wave64.
// ---------------------------------------------------------------------------
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Rounding error of a + b (TwoSum, exact in round-to-nearest).
__device__ __forceinline__ float twosum_err(float a, float b) {
  const float s = a + b;
  const float bp = s - a;
  return (a - (s - bp)) + (b - bp);
}

// Compensated update of a row the caller owns (columns of one colour class
// have disjoint rows): exact product error by FMA, exact sum error by TwoSum.
__device__ __forceinline__ void scatter_plain(float4 *zs, int i, float d, float v) {
  const float p = d * v;
  const float pe = fmaf(d, v, -p);
  float *q = reinterpret_cast<float *>(zs + i);
  const float old = q[0];
  q[0] = old + p;
  q[1] += twosum_err(old, p) + pe;
}

// ---------------------------------------------------------------------------
// Workspace (carved from the caller's buffer).
// ---------------------------------------------------------------------------
struct Ws {
  // problem-static
  float *c;              // [k] curvature bound
  int32_t *live;         // [k] non-empty columns, ascending
  int32_t *all_soff;     // [k+1] short-column index of every column (natural order)
  int32_t *all_loff;     // [k+1] long-piece offsets of every column
  int4 *desc_all_s;      // [k] short-column descriptors, natural order
  int4 *live_rec;        // [k] per live index: the short descriptor, or for a long
                         //     column {first piece, column, pieces, 0}
  int4 *desc_all_l;      // [max_lpieces] long-piece descriptors, natural order
  int32_t *tmp_cnt;      // [k+1] scratch counts
  int32_t *tmp_cnt2;     // [k+1] scratch counts
  int32_t *scan_part;    // [scan partials]
  int32_t *cls_off;      // [k+1] colour class offsets (COLORING)
  int32_t *cls_mem;      // [k] live members by colour, column order inside a class
  int32_t *rad_h, *rad_o;  // [radix_hist_len(k)] digit counts and offsets of a radix sort
  // per-epoch order
  int32_t *col_of_pos;   // [k]
  int32_t *soff;         // [k+1] scratch (live-column scan at set-up)
  int32_t *loff;         // [k+1] long-piece offsets of the positions
  int4 *desc_s;          // [k] descriptor of every position (length 0: long column)
  int4 *desc_l;          // [max_lpieces] long descriptors of the epoch order
  int32_t *win_off;      // [k+1] colour windows (COLORING)
  int32_t *wbl;          // [k+2] first long piece of every window
  // per-window
  float *delta;          // [k]
  float *phi;            // [k]
  float *gacc;           // [max_lpieces] partial sums of split columns
  float *wsnap;          // [k] w of split columns at Propose time
  int32_t *acc;          // [k]
  // state
  float4 *zs;            // [n] {z_hi, z_lo, y, 0}: compensated fitted value and label
                         // of a row in one 16-byte record (one gather per entry)
  float *w_ckpt;         // [k]
  float *rs;             // [n] residual l'(y, z) of every row, refreshed before a
                         // Propose that reads it (large windows)
  // FP64 check
  double *z64, *r64;     // [n]
  double *g64;           // [k]
  double *red;           // [16] reductions, counters, flags; [12] epoch counter
  double *rrep;          // [kChkRep * 16] replicas of the check's reductions, one line each
  unsigned long long *scat;  // [kChkRep * 16] nonzeros scattered by Update (GENCD_PROFILE)
  // spectral-radius estimate (only when |J| is chosen from it, or blocks)
  double *rho_dinv;      // [k] 1/||X_j|| (0 for empty columns)
  double *rho_x;         // [k] D^{-1/2} v, the scaled iterate
  double *rho_hist;      // [kRhoMaxIters] ||G v||^2 per iteration
  // Block Shotgun (only with preset blocks)
  int64_t nblocks;
  int32_t *bbase;        // [k] preset order of the live columns
  int32_t *bcol;         // [k] block of every column (-1: empty)
  int32_t *bp;           // [nblocks] P_b* of every block
  int32_t *bstart;       // [nblocks+1] per-epoch position offsets of the blocks
  int32_t *bwin;         // [nblocks+1] per-epoch window offsets of the blocks
  double *bs;            // [n][nblocks] per-block products X x in the power iteration
  double *bhist;         // [kBlockRhoMaxIters][nblocks] ||G_b v_b||^2
  size_t scan_part_len;
  int64_t max_lpieces;
};

int64_t max_lpieces_for(int64_t k, int64_t nnz, int piece, int short_max);
// Default schedule: lanes per short column and nonzeros per long piece.
constexpr int kDefaultGroup = 8;
constexpr int kDefaultPiece = 256;
constexpr int kRhoIters = 20;       // power iterations behind an automatic |J|
constexpr int kRhoMaxIters = 1024;  // cap for the standalone estimate
constexpr int kBlockRhoMaxIters = 64;    // power iterations of the per-block estimate
constexpr int64_t kMaxBlocks = 4096;     // preset blocks of Block Shotgun
// The check's block results go to kChkRep replicas (workgroup b to replica
// b mod kChkRep), each on its own 128-byte line: atomics on one address
// serialise, so a single accumulator would cost one atomic per workgroup in
// sequence.  The host folds the replicas when it reads the check.
constexpr int kChkRep = 64;
size_t workspace_layout(int64_t n, int64_t k, int64_t nnz, int piece, int short_max, bool rho,
                        int64_t nblocks, void *base, Ws *ws);
size_t scan_partials_for(int64_t len);

// Exclusive scan of int32 counts: out[0..len] (out[len] = total).
int scan_exclusive(const int32_t *in, int32_t *out, int64_t len, int32_t *partials,
                   hipStream_t s);

// Stable LSD radix sort of m (uint32 key, int32 value) pairs on the low
// `bits` key bits (8 per pass).  (k0, v0) hold the input and (k1, v1) are
// scratch of length m; the sorted pairs end in buffer *out_buf (0: k0/v0,
// 1: k1/v1).  hist and offs hold radix_hist_len(m) int32 each, part
// scan_partials_for(radix_hist_len(m)).
int64_t radix_hist_len(int64_t m);
int radix_sort_pairs(uint32_t *k0, int32_t *v0, uint32_t *k1, int32_t *v1, int64_t m, int bits,
                     int32_t *hist, int32_t *offs, int32_t *part, hipStream_t s, int *out_buf);

// Epochs from a check to the next, `done` epochs after the start of the
// solve: check_every > 0 fixes it; check_every = 0 adapts it to a tenth of
// the epochs run so far (1 for the first twenty, at most 64), so a solve
// that first meets its tolerance at epoch N is checked by about 1.1 N;
// check_every = -m adapts it to an m-th (checked by about (1 + 1/m) N).
inline int64_t check_interval(int64_t check_every, int64_t done) {
  if (check_every > 0) return check_every;
  const int64_t m = check_every < 0 ? -check_every : 10;
  const int64_t c = done / m;
  return c < 1 ? 1 : (c > 64 ? 64 : c);
}

// Number of bits needed for values up to v (0 for v = 0).
inline int bits_for(uint64_t v) {
  int b = 0;
  while (b < 64 && (v >> b) != 0) ++b;
  return b;
}

}  // namespace gencd
