// HIP kernels of the GenCD hot path for gfx950 (wave64, 256-thread groups).
//
// Work decomposition.  Column nonzero counts are heavy-tailed (most columns
// hold a handful of nonzeros, a few hold nearly n), so columns come in two
// classes, each with its own list of 16-byte piece descriptors:
//   * short columns (at most GS * kUnroll nonzeros) are one piece each and a
//     group of GS lanes (GS in {4, 8, 16, 32}) proposes / updates a column, so
//     one wave serves 64 / GS columns at once;
//   * long columns are cut into pieces of at most `piece` nonzeros, one
//     wave64 per piece; the partial sums of a split column are published and
//     combined, in piece order, by the next launch.
// Inside a group the lanes read consecutive CSC entries (coalesced row_idx /
// val loads), keep kUnroll of them in flight, gather the state and reduce.
//
// Selection (section 2.1) is precomputed per epoch: position p of the epoch
// order holds column col_of_pos[p] and the descriptor desc_s[p] (length 0
// when the column is long), so a short group goes from its position straight
// to its column.  loff is the exclusive scan of long pieces over positions;
// an iteration's selected set J (a position range) maps to one long-piece
// range whose bounds sit in device memory (a captured epoch replays without
// host involvement).
#include <hip/hip_ext.h>

#include "gencd_common.hpp"
#include "gencd_kernels.hpp"

namespace gencd {

// ---------------------------------------------------------------------------
// Exclusive scan of int32 (three passes: tile sums, scan of tile sums, apply)
// ---------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

size_t scan_partials_for(int64_t len) { return size_t((len + kScanTile - 1) / kScanTile) + 2; }

__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t &total) {
  __shared__ int32_t wsum[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    int32_t y = __shfl_up(x, off, kWave);
    if (lane >= off) x += y;
  }
  if (lane == kWave - 1) wsum[wid] = x;
  __syncthreads();
  int32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    if (w < wid) pre += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(const int32_t *in, int64_t len,
                                                        int32_t *part) {
  int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  int32_t s = 0;
#pragma unroll
  for (int u = 0; u < kScanItems; ++u)
    if (base + u < len) s += in[base + u];
  int32_t tot;
  block_excl_scan(s, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_part(int32_t *part, int64_t nparts) {
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < nparts; b0 += kBlock) {
    int64_t i = b0 + threadIdx.x;
    int32_t v = i < nparts ? part[i] : 0;
    int32_t tot;
    int32_t ex = block_excl_scan(v, tot);
    if (i < nparts) part[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[nparts] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const int32_t *in, int64_t len,
                                                        const int32_t *part, int64_t nparts,
                                                        int32_t *out) {
  int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  int32_t v[kScanItems];
  int32_t s = 0;
#pragma unroll
  for (int u = 0; u < kScanItems; ++u) {
    v[u] = (base + u < len) ? in[base + u] : 0;
    s += v[u];
  }
  int32_t tot;
  int32_t ex = block_excl_scan(s, tot) + part[blockIdx.x];
#pragma unroll
  for (int u = 0; u < kScanItems; ++u) {
    if (base + u < len) out[base + u] = ex;
    ex += v[u];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[len] = part[nparts];
}

int scan_exclusive(const int32_t *in, int32_t *out, int64_t len, int32_t *part, hipStream_t s) {
  if (len <= 0) {
    hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(kBlock), 0, s, part, int64_t(0));
    // out[0] = 0
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kBlock), 0, s, in, int64_t(0), part,
                       int64_t(0), out);
    return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
  }
  int64_t nparts = (len + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3(unsigned(nparts)), dim3(kBlock), 0, s, in, len, part);
  hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(kBlock), 0, s, part, nparts);
  hipLaunchKernelGGL(k_scan_apply, dim3(unsigned(nparts)), dim3(kBlock), 0, s, in, len, part,
                     nparts, out);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (uint32 key, int32 value) pairs, 8 key bits per
// pass.  A pass has three steps: every tile of kRadixTile items counts its
// digits (k_radix_hist, digit-major so that one exclusive scan turns the
// counts into output offsets), the scan, and a stable scatter
// (k_radix_scatter).  The scatter walks its tile in input order, kBlock
// items per round; inside a round each wave finds the lanes holding the
// same digit from eight ballots (one per digit bit), so an item's rank is
// the digit's count from earlier rounds and earlier waves plus its peers in
// lower lanes.
// ---------------------------------------------------------------------------
constexpr int kRadixBins = 256;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kBlock * kRadixItems;
static_assert(kRadixBins == kBlock, "one digit counter per thread");

int64_t radix_hist_len(int64_t m) {
  const int64_t tiles = (m + kRadixTile - 1) / kRadixTile;
  return int64_t(kRadixBins) * (tiles > 0 ? tiles : 1) + 1;
}

// Lanes of the wave whose 9-bit digit equals this lane's (bit 8 marks an
// item past the end).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 9; ++b) {
    const uint64_t bal = __ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? bal : ~bal;
  }
  return m;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t *keys, int64_t m, int shift,
                                                        int64_t ntiles, int32_t *hist) {
  __shared__ int32_t h[kRadixBins];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int lane = int(threadIdx.x) & (kWave - 1);
  const int64_t t0 = int64_t(blockIdx.x) * kRadixTile;
  for (int i = 0; i < kRadixItems; ++i) {
    const int64_t q = t0 + int64_t(i) * kBlock + threadIdx.x;
    const uint32_t d = q < m ? (keys[q] >> shift) & 0xFFu : 0x100u;
    const uint64_t peers = digit_peers(d);  // one LDS atomic per distinct digit of a wave
    if (d < 0x100u && __popcll(peers & ((1ull << lane) - 1)) == 0)
      atomicAdd(&h[d], int32_t(__popcll(peers)));
  }
  __syncthreads();
  hist[int64_t(threadIdx.x) * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t *kin, const int32_t *vin,
                                                           int64_t m, int shift, int64_t ntiles,
                                                           const int32_t *offs, uint32_t *kout,
                                                           int32_t *vout) {
  constexpr int NW = kBlock / kWave;
  __shared__ int32_t base[kRadixBins];
  __shared__ int32_t goff[kRadixBins];
  __shared__ int32_t wcnt[NW][kRadixBins];
  const int t = int(threadIdx.x), lane = t & (kWave - 1), wv = t / kWave;
  base[t] = 0;
  goff[t] = offs[int64_t(t) * ntiles + blockIdx.x];
  const int64_t t0 = int64_t(blockIdx.x) * kRadixTile;
  for (int i = 0; i < kRadixItems; ++i) {
    const int64_t q = t0 + int64_t(i) * kBlock + t;
    const bool ok = q < m;
    const uint32_t key = ok ? kin[q] : 0u;
    const int32_t val = ok ? vin[q] : 0;
    const uint32_t d = ok ? (key >> shift) & 0xFFu : 0x100u;
#pragma unroll
    for (int w = 0; w < NW; ++w) wcnt[w][t] = 0;  // column t: only this thread touches it here
    __syncthreads();
    const uint64_t peers = digit_peers(d);
    const int below = __popcll(peers & ((1ull << lane) - 1));
    if (ok && below == 0) wcnt[wv][d] = __popcll(peers);
    __syncthreads();
    if (ok) {
      int32_t r = base[d] + below;
      for (int w = 0; w < wv; ++w) r += wcnt[w][d];
      const int64_t dst = int64_t(goff[d]) + r;
      kout[dst] = key;
      vout[dst] = val;
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) add += wcnt[w][t];
    base[t] += add;  // read after the next round's first barrier
  }
}

int radix_sort_pairs(uint32_t *k0, int32_t *v0, uint32_t *k1, int32_t *v1, int64_t m, int bits,
                     int32_t *hist, int32_t *offs, int32_t *part, hipStream_t s, int *out_buf) {
  *out_buf = 0;
  if (m <= 0 || bits <= 0) return GENCD_OK;
  const int64_t ntiles = (m + kRadixTile - 1) / kRadixTile;
  uint32_t *kb[2] = {k0, k1};
  int32_t *vb[2] = {v0, v1};
  int cur = 0;
  for (int shift = 0; shift < bits && shift < 32; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(unsigned(ntiles)), dim3(kBlock), 0, s, kb[cur], m, shift,
                       ntiles, hist);
    const int st = scan_exclusive(hist, offs, int64_t(kRadixBins) * ntiles, part, s);
    if (st) return st;
    hipLaunchKernelGGL(k_radix_scatter, dim3(unsigned(ntiles)), dim3(kBlock), 0, s, kb[cur],
                       vb[cur], m, shift, ntiles, offs, kb[cur ^ 1], vb[cur ^ 1]);
    cur ^= 1;
  }
  *out_buf = cur;
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *p, int64_t m, T v) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < m;
       i += int64_t(gridDim.x) * kBlock)
    p[i] = v;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(T *dst, const T *src, int64_t m) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < m;
       i += int64_t(gridDim.x) * kBlock)
    dst[i] = src[i];
}

static unsigned grid_for(int64_t m, unsigned cap = 4096) {
  int64_t b = (m + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return unsigned(b);
}

int fill_f32(float *p, int64_t m, float v, hipStream_t s) {
  if (m <= 0) return GENCD_OK;
  hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(m)), dim3(kBlock), 0, s, p, m, v);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}
int fill_i32(int32_t *p, int64_t m, int32_t v, hipStream_t s) {
  if (m <= 0) return GENCD_OK;
  hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(m)), dim3(kBlock), 0, s, p, m, v);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}
int fill_f64(double *p, int64_t m, double v, hipStream_t s) {
  if (m <= 0) return GENCD_OK;
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(m)), dim3(kBlock), 0, s, p, m, v);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}
int copy_f32(float *d, const float *src, int64_t m, hipStream_t s) {
  if (m <= 0) return GENCD_OK;
  hipLaunchKernelGGL(k_copy<float>, dim3(grid_for(m)), dim3(kBlock), 0, s, d, src, m);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}
int copy_i32(int32_t *d, const int32_t *src, int64_t m, hipStream_t s) {
  if (m <= 0) return GENCD_OK;
  hipLaunchKernelGGL(k_copy<int32_t>, dim3(grid_for(m)), dim3(kBlock), 0, s, d, src, m);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Validation (structure of the CSC matrix, logistic labels)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_validate_matrix(const int64_t *col_ptr,
                                                             const int32_t *row_idx, int64_t n,
                                                             int64_t k, int64_t nnz,
                                                             unsigned long long *bad) {
  for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < k;
       j += int64_t(gridDim.x) * kBlock) {
    int64_t a = col_ptr[j], b = col_ptr[j + 1];
    bool ok = a >= 0 && b >= a && b <= nnz && (j > 0 || a == 0) && (j + 1 < k || b == nnz);
    if (ok) {
      int32_t prev = -1;
      for (int64_t e = a; e < b; ++e) {
        int32_t r = row_idx[e];
        if (r <= prev || r >= n) {
          ok = false;
          break;
        }
        prev = r;
      }
    }
    if (!ok) atomicOr(bad, 1ull);
  }
}

__global__ __launch_bounds__(kBlock) void k_validate_labels(const float *y, int64_t n,
                                                             unsigned long long *bad) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    float v = y[i];
    if (!(v == 1.0f || v == -1.0f)) atomicOr(bad, 2ull);
  }
}

int launch_validate(const gencd_csc *X, const float *y, int loss, bool matrix,
                    unsigned long long *bad, hipStream_t s) {
  if (matrix)
    hipLaunchKernelGGL(k_validate_matrix, dim3(grid_for(X->k)), dim3(kBlock), 0, s, X->col_ptr,
                       X->row_idx, X->n, X->k, X->nnz, bad);
  if (loss == GENCD_LOGISTIC)
    hipLaunchKernelGGL(k_validate_labels, dim3(grid_for(X->n)), dim3(kBlock), 0, s, y, X->n, bad);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Piece descriptors.  A descriptor is one 16-byte load:
//   x = first CSC entry of the piece, y = column, z = position in the order
//   (-1 for the static natural-order lists), w = length | single<<31
// where `single` marks a column that fits in one piece.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int4 make_desc(int64_t beg, int32_t j, int32_t p, int32_t len,
                                          bool single) {
  return make_int4(int32_t(uint32_t(beg)), j, p, int32_t(uint32_t(len) | (single ? 0x80000000u : 0u)));
}
__device__ __forceinline__ int64_t desc_beg(const int4 &d) { return int64_t(uint32_t(d.x)); }
__device__ __forceinline__ int32_t desc_len(const int4 &d) { return int32_t(uint32_t(d.w) & 0x7FFFFFFFu); }
__device__ __forceinline__ bool desc_single(const int4 &d) { return (uint32_t(d.w) >> 31) != 0; }

// Role of a wave in a two-class launch: the first `nl` waves walk the long
// pieces (one piece per wave), the others walk the short columns (64/GS per
// wave).  At least one wave is kept for each role.  Waves are numbered
// slot-major (wave slot in the workgroup, then workgroup), so the long waves
// take the first wave of every workgroup before any workgroup gets a second
// one: their scattered gathers spread over all compute units instead of
// queueing on the address units of a few.  No kernel using roles shares LDS
// or barriers between waves.
struct Roles {
  int64_t wave, nwaves, nl;
  int wl;
};
__device__ __forceinline__ Roles roles(int32_t nl_req) {
  Roles r;
  r.wave = int64_t(threadIdx.x / kWave) * gridDim.x + blockIdx.x;
  r.nwaves = int64_t(gridDim.x) * (kBlock / kWave);
  int64_t nl = nl_req < 1 ? 1 : nl_req;
  if (nl > r.nwaves - 1) nl = r.nwaves - 1;
  r.nl = nl;
  r.wl = threadIdx.x & (kWave - 1);
  return r;
}

// ---------------------------------------------------------------------------
// Preprocessing: piece decomposition, live columns, curvature (row a1)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_col_counts(const int64_t *col_ptr, int64_t k,
                                                        int piece, int short_max,
                                                        int32_t *scnt, int32_t *lcnt,
                                                        int32_t *live_flag) {
  for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < k;
       j += int64_t(gridDim.x) * kBlock) {
    const int64_t m = col_ptr[j + 1] - col_ptr[j];
    scnt[j] = (m > 0 && m <= short_max) ? 1 : 0;
    lcnt[j] = m > short_max ? int32_t((m + piece - 1) / piece) : 0;
    live_flag[j] = m > 0 ? 1 : 0;
  }
}

__global__ __launch_bounds__(kBlock) void k_col_scatter(const int64_t *col_ptr, int64_t k,
                                                         int piece, const int32_t *all_soff,
                                                         const int32_t *all_loff,
                                                         const int32_t *live_pos,
                                                         int4 *desc_all_s, int4 *desc_all_l,
                                                         int32_t *live, int4 *live_rec) {
  for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < k;
       j += int64_t(gridDim.x) * kBlock) {
    const int64_t cb = col_ptr[j], ce = col_ptr[j + 1];
    if (all_soff[j + 1] > all_soff[j])
      desc_all_s[all_soff[j]] = make_desc(cb, int32_t(j), -1, int32_t(ce - cb), true);
    const int32_t a = all_loff[j], b = all_loff[j + 1];
    for (int32_t q = a; q < b; ++q) {
      const int64_t beg = cb + int64_t(q - a) * piece;
      const int64_t len = (ce - beg) < piece ? (ce - beg) : piece;
      desc_all_l[q] = make_desc(beg, int32_t(j), -1, int32_t(len), b - a == 1);
    }
    if (ce > cb) {
      live[live_pos[j]] = int32_t(j);
      live_rec[live_pos[j]] = all_soff[j + 1] > all_soff[j]
                                  ? make_desc(cb, int32_t(j), -1, int32_t(ce - cb), true)
                                  : make_int4(a, int32_t(j), b - a, 0);
    }
  }
}

// Sum of squares per column in FP64 (both piece classes).
template <int GS>
__global__ __launch_bounds__(kBlock) void k_colsq(const float *val, const int4 *ds, int32_t ns,
                                                   const int4 *dl, int32_t nlp, int32_t nl_req,
                                                   double *acc) {
  const Roles r = roles(nl_req);
  const bool lng = r.wave < r.nl;
  const int G = lng ? kWave : GS;
  const int lane = lng ? r.wl : (r.wl & (GS - 1));
  const int64_t first = lng ? r.wave : (r.wave - r.nl) * (kWave / GS) + r.wl / GS;
  const int64_t step = lng ? r.nl : (r.nwaves - r.nl) * (kWave / GS);
  const int64_t cnt = lng ? nlp : ns;
  const int4 *dd = lng ? dl : ds;
  for (int64_t q = first; q < cnt; q += step) {
    const int4 d = dd[q];
    const int64_t beg = desc_beg(d);
    const int32_t len = desc_len(d);
    double s = 0.0;
    for (int32_t base = 0; base < len; base += G * kUnroll) {
      float v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int32_t e = base + u * G + lane;
        v[u] = e < len ? val[beg + e] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) s += double(v[u]) * double(v[u]);
    }
    s = lng ? group_sum<kWave>(s) : group_sum<GS>(s);
    if (lane == 0) {
      if (desc_single(d))
        acc[d.y] = s;
      else
        atomicAdd(&acc[d.y], s);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_curvature(int64_t k, const double *ss, double beta,
                                                       double inv_n, float *c) {
  for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < k;
       j += int64_t(gridDim.x) * kBlock)
    c[j] = float(beta * ss[j] * inv_n);
}

static unsigned waves_grid(int64_t waves, unsigned cap = 8192) {
  int64_t b = (waves + (kBlock / kWave) - 1) / (kBlock / kWave);
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return unsigned(b);
}

int launch_preprocess(const gencd_csc *X, int loss, int piece, int short_max, const Ws &w,
                      hipStream_t s) {
  (void)loss;
  const int64_t k = X->k;
  // counts: short -> tmp_cnt, long pieces -> tmp_cnt2, live flags -> col_of_pos (scratch)
  hipLaunchKernelGGL(k_col_counts, dim3(grid_for(k)), dim3(kBlock), 0, s, X->col_ptr, k, piece,
                     short_max, w.tmp_cnt, w.tmp_cnt2, w.col_of_pos);
  int st = scan_exclusive(w.tmp_cnt, w.all_soff, k, w.scan_part, s);
  if (st) return st;
  st = scan_exclusive(w.tmp_cnt2, w.all_loff, k, w.scan_part, s);
  if (st) return st;
  st = scan_exclusive(w.col_of_pos, w.soff, k, w.scan_part, s);  // live positions
  if (st) return st;
  hipLaunchKernelGGL(k_col_scatter, dim3(grid_for(k)), dim3(kBlock), 0, s, X->col_ptr, k, piece,
                     w.all_soff, w.all_loff, w.soff, w.desc_all_s, w.desc_all_l, w.live,
                     w.live_rec);
  return fill_f64(w.g64, k, 0.0, s);
}

// grid for a two-class pass over ns short columns and nlp long pieces
// Waves of a two-role launch: one per long piece up to kMaxLongWaves (whole-
// matrix passes such as the FP64 check walk many pieces per wave beyond
// that, each a dependent descriptor -> weight -> entries chain, so more waves
// keep more chains in flight), and one per 64 / gs short columns up to 28672.
constexpr int64_t kMaxLongWaves = 16384;
static void two_class_grid(int64_t ns, int64_t nlp, int gs, unsigned *blocks, int32_t *nl) {
  int64_t lw = nlp < kMaxLongWaves ? nlp : kMaxLongWaves;
  int64_t sw = (ns + (kWave / gs) - 1) / (kWave / gs);
  if (sw > 28672) sw = 28672;
  if (lw < 1) lw = 1;
  if (sw < 1) sw = 1;
  *nl = int32_t(lw);
  *blocks = waves_grid(lw + sw, 12288);
}

int launch_curvature(const gencd_csc *X, int loss, int32_t n_short, int32_t n_lpieces,
                     const Ws &w, hipStream_t s) {
  unsigned blocks;
  int32_t nl;
  two_class_grid(n_short, n_lpieces, 8, &blocks, &nl);
  if (n_short + n_lpieces > 0)
    hipLaunchKernelGGL(k_colsq<8>, dim3(blocks), dim3(kBlock), 0, s, X->val, w.desc_all_s,
                       n_short, w.desc_all_l, n_lpieces, nl, w.g64);
  double beta = loss == GENCD_SQUARED ? 1.0 : 0.25;
  hipLaunchKernelGGL(k_curvature, dim3(grid_for(X->k)), dim3(kBlock), 0, s, X->k, w.g64, beta,
                     1.0 / double(X->n), w.c);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Per-epoch selection order
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_select_perm(int64_t m, PermKey pk, int32_t *out) {
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < m;
       p += int64_t(gridDim.x) * kBlock)
    out[p] = int32_t(perm_apply(pk, uint64_t(p)));
}

int launch_select_perm(int64_t m, uint64_t seed, int64_t epoch, int32_t *out, hipStream_t s) {
  if (m <= 0) return GENCD_OK;
  PermKey pk = make_perm_key(m, seed, epoch);
  hipLaunchKernelGGL(k_select_perm, dim3(grid_for(m)), dim3(kBlock), 0, s, m, pk, out);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// Class counts of the columns at the positions of an order.
__device__ __forceinline__ void pos_counts(int32_t j, const int32_t *all_soff,
                                           const int32_t *all_loff, int32_t &sc, int32_t &lc) {
  sc = all_soff[j + 1] - all_soff[j];
  lc = all_loff[j + 1] - all_loff[j];
}

// natural != 0: live columns in index order (cyclic rule).  The epoch
// number is read from device memory so that a captured epoch replays.
// One 16-byte gather per position (the live column's record) gives the
// column, its class counts and, for a short column, its descriptor, which
// is written here; k_order_desc then only lays out the long pieces.
__global__ __launch_bounds__(kBlock) void k_epoch_order(const int4 *live_rec, int64_t k_live,
                                                         uint64_t seed, const int64_t *epoch,
                                                         int natural, int32_t *col_of_pos,
                                                         int32_t *sc, int32_t *lc,
                                                         int4 *desc_s) {
  const PermKey pk = make_perm_key(k_live, seed, *epoch);
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < k_live;
       p += int64_t(gridDim.x) * kBlock) {
    int64_t src = natural ? p : int64_t(perm_apply(pk, uint64_t(p)));
    int4 r = live_rec[src];
    col_of_pos[p] = r.y;
    if (desc_len(r) > 0) {  // short column
      sc[p] = 1;
      lc[p] = 0;
      r.z = int32_t(p);
      desc_s[p] = r;
    } else {
      sc[p] = 0;
      lc[p] = r.z;
      desc_s[p] = make_int4(0, r.y, int32_t(p), 0);  // long: length 0
    }
  }
}

__global__ void k_inc_epoch(int64_t *epoch) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *epoch += 1;
}

// class counts for an explicit column list (step API and colour windows)
__global__ __launch_bounds__(kBlock) void k_list_counts(const int32_t *cols, int64_t m,
                                                         const int32_t *all_soff,
                                                         const int32_t *all_loff, int32_t *sc,
                                                         int32_t *lc) {
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < m;
       p += int64_t(gridDim.x) * kBlock)
    pos_counts(cols[p], all_soff, all_loff, sc[p], lc[p]);
}

// Descriptors of the order: each position's static descriptor, re-tagged
// with the position.  A thread takes a position; then the whole wave copies
// the pieces of its long columns, one column at a time, so that a heavy
// column's hundreds of pieces take a round or two of 64 x kUnroll loads
// instead of a long serial loop on a few lanes.  The loop is uniform over
// the wave (every lane runs the same bases).
__global__ __launch_bounds__(kBlock) void k_order_desc(const int32_t *col_of_pos, int64_t m,
                                                        const int32_t *loff,
                                                        const int32_t *all_soff,
                                                        const int32_t *all_loff,
                                                        const int4 *desc_all_s,
                                                        const int4 *desc_all_l, int4 *desc_s,
                                                        int4 *desc_l, int32_t shorts_done) {
  const int lane = int(threadIdx.x) & (kWave - 1);
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t base = int64_t(blockIdx.x) * kBlock + threadIdx.x - lane; base < m;
       base += stride) {
    const int64_t p = base + lane;
    int32_t j = 0;
    bool lng = false;
    if (p < m && shorts_done) {  // every desc_s written: find the long positions
      lng = loff[p + 1] > loff[p];
      if (lng) j = col_of_pos[p];
    } else if (p < m) {
      j = col_of_pos[p];
      const int32_t sj = all_soff[j];
      if (all_soff[j + 1] > sj) {  // short column
        int4 d = desc_all_s[sj];
        d.z = int32_t(p);
        desc_s[p] = d;
      } else {
        desc_s[p] = make_int4(0, j, int32_t(p), 0);  // long: length 0
        lng = true;
      }
    }
    unsigned long long left = __ballot(lng);
    while (left) {
      const int g = __builtin_ctzll(left);  // a lane whose position is long
      left &= left - 1;
      const int64_t pg = base + g;
      const int32_t jg = __shfl(j, g);
      const int32_t a = loff[pg], b = loff[pg + 1], src = all_loff[jg];
      for (int32_t q0 = a; q0 < b; q0 += kWave * kUnroll) {
        int4 d[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int32_t q = q0 + u * kWave + lane;
          if (q < b) d[u] = desc_all_l[src + (q - a)];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int32_t q = q0 + u * kWave + lane;
          if (q < b) {
            d[u].z = int32_t(pg);
            desc_l[q] = d[u];
          }
        }
      }
    }
  }
}

// Colour windows: size of the class visited at step t of the epoch.
__global__ __launch_bounds__(kBlock) void k_color_win_sizes(const int32_t *cls_off, int64_t C,
                                                             uint64_t seed, const int64_t *epoch,
                                                             int32_t *sz) {
  const PermKey pk = make_perm_key(C, seed, *epoch);
  for (int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x; t < C;
       t += int64_t(gridDim.x) * kBlock) {
    int64_t c = int64_t(perm_apply(pk, uint64_t(t)));
    sz[t] = cls_off[c + 1] - cls_off[c];
  }
}

__global__ __launch_bounds__(kBlock) void k_color_fill(const int32_t *cls_off,
                                                        const int32_t *cls_mem, int64_t C,
                                                        uint64_t seed, const int64_t *epoch,
                                                        const int32_t *win_off,
                                                        int32_t *col_of_pos) {
  const PermKey pk = make_perm_key(C, seed, *epoch);
  for (int64_t t = blockIdx.x; t < C; t += gridDim.x) {
    int64_t c = int64_t(perm_apply(pk, uint64_t(t)));
    int32_t a = cls_off[c], b = cls_off[c + 1];
    int32_t o = win_off[t];
    for (int32_t u = a + threadIdx.x; u < b; u += kBlock) col_of_pos[o + (u - a)] = cls_mem[u];
  }
}

// Long-piece ranges of every window: wbl[t] = first long piece of window t.
__global__ __launch_bounds__(kBlock) void k_window_bounds(const int32_t *loff,
                                                           const int32_t *win_off, int64_t S,
                                                           int64_t m, int64_t T, int32_t *wbl) {
  for (int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x; t <= T;
       t += int64_t(gridDim.x) * kBlock) {
    int64_t pos = win_off ? int64_t(win_off[t]) : (t * S < m ? t * S : m);
    wbl[t] = loff[pos];
  }
}

static int order_tail(const Ws &w, int64_t m, const int32_t *win_off, int64_t S, int64_t T,
                      hipStream_t s, bool shorts_done = false) {
  int st = scan_exclusive(w.tmp_cnt2, w.loff, m, w.scan_part, s);
  if (st) return st;
  if (m > 0)
    hipLaunchKernelGGL(k_order_desc, dim3(grid_for(m)), dim3(kBlock), 0, s, w.col_of_pos, m,
                       w.loff, w.all_soff, w.all_loff, w.desc_all_s, w.desc_all_l, w.desc_s,
                       w.desc_l, int32_t(shorts_done ? 1 : 0));
  hipLaunchKernelGGL(k_window_bounds, dim3(grid_for(T + 1)), dim3(kBlock), 0, s, w.loff, win_off,
                     S, m, T, w.wbl);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

int launch_epoch_order(const Ws &w, int64_t k_live, int rule, uint64_t seed,
                       const int64_t *epoch, int64_t num_colors, int64_t S, int64_t T,
                       hipStream_t s) {
  if (rule == GENCD_COLORING) {
    hipLaunchKernelGGL(k_color_win_sizes, dim3(grid_for(num_colors)), dim3(kBlock), 0, s,
                       w.cls_off, num_colors, seed, epoch, w.tmp_cnt);
    int st = scan_exclusive(w.tmp_cnt, w.win_off, num_colors, w.scan_part, s);
    if (st) return st;
    hipLaunchKernelGGL(k_color_fill, dim3(unsigned(num_colors < 8192 ? num_colors : 8192)),
                       dim3(kBlock), 0, s, w.cls_off, w.cls_mem, num_colors, seed, epoch,
                       w.win_off, w.col_of_pos);
    hipLaunchKernelGGL(k_list_counts, dim3(grid_for(k_live)), dim3(kBlock), 0, s, w.col_of_pos,
                       k_live, w.all_soff, w.all_loff, w.tmp_cnt, w.tmp_cnt2);
    return order_tail(w, k_live, w.win_off, 0, num_colors, s);
  }
  hipLaunchKernelGGL(k_epoch_order, dim3(grid_for(k_live)), dim3(kBlock), 0, s, w.live_rec,
                     k_live, seed, epoch, rule == GENCD_CYCLIC ? 1 : 0, w.col_of_pos, w.tmp_cnt,
                     w.tmp_cnt2, w.desc_s);
  return order_tail(w, k_live, nullptr, S, T, s, true);
}

int launch_inc_epoch(int64_t *epoch, hipStream_t s) {
  hipLaunchKernelGGL(k_inc_epoch, dim3(1), dim3(64), 0, s, epoch);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

int launch_list_order(const Ws &w, const int32_t *J, int64_t nJ, hipStream_t s) {
  int st = copy_i32(w.col_of_pos, J, nJ, s);
  if (st) return st;
  hipLaunchKernelGGL(k_list_counts, dim3(grid_for(nJ)), dim3(kBlock), 0, s, w.col_of_pos, nJ,
                     w.all_soff, w.all_loff, w.tmp_cnt, w.tmp_cnt2);
  return order_tail(w, nJ, nullptr, nJ, 1, s);
}

// ---------------------------------------------------------------------------
// One iteration: Propose (Algorithm 2 / 4), Accept (section 2.3), Update
// (Algorithm 3).  The residual l'(y, z) is evaluated on the fly from
// z = z_hi + z_lo, which Propose only reads; Update writes z in the next
// launch, so every proposal of an iteration sees the state at its start.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void window_of(const IterArgs &a, int32_t &P0, int32_t &P1) {
  if (a.win_off) {
    P0 = a.win_off[a.t];
    P1 = a.win_off[a.t + 1];
  } else {
    P0 = a.win_lo;
    P1 = a.win_hi;
  }
}

// Sum of the partial gradients of a split column, in piece order (the same
// order, hence the same float result, in every wave that computes it).
__device__ __forceinline__ float split_sum(const float *part, int32_t pf, int32_t np, int lane) {
  float t = 0.0f;
  for (int32_t u0 = 0; u0 < np; u0 += kWave * kUnroll) {
    float v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int32_t idx = u0 + u * kWave + lane;
      v[u] = idx < np ? part[pf + idx] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) t += v[u];
  }
  return group_sum<kWave>(t);
}

// Propose of one piece by a group of G lanes.
// U entries per lane per batch: long pieces (G = 64) take 8 so that a
// 512-entry piece is one round of dependent loads; short groups take 4.
// RS: l'(y, z) comes from the refreshed residual vector (a 4-byte gather
// from an array a quarter of the packed rows' size); otherwise it is formed
// per entry from the row's packed {z_hi, z_lo, y}.  Both evaluate the same
// FP32 expression.
template <int G, int MODE, int U = kUnroll, bool RS = false>
__device__ __forceinline__ void propose_piece(const IterArgs &a, const int4 dsc, int64_t q,
                                              int lane, int32_t P0) {
  const int64_t beg = desc_beg(dsc);
  const int32_t len = desc_len(dsc);
  const int32_t j = dsc.y, p = dsc.z;
  const bool single = desc_single(dsc);
  float wj = 0.0f, cj = 0.0f;
  if (lane == 0) {  // issued early, consumed after the reduction
    wj = a.w[j];
    if (single) cj = a.c[j];
  }
  float s = 0.0f;
  for (int32_t base = 0; base < len; base += G * U) {
    int32_t ri[U];
    float vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t e = base + u * G + lane;
      ri[u] = e < len ? a.row_idx[beg + e] : -1;
      vv[u] = e < len ? a.val[beg + e] : 0.0f;
    }
    if constexpr (RS) {
      float rr[U];
#pragma unroll
      for (int u = 0; u < U; ++u) rr[u] = a.rs[ri[u] >= 0 ? ri[u] : 0];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ri[u] >= 0) s += vv[u] * rr[u];
    } else {
      float zh[U], zl[U], yy[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t i = ri[u] >= 0 ? ri[u] : 0;
        const float4 zr = a.zs[i];  // one 16-byte gather: z_hi, z_lo, y
        zh[u] = zr.x;
        zl[u] = zr.y;
        yy[u] = zr.z;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ri[u] >= 0) s += vv[u] * dloss_f32(a.loss, yy[u], zh[u] + zl[u]);
    }
  }
  s = group_sum<G>(s);
  if (lane != 0) return;
  const int32_t slot = p - P0;
  if (!single) {
    a.gacc[q] = s;
    if (MODE != 2) a.wsnap[slot] = wj;  // stable copy for Update
    return;
  }
  const float g = s / a.n_f;
  float d, ph;
  propose_f32(g, cj, wj, a.lam, d, ph);
  a.delta[slot] = d;
  a.phi[slot] = ph;
  if (a.gout) a.gout[slot] = g;
  if (MODE != 2) {
    if (a.improve > 0)
      a.wsnap[slot] = wj;  // k_improve writes w_j from the improved increment
    else if (d != 0.0f)
      a.w[j] = wj + d;
  }
}

// Propose (Algorithm 2 / 4).  A column that fits in one piece is finalised
// here (delta, phi; accept-all rules also apply w_j += delta_j).  A split
// column only publishes its partial sums; Update (accept-all rules) or
// Accept (greedy rules) finalise it in the next launch, so no workgroup
// ever waits for another.
// MODE 0: accept all, atomic scatter (Shotgun, stochastic, cyclic)
// MODE 1: accept all, plain scatter (Coloring: rows of a class are disjoint)
// MODE 2: deferred acceptance (Thread-Greedy, Greedy)
// UL: entries per lane per batch on long pieces (piece / 64, 4 or 8).
template <int GS, int MODE, int UL, bool RS>
__global__ __launch_bounds__(kBlock) void k_propose(IterArgs a) {
  const Roles r = roles(a.nl);
  int32_t P0, P1;
  window_of(a, P0, P1);
  if (r.wave < r.nl) {
    const int32_t q1 = a.wbl[a.t + 1];
    for (int64_t q = a.wbl[a.t] + r.wave; q < q1; q += r.nl)
      propose_piece<kWave, MODE, UL, RS>(a, a.desc_l[q], q, r.wl, P0);
  } else {
    const int64_t step = (r.nwaves - r.nl) * (kWave / GS);
    for (int64_t p = P0 + (r.wave - r.nl) * (kWave / GS) + r.wl / GS; p < P1; p += step) {
      const int4 dsc = a.desc_s[p];
      if (desc_len(dsc) == 0) continue;  // long column: the long waves take it
      propose_piece<GS, MODE, kUnroll, RS>(a, dsc, p, r.wl & (GS - 1), P0);
    }
  }
}

// Residual refresh (the r = l'(y, z) of Algorithm 1's state) for a Propose
// that reads it: one pass over the rows.
__global__ __launch_bounds__(kBlock) void k_refresh(int64_t n, int32_t loss, const float4 *zs,
                                                     float *rs) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const float4 zr = zs[i];
    rs[i] = dloss_f32(loss, zr.z, zr.x + zr.y);
  }
}

// Finalise the split columns among positions [lo, hi) of the window: find
// them in parallel (kSplitCap * NT slots, so a 4096-position window is
// searched in one go), then each wave of the NT-thread workgroup takes one
// and sums its partials (in piece order, as Update does) with shuffles, and
// writes delta, phi (and g).  smulti holds kSplitCap * NT entries.
constexpr int kSplitCap = 4;
template <int NT>
__device__ void finalize_split(const IterArgs &a, int64_t lo, int64_t hi, int32_t P0,
                               int32_t *smulti, int32_t *nmulti) {
  const int lane = int(threadIdx.x) & (kWave - 1);
  auto process = [&](int32_t cnt) {
    for (int32_t m = int32_t(threadIdx.x) / kWave; m < cnt; m += NT / kWave) {
      const int32_t p = smulti[m];
      const int32_t pf = a.loff[p], np = a.loff[p + 1] - pf;
      const float g = split_sum(a.gacc, pf, np, lane) / a.n_f;
      if (lane == 0) {
        const int32_t j = a.col_of_pos[p];
        float d, ph;
        propose_f32(g, a.c[j], a.w[j], a.lam, d, ph);
        a.delta[p - P0] = d;
        a.phi[p - P0] = ph;
        if (a.gout) a.gout[p - P0] = g;
      }
    }
  };
  if (threadIdx.x == 0) *nmulti = 0;
  __syncthreads();
  for (int64_t c0 = lo; c0 < hi; c0 += NT) {
    if (*nmulti + NT > kSplitCap * NT) {  // no room for a further NT: finalise these first
      const int32_t cnt = *nmulti;
      process(cnt);
      __syncthreads();
      if (threadIdx.x == 0) *nmulti = 0;
      __syncthreads();
    }
    const int64_t pp = c0 + threadIdx.x;
    if (pp < hi && a.loff[pp + 1] - a.loff[pp] > 1) smulti[atomicAdd(nmulti, 1)] = int32_t(pp);
    __syncthreads();
  }
  process(*nmulti);
  __syncthreads();
}

// Accept for Thread-Greedy / Greedy (section 2.3): in each block of B
// positions the first position with minimal phi.  One workgroup per block;
// it first finalises the block's split columns from their partial sums.
// With `chunk` set, this is the first stage of a global accept (Greedy: one
// block holding the whole window): B is the chunk size, and each workgroup
// only records its chunk's winner in bw_pos / bw_phi for k_accept_final.
__global__ __launch_bounds__(kBlock) void k_accept(IterArgs a, int64_t B, int32_t chunk) {
  __shared__ float sphi[kBlock];
  __shared__ int32_t spos[kBlock];
  __shared__ int32_t smulti[kSplitCap * kBlock];
  __shared__ int32_t nmulti;
  int32_t P0, P1;
  window_of(a, P0, P1);
  const int64_t nblk = (int64_t(P1 - P0) + B - 1) / B;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int64_t lo = P0 + b * B, hi = min(lo + B, int64_t(P1));
    finalize_split<kBlock>(a, lo, hi, P0, smulti, &nmulti);
    float best = INFINITY;
    int32_t bpos = INT32_MAX;
    for (int64_t p = lo + threadIdx.x; p < hi; p += kBlock) {
      a.acc[p - P0] = 0;
      float v = a.phi[p - P0];
      if (v < best) {  // a thread visits its positions in increasing order
        best = v;
        bpos = int32_t(p);
      }
    }
    sphi[threadIdx.x] = best;
    spos[threadIdx.x] = bpos;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < off) {
        float v2 = sphi[threadIdx.x + off];
        int32_t p2 = spos[threadIdx.x + off];
        if (v2 < sphi[threadIdx.x] || (v2 == sphi[threadIdx.x] && p2 < spos[threadIdx.x])) {
          sphi[threadIdx.x] = v2;
          spos[threadIdx.x] = p2;
        }
      }
      __syncthreads();
    }
    if (chunk) {
      if (threadIdx.x == 0) {
        a.bw_pos[b] = spos[0];
        a.bw_phi[b] = __float_as_int(sphi[0]);
      }
    } else if (threadIdx.x == 0 && spos[0] != INT32_MAX) {
      const int32_t p = spos[0];
      a.acc[p - P0] = 1;
      const int32_t j = a.col_of_pos[p];
      const float d = a.delta[p - P0];
      if (a.improve > 0)
        a.wsnap[p - P0] = a.w[j];
      else if (d != 0.0f)
        a.w[j] += d;
      atomicAdd(a.counters + 0, (unsigned long long)(a.col_ptr[j + 1] - a.col_ptr[j]));
      atomicAdd(a.counters + 1, 1ull);
    }
    __syncthreads();
  }
}

// Second stage of the global accept: the first minimal phi over the chunk
// winners (chunks are in position order, so ties still go to the lowest
// position), accepted as k_accept accepts a block's winner.
__global__ __launch_bounds__(kBlock) void k_accept_final(IterArgs a, int64_t nchunks) {
  __shared__ float sphi[kBlock];
  __shared__ int32_t spos[kBlock];
  int32_t P0, P1;
  window_of(a, P0, P1);
  float best = INFINITY;
  int32_t bpos = INT32_MAX;
  for (int64_t b = threadIdx.x; b < nchunks; b += kBlock) {
    const int32_t p = a.bw_pos[b];
    const float v = __int_as_float(a.bw_phi[b]);
    if (p != INT32_MAX && v < best) {
      best = v;
      bpos = p;
    }
  }
  sphi[threadIdx.x] = best;
  spos[threadIdx.x] = bpos;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      float v2 = sphi[threadIdx.x + off];
      int32_t p2 = spos[threadIdx.x + off];
      if (v2 < sphi[threadIdx.x] || (v2 == sphi[threadIdx.x] && p2 < spos[threadIdx.x])) {
        sphi[threadIdx.x] = v2;
        spos[threadIdx.x] = p2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && spos[0] != INT32_MAX) {
    const int32_t p = spos[0];
    a.acc[p - P0] = 1;
    const int32_t j = a.col_of_pos[p];
    const float d = a.delta[p - P0];
    if (a.improve > 0)
      a.wsnap[p - P0] = a.w[j];
    else if (d != 0.0f)
      a.w[j] += d;
    atomicAdd(a.counters + 0, (unsigned long long)(a.col_ptr[j + 1] - a.col_ptr[j]));
    atomicAdd(a.counters + 1, 1ull);
  }
}

// Global acceptance (Thread-Greedy accepting the best |J'| of the window,
// section 4.1): the K = min(accept_top, |window|) positions with the smallest
// (phi, position) keys.  One workgroup finds the K-th smallest 64-bit key
// (phi mapped to an order-preserving integer, -0 folded into +0, in the
// high word; the window offset in the low word) by an 8-pass radix select
// over LDS histograms, then accepts every key up to it: exactly K positions.
constexpr int kTopThreads = 1024;

__device__ __forceinline__ unsigned long long top_key(float phi, int64_t off) {
  uint32_t u = __float_as_uint(phi);
  if ((u & 0x7FFFFFFFu) == 0u) u = 0u;
  u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return (static_cast<unsigned long long>(u) << 32) | static_cast<unsigned long long>(off);
}

// Keys of a window of at most kTopKeys positions are computed once and held
// in registers (kTopKeys / kTopThreads per thread); larger windows re-read
// phi in every pass.  Each wave counts into its own LDS histogram: near
// the optimum most proxies are exactly 0 and share one bin, and a single
// histogram would serialise their atomics.
constexpr int kTopPer = 4;
constexpr int64_t kTopKeys = int64_t(kTopThreads) * kTopPer;
constexpr int kTopWaves = kTopThreads / kWave;

// Exclusive prefix sum over the kTopThreads threads of the workgroup.
__device__ __forceinline__ int32_t top_block_scan(int32_t v, int32_t &total) {
  __shared__ int32_t wsum[kTopWaves];
  const int lane = int(threadIdx.x) & (kWave - 1), wid = int(threadIdx.x) / kWave;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t t = __shfl_up(x, off, kWave);
    if (lane >= off) x += t;
  }
  if (lane == kWave - 1) wsum[wid] = x;
  __syncthreads();
  int32_t pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kTopWaves; ++w) {
    if (w < wid) pre += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

__global__ __launch_bounds__(kTopThreads) void k_accept_top(IterArgs a) {
  __shared__ int32_t smulti[kSplitCap * kTopThreads];
  __shared__ int32_t nmulti;
  __shared__ uint32_t whist[kTopWaves][256];
  __shared__ uint32_t hist[256];
  __shared__ unsigned long long s_prefix;
  __shared__ int64_t s_rank, s_bincnt;
  __shared__ unsigned long long s_cnt[2][kTopWaves];
  int32_t P0, P1;
  window_of(a, P0, P1);
  const int64_t m = int64_t(P1) - P0;
  if (m <= 0) return;
  finalize_split<kTopThreads>(a, P0, P1, P0, smulti, &nmulti);
  const int64_t K = a.accept_top < m ? a.accept_top : m;
  const bool cached = m <= kTopKeys;
  unsigned long long kreg[kTopPer];
#pragma unroll
  for (int u = 0; u < kTopPer; ++u) {
    const int64_t q = int64_t(threadIdx.x) + int64_t(u) * kTopThreads;
    kreg[u] = (cached && q < m) ? top_key(a.phi[q], q) : ~0ull;
  }
  if (threadIdx.x == 0) {
    s_prefix = 0ull;
    s_rank = K;  // 1-based rank of the wanted key among the candidates
  }
  const int wv = int(threadIdx.x) / kWave;
  bool by_rank = false;  // uniform: every thread reads the same shared values
  unsigned long long mask = 0ull;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int u = int(threadIdx.x); u < kTopWaves * 256; u += kTopThreads) (&whist[0][0])[u] = 0u;
    __syncthreads();
    const unsigned long long prefix = s_prefix;
    if (cached) {
#pragma unroll
      for (int u = 0; u < kTopPer; ++u) {
        const int64_t q = int64_t(threadIdx.x) + int64_t(u) * kTopThreads;
        if (q < m && (kreg[u] & mask) == prefix)
          atomicAdd(&whist[wv][(kreg[u] >> shift) & 255ull], 1u);
      }
    } else {
      for (int64_t q = threadIdx.x; q < m; q += kTopThreads) {
        const unsigned long long key = top_key(a.phi[q], q);
        if ((key & mask) == prefix) atomicAdd(&whist[wv][(key >> shift) & 255ull], 1u);
      }
    }
    __syncthreads();
    if (threadIdx.x < 256) {
      uint32_t t = 0u;
#pragma unroll
      for (int w = 0; w < kTopWaves; ++w) t += whist[w][threadIdx.x];
      hist[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
      // the bin holding rank r: wave prefix sum over 4 bins per lane
      const int lane = int(threadIdx.x);
      const int64_t r = s_rank;
      int64_t c[4], tot = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        c[i] = hist[4 * lane + i];
        tot += c[i];
      }
      int64_t incl = tot;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const int64_t o = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += o;
      }
      int64_t cum = incl - tot;
      if (cum < r && r <= incl) {  // exactly one lane
        int i = 0;
        for (; i < 3; ++i) {
          if (cum + c[i] >= r) break;
          cum += c[i];
        }
        s_rank = r - cum;
        s_bincnt = c[i];
        s_prefix = prefix | (static_cast<unsigned long long>(4 * lane + i) << shift);
      }
    }
    mask |= 255ull << shift;
    __syncthreads();
    // after the proxy half of the key: if every candidate left is taken,
    // the positions need no further passes; with cached keys, the ties of
    // the K-th proxy are resolved by position rank (the low half of the key
    // is the position) instead of four more passes
    if (shift == 32) {
      if (s_rank == s_bincnt) {
        if (threadIdx.x == 0) s_prefix |= 0xFFFFFFFFull;
        __syncthreads();
        break;
      }
      if (cached) {
        by_rank = true;
        break;
      }
    }
  }
  const unsigned long long kth = s_prefix;
  unsigned long long nnz = 0ull, cnt = 0ull;
  auto accept = [&](int64_t q, bool take) {
    a.acc[q] = take ? 1 : 0;
    if (take) {
      const int32_t j = a.col_of_pos[P0 + q];
      const float d = a.delta[q];
      if (a.improve > 0)
        a.wsnap[q] = a.w[j];
      else if (d != 0.0f)
        a.w[j] += d;
      nnz += static_cast<unsigned long long>(a.col_ptr[j + 1] - a.col_ptr[j]);
      cnt += 1ull;
    }
  };
  if (by_rank) {
    // every key whose proxy half is below the K-th one, and the first s_rank
    // (in position order) of those equal to it
    const uint32_t ph = uint32_t(kth >> 32);
    const int64_t rk = s_rank;
    int64_t before = 0;  // tied keys in the earlier segments of positions
#pragma unroll
    for (int u = 0; u < kTopPer; ++u) {
      const int64_t q = int64_t(threadIdx.x) + int64_t(u) * kTopThreads;
      const uint32_t kh = uint32_t(kreg[u] >> 32);
      const bool tie = q < m && kh == ph;
      int32_t seg;
      const int32_t ex = top_block_scan(tie ? 1 : 0, seg);
      if (q < m) accept(q, kh < ph || (tie && before + ex < rk));
      before += seg;
    }
  } else if (cached) {
#pragma unroll
    for (int u = 0; u < kTopPer; ++u) {
      const int64_t q = int64_t(threadIdx.x) + int64_t(u) * kTopThreads;
      if (q < m) accept(q, kreg[u] <= kth);
    }
  } else {
    for (int64_t q = threadIdx.x; q < m; q += kTopThreads) accept(q, top_key(a.phi[q], q) <= kth);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    nnz += __shfl_xor(nnz, off);
    cnt += __shfl_xor(cnt, off);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_cnt[0][threadIdx.x / kWave] = nnz;
    s_cnt[1][threadIdx.x / kWave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tn = 0ull, tc = 0ull;
    for (int w = 0; w < kTopWaves; ++w) {
      tn += s_cnt[0][w];
      tc += s_cnt[1][w];
    }
    atomicAdd(a.counters + 0, tn);
    atomicAdd(a.counters + 1, tc);
  }
}

// Scatter z += d x over one piece (G lanes), U entries per lane per batch.
template <int G, int U>
__device__ __forceinline__ void load_batch(const IterArgs &a, int64_t beg, int32_t len,
                                           int32_t base, int lane, int32_t (&ri)[U],
                                           float (&vv)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int32_t e = base + u * G + lane;
    ri[u] = e < len ? a.row_idx[beg + e] : -1;
    vv[u] = e < len ? a.val[beg + e] : 0.0f;
  }
}

template <int MODE, int U>
__device__ __forceinline__ void scatter_batch(const IterArgs &a, const int32_t (&ri)[U],
                                              const float (&vv)[U], float d) {
  if (MODE == 1) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ri[u] >= 0) scatter_plain(a.zs, ri[u], d, vv[u]);
  } else if (!a.exact_accum) {
    // increments accumulate in the low word (non-returning atomics); the
    // pair is renormalised exactly at the end of the epoch
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ri[u] >= 0) atomicAdd(&a.zs[ri[u]].y, d * vv[u]);
  } else {
    // issue all the returning atomics first, then the compensations
    float pp[U], old[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      pp[u] = d * vv[u];
      old[u] = ri[u] >= 0 ? atomicAdd(&a.zs[ri[u]].x, pp[u]) : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ri[u] < 0) continue;
      const float corr = twosum_err(old[u], pp[u]) + fmaf(d, vv[u], -pp[u]);
      if (corr != 0.0f) atomicAdd(&a.zs[ri[u]].y, corr);
    }
  }
}

// Entries from `from` on (batches of G * U).
template <int G, int MODE, int U = kUnroll>
__device__ __forceinline__ void scatter_piece(const IterArgs &a, int64_t beg, int32_t len, float d,
                                              int lane, int32_t from = 0) {
  for (int32_t base = from; base < len; base += G * U) {
    int32_t ri[U];
    float vv[U];
    load_batch<G, U>(a, beg, len, base, lane, ri, vv);
    scatter_batch<MODE, U>(a, ri, vv, d);
  }
}

// Update (Algorithm 3): z += delta_j X_j for the accepted, nonzero proposals.
// Accept-all rules finalise split columns here: every piece recomputes the
// same delta from the partial sums and the weight snapshot; the column's
// first piece writes w_j, delta_j and phi_j.
template <int GS, int MODE, int UL>
__global__ __launch_bounds__(kBlock) void k_update(IterArgs a) {
  const Roles r = roles(a.nl);
  int32_t P0, P1;
  window_of(a, P0, P1);
  uint32_t scattered = 0;  // nonzeros this lane's group scattered (counted with a.scat)
  if (r.wave < r.nl) {
    const int32_t q1 = a.wbl[a.t + 1];
    for (int64_t q = a.wbl[a.t] + r.wave; q < q1; q += r.nl) {
      const int4 dsc = a.desc_l[q];
      const int32_t slot = dsc.z - P0;
      float d;
      if (MODE == 2) {
        if (!a.acc[slot]) continue;
        d = a.delta[slot];
      } else if (desc_single(dsc) || a.improve > 0) {
        d = a.delta[slot];  // single piece, or improved by k_improve
      } else {
        const int32_t pf = a.loff[dsc.z], np = a.loff[dsc.z + 1] - pf;
        const int32_t j = dsc.y;
        const float ws = a.wsnap[slot];
        const float cj = a.c[j];
        const float g = split_sum(a.gacc, pf, np, r.wl) / a.n_f;
        float ph;
        propose_f32(g, cj, ws, a.lam, d, ph);
        if (q == pf && r.wl == 0) {
          a.delta[slot] = d;
          a.phi[slot] = ph;
          if (a.gout) a.gout[slot] = g;
          if (d != 0.0f) a.w[j] = ws + d;
        }
      }
      if (d == 0.0f) continue;
      if (r.wl == 0) scattered += uint32_t(desc_len(dsc));
      scatter_piece<kWave, MODE, UL>(a, desc_beg(dsc), desc_len(dsc), d, r.wl);
    }
  } else {
    const int64_t step = (r.nwaves - r.nl) * (kWave / GS);
    const int lane = r.wl & (GS - 1);
    for (int64_t p = P0 + (r.wave - r.nl) * (kWave / GS) + r.wl / GS; p < P1; p += step) {
      const int4 dsc = a.desc_s[p];  // loads of dsc, acc and delta are independent
      const int64_t slot = p - P0;
      if (MODE == 2 && !a.acc[slot]) continue;
      const float d = a.delta[slot];
      if (d == 0.0f || desc_len(dsc) == 0) continue;
      if (lane == 0) scattered += uint32_t(desc_len(dsc));
      scatter_piece<GS, MODE>(a, desc_beg(dsc), desc_len(dsc), d, lane);
    }
  }
  if (a.scat) {  // profiling only: one atomic per wave, spread over the replica lines
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) scattered += __shfl_xor(scattered, off);
    if (r.wl == 0 && scattered > 0)
      atomicAdd(a.scat + (blockIdx.x % kChkRep) * 16, (unsigned long long)scattered);
  }
}

// Exact renormalisation of the fitted values: (z_hi, z_lo) <- TwoSum.
__global__ __launch_bounds__(kBlock) void k_renorm(int64_t n, float4 *zs) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    float2 *hl = reinterpret_cast<float2 *>(zs + i);
    const float2 v = *hl;
    *hl = make_float2(v.x + v.y, twosum_err(v.x, v.y));
  }
}

int launch_renorm(int64_t n, float4 *zs, hipStream_t s) {
  hipLaunchKernelGGL(k_renorm, dim3(grid_for(n, 2048)), dim3(kBlock), 0, s, n, zs);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

__global__ __launch_bounds__(kBlock) void k_pack_state(int64_t n, const float *z_hi,
                                                        const float *z_lo, const float *y,
                                                        float4 *zs) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    zs[i] = make_float4(z_hi[i], z_lo[i], y[i], 0.0f);
}

__global__ __launch_bounds__(kBlock) void k_unpack_state(int64_t n, const float4 *zs, float *z_hi,
                                                          float *z_lo) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const float4 v = zs[i];
    z_hi[i] = v.x;
    z_lo[i] = v.y;
  }
}

int launch_pack_state(int64_t n, const float *z_hi, const float *z_lo, const float *y, float4 *zs,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_pack_state, dim3(grid_for(n)), dim3(kBlock), 0, s, n, z_hi, z_lo, y, zs);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

int launch_unpack_state(int64_t n, const float4 *zs, float *z_hi, float *z_lo, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack_state, dim3(grid_for(n)), dim3(kBlock), 0, s, n, zs, z_hi, z_lo);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// "Improve delta_j" (Algorithm 3, section 4.1): one wave per accepted
// position of the window runs up to `improve` further quadratic-
// approximation steps on the column's 1-D objective from the state at the
// start of the iteration:
//   g = (1/n) sum_i x_ij l'(y_i, z_i + d x_ij),  d += Eq. 7 increment at w_j + d,
// stopping once a step no longer changes d in FP32.  The first
// kImproveRegs * 64 entries stay in registers across steps; longer columns
// re-read the rest each step.  Split columns (accept-all rules) get their
// first increment here from the partial sums.  Writes delta and w_j =
// wsnap + d (Propose / Accept left w_j untouched and its value in wsnap).
constexpr int kImproveRegs = 4;

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_improve(IterArgs a) {
  int32_t P0, P1;
  window_of(a, P0, P1);
  const int lane = int(threadIdx.x) & (kWave - 1);
  const int64_t nw = int64_t(gridDim.x) * (kBlock / kWave);
  for (int64_t p = P0 + (int64_t(blockIdx.x) * kBlock + threadIdx.x) / kWave; p < P1; p += nw) {
    const int64_t slot = p - P0;
    if (MODE == 2 && !a.acc[slot]) continue;
    const int32_t j = a.col_of_pos[p];
    const int64_t cb = a.col_ptr[j];
    const int64_t len = a.col_ptr[j + 1] - cb;
    const float cj = a.c[j];
    const float w0 = a.wsnap[slot];
    float d;
    if (MODE != 2 && a.loff[p + 1] - a.loff[p] > 1) {
      const int32_t pf = a.loff[p], np = a.loff[p + 1] - pf;
      const float g = split_sum(a.gacc, pf, np, lane) / a.n_f;
      float ph;
      propose_f32(g, cj, w0, a.lam, d, ph);
      if (lane == 0) {
        a.phi[slot] = ph;
        if (a.gout) a.gout[slot] = g;
      }
    } else {
      d = a.delta[slot];
    }
    if (d != 0.0f) {
      int32_t ri[kImproveRegs];
      float vv[kImproveRegs], zb[kImproveRegs], yy[kImproveRegs];
#pragma unroll
      for (int u = 0; u < kImproveRegs; ++u) {
        const int64_t e = int64_t(u) * kWave + lane;
        ri[u] = e < len ? a.row_idx[cb + e] : -1;
        vv[u] = e < len ? a.val[cb + e] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < kImproveRegs; ++u) {
        const float4 zr = a.zs[ri[u] >= 0 ? ri[u] : 0];
        zb[u] = zr.x + zr.y;
        yy[u] = zr.z;
      }
      for (int32_t s = 0; s < a.improve; ++s) {
        float sum = 0.0f;
#pragma unroll
        for (int u = 0; u < kImproveRegs; ++u)
          if (ri[u] >= 0) sum += vv[u] * dloss_f32(a.loss, yy[u], zb[u] + d * vv[u]);
        for (int64_t e0 = int64_t(kImproveRegs) * kWave + lane; e0 < len;
             e0 += int64_t(kUnroll) * kWave) {
          int32_t rj[kUnroll];
          float vj[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            const int64_t e = e0 + int64_t(u) * kWave;
            rj[u] = e < len ? a.row_idx[cb + e] : -1;
            vj[u] = e < len ? a.val[cb + e] : 0.0f;
          }
          float4 zr[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) zr[u] = a.zs[rj[u] >= 0 ? rj[u] : 0];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u)
            if (rj[u] >= 0) sum += vj[u] * dloss_f32(a.loss, zr[u].z, (zr[u].x + zr[u].y) + d * vj[u]);
        }
        const float g = group_sum<kWave>(sum) / a.n_f;  // identical in every lane
        float inc, ph;
        propose_f32(g, cj, w0 + d, a.lam, inc, ph);
        const float dn = d + inc;
        if (dn == d) break;  // the step no longer changes d: every later one would repeat it
        d = dn;
      }
    }
    if (lane == 0) {
      a.delta[slot] = d;
      a.w[j] = w0 + d;
    }
  }
}

// positions per first-stage workgroup of a global accept
constexpr int64_t kAcceptChunk = 2048;

// With events, Propose is launched through the extension that stamps the
// kernel's own dispatch with them.
template <void (*K)(IterArgs)>
static void launch_propose(const IterArgs &a, dim3 grid, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  if (ev0 && ev1)
    hipExtLaunchKernelGGL(K, grid, dim3(kBlock), 0, s, ev0, ev1, 0, a);
  else
    hipLaunchKernelGGL(K, grid, dim3(kBlock), 0, s, a);
}

template <void (*K)(IterArgs)>
static void launch_update(const IterArgs &a, dim3 grid, hipStream_t s, hipEvent_t ev2,
                          hipEvent_t ev3) {
  launch_propose<K>(a, grid, s, ev2, ev3);
}

template <int GS, int UL>
static int launch_iteration_g(const IterArgs &a, int mode, int64_t block, unsigned blocks,
                              int64_t nblocks_accept, unsigned improve_blocks, hipStream_t s,
                              hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2, hipEvent_t ev3) {
  const dim3 grid(blocks), blk(kBlock);
  if (a.rs) {
    hipLaunchKernelGGL(k_refresh, dim3(grid_for(a.nrows)), blk, 0, s, a.nrows, a.loss, a.zs, a.rs);
    if (mode == 0)
      launch_propose<k_propose<GS, 0, UL, true>>(a, grid, s, ev0, ev1);
    else if (mode == 1)
      launch_propose<k_propose<GS, 1, UL, true>>(a, grid, s, ev0, ev1);
    else
      launch_propose<k_propose<GS, 2, UL, true>>(a, grid, s, ev0, ev1);
  } else if (mode == 0) {
    launch_propose<k_propose<GS, 0, UL, false>>(a, grid, s, ev0, ev1);
  } else if (mode == 1) {
    launch_propose<k_propose<GS, 1, UL, false>>(a, grid, s, ev0, ev1);
  } else {
    launch_propose<k_propose<GS, 2, UL, false>>(a, grid, s, ev0, ev1);
  }
  if (mode == 0) {
    if (a.improve > 0)
      hipLaunchKernelGGL(k_improve<0>, dim3(improve_blocks), blk, 0, s, a);
    launch_update<k_update<GS, 0, UL>>(a, grid, s, ev2, ev3);
  } else if (mode == 1) {
    if (a.improve > 0)
      hipLaunchKernelGGL(k_improve<1>, dim3(improve_blocks), blk, 0, s, a);
    launch_update<k_update<GS, 1, UL>>(a, grid, s, ev2, ev3);
  } else {
    if (a.accept_top > 0) {
      hipLaunchKernelGGL(k_accept_top, dim3(1), dim3(kTopThreads), 0, s, a);
    } else if (nblocks_accept == 1 && block > kAcceptChunk) {
      // one block over the whole window (Greedy): chunk winners, then the best
      const int64_t nc = (block + kAcceptChunk - 1) / kAcceptChunk;
      hipLaunchKernelGGL(k_accept, dim3(unsigned(nc < 4096 ? nc : 4096)), blk, 0, s, a,
                         int64_t(kAcceptChunk), 1);
      hipLaunchKernelGGL(k_accept_final, dim3(1), blk, 0, s, a, nc);
    } else {
      unsigned nb =
          unsigned(nblocks_accept < 4096 ? (nblocks_accept > 0 ? nblocks_accept : 1) : 4096);
      hipLaunchKernelGGL(k_accept, dim3(nb), blk, 0, s, a, block, 0);
    }
    if (a.improve > 0)
      hipLaunchKernelGGL(k_improve<2>, dim3(improve_blocks), blk, 0, s, a);
    launch_update<k_update<GS, 2, UL>>(a, grid, s, ev2, ev3);
  }
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

template <int GS>
static int launch_iteration_u(const IterArgs &a, int mode, int64_t block, unsigned blocks,
                              int64_t nblocks_accept, unsigned improve_blocks, hipStream_t s,
                              hipEvent_t ev0, hipEvent_t ev1, hipEvent_t ev2, hipEvent_t ev3) {
  if (a.piece <= kWave * kUnroll)
    return launch_iteration_g<GS, kUnroll>(a, mode, block, blocks, nblocks_accept, improve_blocks,
                                           s, ev0, ev1, ev2, ev3);
  return launch_iteration_g<GS, 2 * kUnroll>(a, mode, block, blocks, nblocks_accept,
                                             improve_blocks, s, ev0, ev1, ev2, ev3);
}

// ---------------------------------------------------------------------------
// Fused asynchronous Shotgun (accept-all rules, GENCD_FUSED): Propose and
// Update in one launch, as section 4.1 notes Shotgun allows.  Each column
// forms g from the current z (other columns of its window may already have
// updated shared rows), takes its Eq. 7 step and scatters at once.  A split
// column publishes partial sums and w_j (position-indexed snapshot); the
// next launch, or the flush launch at the end of the epoch, applies it.
// ---------------------------------------------------------------------------
template <int G, int U>
__device__ __forceinline__ void fused_column(const IterArgs &a, int64_t beg, int32_t len,
                                             int32_t j, int lane) {
  const float wj = a.w[j], cj = a.c[j];  // the same address in every lane: one load each
  float s = 0.0f;
  int32_t ri[U];
  float vv[U];
  for (int32_t base = 0; base < len; base += G * U) {
    load_batch<G, U>(a, beg, len, base, lane, ri, vv);
    float zh[U], zl[U], yy[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float4 zr = a.zs[ri[u] >= 0 ? ri[u] : 0];
      zh[u] = zr.x;
      zl[u] = zr.y;
      yy[u] = zr.z;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (ri[u] >= 0) s += vv[u] * dloss_f32(a.loss, yy[u], zh[u] + zl[u]);
  }
  s = group_sum<G>(s);  // identical in every lane of the group
  float d, ph;
  propose_f32(s / a.n_f, cj, wj, a.lam, d, ph);
  if (d == 0.0f) return;
  if (lane == 0) a.w[j] = wj + d;
  if (len <= G * U)
    scatter_batch<0, U>(a, ri, vv, d);  // the only batch is still in registers
  else
    scatter_piece<G, 0, U>(a, beg, len, d, lane);
}

template <int GS, int UL>
__global__ __launch_bounds__(kBlock) void k_fused(IterArgs a, int32_t flush) {
  const Roles r = roles(a.nl);
  int32_t P0 = 0, P1 = 0;
  if (!flush) window_of(a, P0, P1);
  if (r.wave < r.nl) {
    // current window's pieces, then the previous window's split pieces
    const int32_t q0 = flush ? 0 : a.wbl[a.t], q1 = flush ? 0 : a.wbl[a.t + 1];
    const int32_t qp0 = a.t > 0 ? a.wbl[a.t - 1] : 0, qp1 = a.t > 0 ? a.wbl[a.t] : 0;
    const int64_t ncur = q1 - q0, ntot = ncur + (qp1 - qp0);
    for (int64_t u = r.wave; u < ntot; u += r.nl) {
      if (u < ncur) {
        const int64_t q = q0 + u;
        const int4 dsc = a.desc_l[q];
        if (desc_single(dsc)) {
          fused_column<kWave, UL>(a, desc_beg(dsc), desc_len(dsc), dsc.y, r.wl);
        } else {
          // partial gradient of a split column, and its weight at this time
          const int64_t beg = desc_beg(dsc);
          const int32_t len = desc_len(dsc);
          float s = 0.0f;
          for (int32_t base = 0; base < len; base += kWave * UL) {
            int32_t ri[UL];
            float vv[UL];
            load_batch<kWave, UL>(a, beg, len, base, r.wl, ri, vv);
#pragma unroll
            for (int v = 0; v < UL; ++v) {
              const float4 zr = a.zs[ri[v] >= 0 ? ri[v] : 0];
              if (ri[v] >= 0) s += vv[v] * dloss_f32(a.loss, zr.z, zr.x + zr.y);
            }
          }
          s = group_sum<kWave>(s);
          if (r.wl == 0) {
            a.gacc[q] = s;
            a.wsnap[dsc.z] = a.w[dsc.y];
          }
        }
      } else {
        const int64_t q = qp0 + (u - ncur);
        const int4 dsc = a.desc_l[q];
        if (desc_single(dsc)) continue;  // applied in its own launch
        const int32_t p = dsc.z, j = dsc.y;
        const int32_t pf = a.loff[p], np = a.loff[p + 1] - pf;
        const float ws = a.wsnap[p];
        const float g = split_sum(a.gacc, pf, np, r.wl) / a.n_f;
        float d, ph;
        propose_f32(g, a.c[j], ws, a.lam, d, ph);
        if (d == 0.0f) continue;
        if (q == pf && r.wl == 0) a.w[j] = ws + d;
        scatter_piece<kWave, 0, UL>(a, desc_beg(dsc), desc_len(dsc), d, r.wl);
      }
    }
  } else {
    const int64_t step = (r.nwaves - r.nl) * (kWave / GS);
    const int lane = r.wl & (GS - 1);
    for (int64_t p = P0 + (r.wave - r.nl) * (kWave / GS) + r.wl / GS; p < P1; p += step) {
      const int4 dsc = a.desc_s[p];
      if (desc_len(dsc) == 0) continue;  // long column: the long waves take it
      fused_column<GS, kUnroll>(a, desc_beg(dsc), desc_len(dsc), dsc.y, lane);
    }
  }
}

template <int GS>
static void launch_fused_g(const IterArgs &a, unsigned blocks, bool flush, hipStream_t s) {
  if (a.piece <= kWave * kUnroll)
    hipLaunchKernelGGL((k_fused<GS, kUnroll>), dim3(blocks), dim3(kBlock), 0, s, a, int32_t(flush));
  else
    hipLaunchKernelGGL((k_fused<GS, 2 * kUnroll>), dim3(blocks), dim3(kBlock), 0, s, a,
                       int32_t(flush));
}

int launch_fused(const IterArgs &a, int group, int64_t short_bound, int64_t long_bound, bool flush,
                 hipStream_t s) {
  IterArgs b = a;
  unsigned blocks;
  int32_t nl;
  two_class_grid(flush ? 0 : short_bound, long_bound, group, &blocks, &nl);
  b.nl = nl;
  switch (group) {
    case 4: launch_fused_g<4>(b, blocks, flush, s); break;
    case 8: launch_fused_g<8>(b, blocks, flush, s); break;
    case 16: launch_fused_g<16>(b, blocks, flush, s); break;
    default: launch_fused_g<32>(b, blocks, flush, s); break;
  }
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

int launch_iteration(const IterArgs &a, int group, int mode, int64_t block, int64_t short_bound,
                     int64_t long_bound, int64_t nblocks_accept, hipStream_t s, hipEvent_t ev0,
                     hipEvent_t ev1, hipEvent_t ev2, hipEvent_t ev3) {
  IterArgs b = a;
  unsigned blocks;
  int32_t nl;
  two_class_grid(short_bound, long_bound, group, &blocks, &nl);
  b.nl = nl;
  // k_improve: one wave per window position (grid-stride beyond 16384 blocks)
  const int64_t ib = (short_bound + kBlock / kWave - 1) / (kBlock / kWave);
  const unsigned iblocks = unsigned(ib < 1 ? 1 : (ib > 16384 ? 16384 : ib));
  switch (group) {
    case 4:
      return launch_iteration_u<4>(b, mode, block, blocks, nblocks_accept, iblocks, s, ev0, ev1,
                                   ev2, ev3);
    case 8:
      return launch_iteration_u<8>(b, mode, block, blocks, nblocks_accept, iblocks, s, ev0, ev1,
                                   ev2, ev3);
    case 16:
      return launch_iteration_u<16>(b, mode, block, blocks, nblocks_accept, iblocks, s, ev0, ev1,
                                    ev2, ev3);
    default:
      return launch_iteration_u<32>(b, mode, block, blocks, nblocks_accept, iblocks, s, ev0, ev1,
                                    ev2, ev3);
  }
}

// ---------------------------------------------------------------------------
// FP64 check: z64 = Xw, loss, r64 = l'(y, z64), g64 = X^T r64 / n, KKT, |w|_1,
// duality gap (and the FP32 re-sync z_hi + z_lo = z64)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_check_zero(double *z64, int64_t n, double *g64,
                                                        int64_t k, unsigned long long *red,
                                                        unsigned long long *rep) {
  const int64_t tid = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t nt = int64_t(gridDim.x) * kBlock;
  for (int64_t i = tid; i < n; i += nt) z64[i] = 0.0;
  for (int64_t j = tid; j < k; j += nt) g64[j] = 0.0;
  if (tid < 8) red[tid] = 0ull;
  for (int64_t i = tid; i < int64_t(kChkRep) * 16; i += nt) rep[i] = 0ull;
}

static_assert(kChkRep == kWave, "k_check_dual folds the replicas with one wave");

// This workgroup's replica line of the check reductions.
__device__ __forceinline__ unsigned long long *rep_line(unsigned long long *rep) {
  return rep + (blockIdx.x % kChkRep) * 16;
}

// With nb > 1 the products of the preset blocks are kept apart:
// z64[row * nb + block of the column] (Block Shotgun's power iteration).
template <int G, typename WT>
__device__ __forceinline__ void spmv_piece(const int32_t *row_idx, const float *val, const int4 d,
                                           const WT *w, double *z64, int lane, int64_t nb = 1,
                                           const int32_t *bcol = nullptr) {
  const double wj = double(w[d.y]);
  if (wj == 0.0) return;
  const int64_t b = bcol ? int64_t(bcol[d.y]) : 0;
  const int64_t beg = desc_beg(d);
  const int32_t len = desc_len(d);
  for (int32_t base = 0; base < len; base += G * kUnroll) {
    int32_t ri[kUnroll];
    float vv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int32_t e = base + u * G + lane;
      ri[u] = e < len ? row_idx[beg + e] : -1;
      vv[u] = e < len ? val[beg + e] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (ri[u] >= 0) atomicAdd(&z64[int64_t(ri[u]) * nb + b], wj * double(vv[u]));
  }
}

// z64 += X w over all pieces (w float for the check, double for the
// spectral-radius iteration; nb > 1: per preset block, see spmv_piece)
template <int GS, typename WT>
__global__ __launch_bounds__(kBlock) void k_check_spmv(const int32_t *row_idx, const float *val,
                                                        const int4 *ds, int32_t ns,
                                                        const int4 *dl, int32_t nlp, int32_t nl_req,
                                                        const WT *w, double *z64, int64_t nb = 1,
                                                        const int32_t *bcol = nullptr) {
  const Roles r = roles(nl_req);
  if (r.wave < r.nl) {
    for (int64_t q = r.wave; q < nlp; q += r.nl)
      spmv_piece<kWave, WT>(row_idx, val, dl[q], w, z64, r.wl, nb, bcol);
  } else {
    const int64_t step = (r.nwaves - r.nl) * (kWave / GS);
    for (int64_t q = (r.wave - r.nl) * (kWave / GS) + r.wl / GS; q < ns; q += step)
      spmv_piece<GS, WT>(row_idx, val, ds[q], w, z64, r.wl & (GS - 1), nb, bcol);
  }
}

// Loss sum, residual and (zs non-null) the re-sync of the FP32 state.  The
// re-sync also measures how far the accumulated pair z_hi + z_lo drifted
// from z64: max_i |z_i - z64_i| into replica word 6 (bit pattern of a
// non-negative double) and sum_i z64_i^2 into word 7.
__global__ __launch_bounds__(kBlock) void k_check_rows(int64_t n, int loss, const float *y,
                                                        const double *z64, double *r64,
                                                        float4 *zs, unsigned long long *rep) {
  __shared__ double sred[kBlock], sdr[kBlock], ssq[kBlock];
  double acc = 0.0, drift = 0.0, sq = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const double t = z64[i];
    const double yi = double(y[i]);
    acc += loss_f64(loss, yi, t);
    r64[i] = dloss_f64(loss, yi, t);
    if (zs) {  // re-sync: z_hi + z_lo = z64 to about 2^-48 relative, and the label
      const float4 old = zs[i];
      const double dv = fabs((double(old.x) + double(old.y)) - t);
      if (!(dv <= drift)) drift = dv;  // propagates NaN
      sq += t * t;
      const float h = float(t);
      zs[i] = make_float4(h, float(t - double(h)), y[i], 0.0f);
    }
  }
  sred[threadIdx.x] = acc;
  sdr[threadIdx.x] = drift;
  ssq[threadIdx.x] = sq;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      sred[threadIdx.x] += sred[threadIdx.x + off];
      ssq[threadIdx.x] += ssq[threadIdx.x + off];
      const double o = sdr[threadIdx.x + off];
      if (!(o <= sdr[threadIdx.x])) sdr[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    unsigned long long *line = rep_line(rep);
    atomicAdd(reinterpret_cast<double *>(line), sred[0]);
    if (zs) {
      const double m = sdr[0];
      atomicMax(line + 6, (m != m) ? 0x7FF8000000000000ull : (unsigned long long)__double_as_longlong(m));
      atomicAdd(reinterpret_cast<double *>(line + 7), ssq[0]);
    }
  }
}

template <int G>
__device__ __forceinline__ void cols_piece(const int32_t *row_idx, const float *val, const int4 d,
                                           const double *r64, double *g64, int lane,
                                           int64_t nb = 1, const int32_t *bcol = nullptr) {
  const int64_t beg = desc_beg(d);
  const int32_t len = desc_len(d);
  const int64_t b = bcol ? int64_t(bcol[d.y]) : 0;
  double s = 0.0;
  for (int32_t base = 0; base < len; base += G * kUnroll) {
    int32_t ri[kUnroll];
    float vv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int32_t e = base + u * G + lane;
      ri[u] = e < len ? row_idx[beg + e] : -1;
      vv[u] = e < len ? val[beg + e] : 0.0f;
    }
    double rr[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) rr[u] = r64[int64_t(ri[u] >= 0 ? ri[u] : 0) * nb + b];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (ri[u] >= 0) s += double(vv[u]) * rr[u];
  }
  s = group_sum<G>(s);
  if (lane == 0) {
    if (desc_single(d))
      g64[d.y] = s;
    else
      atomicAdd(&g64[d.y], s);
  }
}

template <int GS>
__global__ __launch_bounds__(kBlock) void k_check_cols(const int32_t *row_idx, const float *val,
                                                        const int4 *ds, int32_t ns,
                                                        const int4 *dl, int32_t nlp, int32_t nl_req,
                                                        const double *r64, double *g64,
                                                        int64_t nb = 1,
                                                        const int32_t *bcol = nullptr) {
  const Roles r = roles(nl_req);
  if (r.wave < r.nl) {
    for (int64_t q = r.wave; q < nlp; q += r.nl)
      cols_piece<kWave>(row_idx, val, dl[q], r64, g64, r.wl, nb, bcol);
  } else {
    const int64_t step = (r.nwaves - r.nl) * (kWave / GS);
    for (int64_t q = (r.wave - r.nl) * (kWave / GS) + r.wl / GS; q < ns; q += step)
      cols_piece<GS>(row_idx, val, ds[q], r64, g64, r.wl & (GS - 1), nb, bcol);
  }
}

__global__ __launch_bounds__(kBlock) void k_check_kkt(int64_t k, double *g64, const float *w,
                                                       double lam, double inv_n,
                                                       unsigned long long *rep) {
  __shared__ double smax[kBlock], sl1[kBlock], sgm[kBlock];
  __shared__ unsigned long long snz[kBlock];
  double vmax = 0.0, l1 = 0.0, gmax = 0.0;
  unsigned long long nz = 0;
  // four columns per thread and round: their loads are issued together
  constexpr int U = 4;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t j0 = int64_t(blockIdx.x) * kBlock + threadIdx.x; j0 < k; j0 += U * stride) {
    double gv[U], wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + u * stride;
      gv[u] = j < k ? g64[j] : 0.0;
      wv[u] = (w && j < k) ? double(w[j]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + u * stride;
      if (j >= k) break;
      const double g = gv[u] * inv_n;
      g64[j] = g;
      if (!(fabs(g) <= gmax)) gmax = fabs(g);
      const double wj = wv[u];
      double v;
      if (wj != 0.0) {
        v = fabs(g + (wj > 0.0 ? lam : -lam));
        l1 += fabs(wj);
        ++nz;
      } else {
        v = fabs(g) - lam;
        if (v < 0.0) v = 0.0;
      }
      if (!(v <= vmax)) vmax = v;  // propagates NaN
    }
  }
  smax[threadIdx.x] = vmax;
  sl1[threadIdx.x] = l1;
  snz[threadIdx.x] = nz;
  sgm[threadIdx.x] = gmax;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      double o = smax[threadIdx.x + off];
      if (!(o <= smax[threadIdx.x])) smax[threadIdx.x] = o;
      double o2 = sgm[threadIdx.x + off];
      if (!(o2 <= sgm[threadIdx.x])) sgm[threadIdx.x] = o2;
      sl1[threadIdx.x] += sl1[threadIdx.x + off];
      snz[threadIdx.x] += snz[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    unsigned long long *red = rep_line(rep);
    double m = smax[0];
    unsigned long long bits = (m != m) ? 0x7FF8000000000000ull : __double_as_longlong(m);
    atomicMax(&red[2], bits);  // non-negative doubles order like their bit patterns
    double gm = sgm[0];
    atomicMax(&red[4], (gm != gm) ? 0x7FF8000000000000ull : __double_as_longlong(gm));
    atomicAdd(reinterpret_cast<double *>(&red[1]), sl1[0]);
    atomicAdd(&red[3], snz[0]);
  }
}

// Dual objective of Eq. (1) at u = s l'(y, z64) / n (summand over rows; the
// scale s = min(1, lambda / |g|_inf) uses the maximum of the previous pass).
__global__ __launch_bounds__(kBlock) void k_check_dual(int64_t n, int loss, const float *y,
                                                        const double *r64, double lam,
                                                        unsigned long long *rep) {
  __shared__ double sred[kBlock];
  __shared__ unsigned long long sgm;
  if (threadIdx.x < kWave) {  // |g|_inf: the maximum over the replicas (kChkRep == kWave)
    unsigned long long v = rep[threadIdx.x * 16 + 4];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
      const unsigned long long o = __shfl_xor(v, off);
      v = o > v ? o : v;
    }
    if (threadIdx.x == 0) sgm = v;
  }
  __syncthreads();
  const double gm = __longlong_as_double((long long)sgm);
  const double s = (gm > lam) ? lam / gm : 1.0;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const double v = s * r64[i];  // n u_i
    const double yi = double(y[i]);
    if (loss == GENCD_SQUARED) {
      acc -= v * yi + 0.5 * v * v;
    } else {
      const double p = -v * yi;  // in [0, 1): binary entropy
      double h = 0.0;
      if (p > 0.0) h -= p * log(p);
      if (p < 1.0) h -= (1.0 - p) * log1p(-p);
      acc += h;
    }
  }
  sred[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sred[threadIdx.x] += sred[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(reinterpret_cast<double *>(rep_line(rep) + 5), sred[0]);
}

int launch_check(const gencd_csc *X, const float *y, int loss, double lam, const float *w,
                 int32_t n_short, int32_t n_lpieces, const Ws &ws, bool resync, hipStream_t s) {
  unsigned long long *red = reinterpret_cast<unsigned long long *>(ws.red);
  const int64_t nk = X->n > X->k ? X->n : X->k;
  unsigned blocks;
  int32_t nl;
  two_class_grid(n_short, n_lpieces, 8, &blocks, &nl);
  unsigned long long *rep = reinterpret_cast<unsigned long long *>(ws.rrep);
  hipLaunchKernelGGL(k_check_zero, dim3(grid_for(nk)), dim3(kBlock), 0, s, ws.z64, X->n, ws.g64,
                     X->k, red, rep);
  if (w && n_short + n_lpieces > 0)
    hipLaunchKernelGGL((k_check_spmv<8, float>), dim3(blocks), dim3(kBlock), 0, s, X->row_idx,
                       X->val, ws.desc_all_s, n_short, ws.desc_all_l, n_lpieces, nl, w, ws.z64);
  hipLaunchKernelGGL(k_check_rows, dim3(grid_for(X->n, 256)), dim3(kBlock), 0, s, X->n, loss, y,
                     ws.z64, ws.r64, resync ? ws.zs : nullptr, rep);
  if (n_short + n_lpieces > 0)
    hipLaunchKernelGGL(k_check_cols<8>, dim3(blocks), dim3(kBlock), 0, s, X->row_idx, X->val,
                       ws.desc_all_s, n_short, ws.desc_all_l, n_lpieces, nl, ws.r64, ws.g64);
  hipLaunchKernelGGL(k_check_kkt, dim3(grid_for(X->k, 256)), dim3(kBlock), 0, s, X->k, ws.g64, w,
                     lam, 1.0 / double(X->n), rep);
  hipLaunchKernelGGL(k_check_dual, dim3(grid_for(X->n, 256)), dim3(kBlock), 0, s, X->n, loss, y,
                     ws.r64, lam, rep);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Spectral radius of G = D^{-1/2} X^T X D^{-1/2} (D = diag(X^T X), non-empty
// columns) by power iteration from the unit vector with equal entries on the
// non-empty columns (section 4.1: Shotgun is safe up to k / (2 rho) columns
// per iteration).  FP64 throughout.  Per iteration:
//   s = X x,  x = D^{-1/2} v          (k_check_spmv<8, double>, into z64)
//   U = X^T s                          (k_check_cols<8>, into g64)
//   hist[t] = ||D^{-1/2} U||^2         (k_rho_norm)
//   x = D^{-1/2} (D^{-1/2} U / rho_t), U = 0, s = 0   (k_rho_scale)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_rho_init(int64_t k, int64_t n, double *ss_u,
                                                      double *dinv, double *x, double v0,
                                                      double *s64, double *hist, int iters) {
  const int64_t tid = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t nt = int64_t(gridDim.x) * kBlock;
  for (int64_t j = tid; j < k; j += nt) {
    const double q = ss_u[j];  // sum of squares of column j
    const double d = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    dinv[j] = d;
    x[j] = d * v0;
    ss_u[j] = 0.0;
  }
  for (int64_t i = tid; i < n; i += nt) s64[i] = 0.0;
  for (int64_t t = tid; t < iters; t += nt) hist[t] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_rho_norm(int64_t k, const double *dinv, const double *u,
                                                      double *hist_t) {
  __shared__ double sred[kBlock];
  double acc = 0.0;
  for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < k;
       j += int64_t(gridDim.x) * kBlock) {
    const double v = dinv[j] * u[j];
    acc += v * v;
  }
  sred[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sred[threadIdx.x] += sred[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(hist_t, sred[0]);
}

__global__ __launch_bounds__(kBlock) void k_rho_scale(int64_t k, int64_t n, const double *dinv,
                                                       double *u, double *x, double *s64,
                                                       const double *hist_t) {
  const double rho = sqrt(*hist_t);
  const int64_t tid = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t nt = int64_t(gridDim.x) * kBlock;
  for (int64_t j = tid; j < k; j += nt) {
    const double v = dinv[j] * u[j];
    x[j] = rho > 0.0 ? dinv[j] * (v / rho) : 0.0;
    u[j] = 0.0;
  }
  for (int64_t i = tid; i < n; i += nt) s64[i] = 0.0;
}

int launch_rho(const gencd_csc *X, int32_t n_short, int32_t n_lpieces, const Ws &ws, int64_t k_live,
               int iters, hipStream_t s) {
  if (!ws.rho_dinv || iters < 1 || iters > kRhoMaxIters || k_live <= 0) return GENCD_ERR_INVALID_ARG;
  const int64_t nk = X->n > X->k ? X->n : X->k;
  unsigned blocks;
  int32_t nl;
  two_class_grid(n_short, n_lpieces, 8, &blocks, &nl);
  hipLaunchKernelGGL(k_rho_init, dim3(grid_for(nk)), dim3(kBlock), 0, s, X->k, X->n, ws.g64,
                     ws.rho_dinv, ws.rho_x, 1.0 / sqrt(double(k_live)), ws.z64, ws.rho_hist, iters);
  for (int t = 0; t < iters; ++t) {
    if (n_short + n_lpieces > 0) {
      hipLaunchKernelGGL((k_check_spmv<8, double>), dim3(blocks), dim3(kBlock), 0, s, X->row_idx,
                         X->val, ws.desc_all_s, n_short, ws.desc_all_l, n_lpieces, nl, ws.rho_x,
                         ws.z64);
      hipLaunchKernelGGL(k_check_cols<8>, dim3(blocks), dim3(kBlock), 0, s, X->row_idx, X->val,
                         ws.desc_all_s, n_short, ws.desc_all_l, n_lpieces, nl, ws.z64, ws.g64);
    }
    hipLaunchKernelGGL(k_rho_norm, dim3(grid_for(X->k, 256)), dim3(kBlock), 0, s, X->k, ws.rho_dinv,
                       ws.g64, ws.rho_hist + t);
    hipLaunchKernelGGL(k_rho_scale, dim3(grid_for(nk)), dim3(kBlock), 0, s, X->k, X->n, ws.rho_dinv,
                       ws.g64, ws.rho_x, ws.z64, ws.rho_hist + t);
  }
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// ---------------------------------------------------------------------------
// Block Shotgun (section 7): preset random blocks, each with its own P_b*
// ---------------------------------------------------------------------------
// Preset order: base[q] = live column at position q of the seeded
// permutation; block of position q = the b with block_lo(b) <= q <
// block_lo(b + 1), i.e. floor(((q + 1) nb - 1) / k_live).
__global__ __launch_bounds__(kBlock) void k_block_base(const int32_t *live, int64_t k_live,
                                                        int64_t nb, PermKey pk, int32_t *base,
                                                        int32_t *bcol) {
  for (int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x; q < k_live;
       q += int64_t(gridDim.x) * kBlock) {
    const int32_t j = live[perm_apply(pk, uint64_t(q))];
    base[q] = j;
    bcol[j] = int32_t(((q + 1) * nb - 1) / k_live);
  }
}

// Per-block power iteration: the power iteration of launch_rho run on every
// block's normalised Gram matrix at once, with one product vector per block
// (bs[row][b]).  Columns are walked one wave each in preset order.
__global__ __launch_bounds__(kBlock) void k_brho_init(int64_t k, int64_t n, int64_t nb,
                                                       int64_t k_live, const int32_t *bcol,
                                                       double *ss_u, double *dinv, double *x,
                                                       double *bs, double *hist, int iters) {
  const int64_t tid = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t nt = int64_t(gridDim.x) * kBlock;
  for (int64_t j = tid; j < k; j += nt) {
    const int32_t b = bcol[j];
    const double q = ss_u[j];
    const double d = (b >= 0 && q > 0.0) ? 1.0 / sqrt(q) : 0.0;
    dinv[j] = d;
    if (b >= 0) {
      const int64_t kb = block_lo(b + 1, k_live, nb) - block_lo(b, k_live, nb);
      x[j] = d * (1.0 / sqrt(double(kb)));
    } else {
      x[j] = 0.0;
    }
    ss_u[j] = 0.0;
  }
  for (int64_t i = tid; i < n * nb; i += nt) bs[i] = 0.0;
  for (int64_t t = tid; t < int64_t(iters) * nb; t += nt) hist[t] = 0.0;
}

// ||D^{-1/2} U||^2 per block.  Each thread walks a contiguous run of preset
// positions (blocks are contiguous runs), flushing its sum at every block
// boundary.
constexpr int kBrhoRun = 64;
__global__ __launch_bounds__(kBlock) void k_brho_norm(const int32_t *base, int64_t k_live,
                                                       const int32_t *bcol, const double *dinv,
                                                       const double *u, double *hist_t) {
  const int64_t tid = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t nt = int64_t(gridDim.x) * kBlock;
  for (int64_t q0 = tid * kBrhoRun; q0 < k_live; q0 += nt * kBrhoRun) {
    const int64_t q1 = q0 + kBrhoRun < k_live ? q0 + kBrhoRun : k_live;
    int32_t cur = -1;
    double acc = 0.0;
    for (int64_t q = q0; q < q1; ++q) {
      const int32_t j = base[q];
      const int32_t b = bcol[j];
      if (b != cur) {
        if (cur >= 0) atomicAdd(&hist_t[cur], acc);
        cur = b;
        acc = 0.0;
      }
      const double v = dinv[j] * u[j];
      acc += v * v;
    }
    if (cur >= 0) atomicAdd(&hist_t[cur], acc);
  }
}

__global__ __launch_bounds__(kBlock) void k_brho_scale(int64_t k, int64_t n, int64_t nb,
                                                        const int32_t *bcol, const double *dinv,
                                                        double *u, double *x, double *bs,
                                                        const double *hist_t) {
  const int64_t tid = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t nt = int64_t(gridDim.x) * kBlock;
  for (int64_t j = tid; j < k; j += nt) {
    const int32_t b = bcol[j];
    if (b < 0) continue;
    const double rho = sqrt(hist_t[b]);
    const double v = dinv[j] * u[j];
    x[j] = rho > 0.0 ? dinv[j] * (v / rho) : 0.0;
    u[j] = 0.0;
  }
  for (int64_t i = tid; i < n * nb; i += nt) bs[i] = 0.0;
}

int launch_block_setup(const gencd_csc *X, int32_t n_short, int32_t n_lpieces, const Ws &ws,
                       int64_t k_live, uint64_t seed, int iters, hipStream_t s) {
  const int64_t nb = ws.nblocks;
  if (nb < 1 || nb > k_live || iters < 1 || iters > kBlockRhoMaxIters) return GENCD_ERR_INVALID_ARG;
  int st = fill_i32(ws.bcol, X->k, -1, s);
  if (st) return st;
  hipLaunchKernelGGL(k_block_base, dim3(grid_for(k_live)), dim3(kBlock), 0, s, ws.live, k_live, nb,
                     make_perm_key(k_live, block_seed(seed, -1), 0), ws.bbase, ws.bcol);
  const int64_t nk = X->n * nb > X->k ? X->n * nb : X->k;
  hipLaunchKernelGGL(k_brho_init, dim3(grid_for(nk)), dim3(kBlock), 0, s, X->k, X->n, nb, k_live,
                     ws.bcol, ws.g64, ws.rho_dinv, ws.rho_x, ws.bs, ws.bhist, iters);
  // the products by pieces, as in the check: a heavy column is spread over
  // many waves instead of walked by one
  unsigned blocks;
  int32_t nl;
  two_class_grid(n_short, n_lpieces, 8, &blocks, &nl);
  const unsigned rg = grid_for((k_live + kBrhoRun - 1) / kBrhoRun);
  for (int t = 0; t < iters; ++t) {
    double *ht = ws.bhist + int64_t(t) * nb;
    if (n_short + n_lpieces > 0) {
      hipLaunchKernelGGL((k_check_spmv<8, double>), dim3(blocks), dim3(kBlock), 0, s, X->row_idx,
                         X->val, ws.desc_all_s, n_short, ws.desc_all_l, n_lpieces, nl, ws.rho_x,
                         ws.bs, nb, ws.bcol);
      hipLaunchKernelGGL(k_check_cols<8>, dim3(blocks), dim3(kBlock), 0, s, X->row_idx, X->val,
                         ws.desc_all_s, n_short, ws.desc_all_l, n_lpieces, nl, ws.bs, ws.g64, nb,
                         ws.bcol);
    }
    hipLaunchKernelGGL(k_brho_norm, dim3(rg), dim3(kBlock), 0, s, ws.bbase, k_live, ws.bcol,
                       ws.rho_dinv, ws.g64, ht);
    hipLaunchKernelGGL(k_brho_scale, dim3(grid_for(nk)), dim3(kBlock), 0, s, X->k, X->n, nb,
                       ws.bcol, ws.rho_dinv, ws.g64, ws.rho_x, ws.bs, ht);
  }
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// Per-epoch order: blocks in a permuted order, each block's members in a
// per-epoch permuted order, windows of P_b* positions inside every block.
__global__ __launch_bounds__(kBlock) void k_block_sizes(int64_t nb, int64_t k_live, uint64_t seed,
                                                         const int64_t *epoch, const int32_t *bp,
                                                         int32_t *cnt, int32_t *wcnt) {
  const PermKey pk = make_perm_key(nb, seed, *epoch);
  for (int64_t u = int64_t(blockIdx.x) * kBlock + threadIdx.x; u < nb;
       u += int64_t(gridDim.x) * kBlock) {
    const int64_t b = int64_t(perm_apply(pk, uint64_t(u)));
    const int64_t kb = block_lo(b + 1, k_live, nb) - block_lo(b, k_live, nb);
    cnt[u] = int32_t(kb);
    wcnt[u] = int32_t((kb + bp[b] - 1) / bp[b]);
  }
}

__global__ __launch_bounds__(kBlock) void k_block_fill(int64_t nb, int64_t k_live, uint64_t seed,
                                                        const int64_t *epoch, const int32_t *bp,
                                                        const int32_t *base, const int32_t *bstart,
                                                        const int32_t *bwin, int32_t *col_of_pos,
                                                        int32_t *win_off) {
  const int64_t e = *epoch;
  const PermKey pk = make_perm_key(nb, seed, e);
  for (int64_t u = blockIdx.x; u < nb; u += gridDim.x) {
    const int64_t b = int64_t(perm_apply(pk, uint64_t(u)));
    const int64_t lo = block_lo(b, k_live, nb), kb = block_lo(b + 1, k_live, nb) - lo;
    const PermKey pkb = make_perm_key(kb, block_seed(seed, b), e);
    const int32_t o = bstart[u];
    for (int64_t i = threadIdx.x; i < kb; i += kBlock)
      col_of_pos[o + i] = base[lo + int64_t(perm_apply(pkb, uint64_t(i)))];
    const int32_t w0 = bwin[u], nw = bwin[u + 1] - w0;
    for (int32_t t = threadIdx.x; t < nw; t += kBlock) win_off[w0 + t] = o + t * bp[b];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) win_off[bwin[nb]] = int32_t(k_live);
}

int launch_block_order(const Ws &w, int64_t k_live, uint64_t seed, const int64_t *epoch, int64_t T,
                       hipStream_t s) {
  const int64_t nb = w.nblocks;
  hipLaunchKernelGGL(k_block_sizes, dim3(grid_for(nb)), dim3(kBlock), 0, s, nb, k_live, seed,
                     epoch, w.bp, w.tmp_cnt, w.tmp_cnt2);
  int st = scan_exclusive(w.tmp_cnt, w.bstart, nb, w.scan_part, s);
  if (st) return st;
  st = scan_exclusive(w.tmp_cnt2, w.bwin, nb, w.scan_part, s);
  if (st) return st;
  hipLaunchKernelGGL(k_block_fill, dim3(unsigned(nb < 8192 ? nb : 8192)), dim3(kBlock), 0, s, nb,
                     k_live, seed, epoch, w.bp, w.bbase, w.bstart, w.bwin, w.col_of_pos,
                     w.win_off);
  hipLaunchKernelGGL(k_list_counts, dim3(grid_for(k_live)), dim3(kBlock), 0, s, w.col_of_pos,
                     k_live, w.all_soff, w.all_loff, w.tmp_cnt, w.tmp_cnt2);
  return order_tail(w, k_live, w.win_off, 0, T, s);
}

// Copy z64 rounded to FP32 into a caller buffer.
__global__ __launch_bounds__(kBlock) void k_round_f32(const double *src, float *dst, int64_t m) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < m;
       i += int64_t(gridDim.x) * kBlock)
    dst[i] = float(src[i]);
}

int launch_round_f32(const double *src, float *dst, int64_t m, hipStream_t s) {
  if (m <= 0) return GENCD_OK;
  hipLaunchKernelGGL(k_round_f32, dim3(grid_for(m)), dim3(kBlock), 0, s, src, dst, m);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

}  // namespace gencd
