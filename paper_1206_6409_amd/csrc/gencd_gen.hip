// Synthetic serving requests generated on the device, so that a stream of
// large requests (hundreds of MB of CSC each) never passes through host
// memory.  The law is the one of the host generator of the test inputs:
// every entry of the n x k matrix is nonzero independently with probability
// `density`, nonzero values are N(0, 1), the ground truth w* has `support`
// N(0, 1) weights on non-empty columns, and the labels are y = Xw* + N(0,
// 0.01) (squared loss) or y = +1 with probability sigma((Xw*)_i), else -1
// (logistic loss).
//
// Random numbers: every draw is the SplitMix64 finaliser (Steele, Lea &
// Flood 2014) of a key and a counter, so each column's stream is
// independent of the launch shape and the result depends only on the seed.
// A column's rows are drawn by geometric skips (the gap to the next nonzero
// of a Bernoulli(density) sequence is floor(log U / log(1 - density))), in
// two passes with the same draws: counts, then rows and values.
#include <cmath>

#include "gencd_common.hpp"
#include "gencd_kernels.hpp"

namespace gencd {

__device__ __forceinline__ uint64_t gen_key(uint64_t seed, uint64_t stream, uint64_t j) {
  return splitmix_fin(seed ^ splitmix_fin(stream * 0x9E3779B97F4A7C15ull + splitmix_fin(j + 1)));
}

// Uniform in (0, 1): 53 random bits, offset by half an ulp.
__device__ __forceinline__ double gen_uniform(uint64_t key, uint64_t i) {
  const uint64_t x = splitmix_fin(key + (i + 1) * 0x9E3779B97F4A7C15ull);
  return (double(x >> 11) + 0.5) * 0x1.0p-53;
}

// N(0, 1) by Box-Muller from draws 2i and 2i + 1.
__device__ __forceinline__ double gen_normal(uint64_t key, uint64_t i) {
  const double u1 = gen_uniform(key, 2 * i), u2 = gen_uniform(key, 2 * i + 1);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Rows of column j: walk the geometric skips; FILL writes them and their values.
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_gen_cols(int64_t n, int64_t k, double log1md,
                                                     uint64_t seed, int32_t *cnt,
                                                     const int64_t *col_ptr, int32_t *row_idx,
                                                     float *val) {
  for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < k;
       j += int64_t(gridDim.x) * kBlock) {
    const uint64_t key = gen_key(seed, 1, uint64_t(j));
    const uint64_t vkey = gen_key(seed, 2, uint64_t(j));
    int64_t row = -1, m = 0;
    const int64_t base = FILL ? col_ptr[j] : 0;
    for (uint64_t i = 0;; ++i) {
      const double gap = floor(log(gen_uniform(key, i)) / log1md);
      if (!(gap < double(n))) break;  // also ends the walk on a huge gap
      row += int64_t(gap) + 1;
      if (row >= n) break;
      if (FILL) {
        row_idx[base + m] = int32_t(row);
        val[base + m] = float(gen_normal(vkey, uint64_t(m)));
      }
      ++m;
    }
    if (!FILL) cnt[j] = int32_t(m);
  }
}

__global__ __launch_bounds__(kBlock) void k_gen_widen(const int32_t *off, int64_t k, int64_t *col_ptr) {
  for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j <= k;
       j += int64_t(gridDim.x) * kBlock)
    col_ptr[j] = int64_t(off[j]);
}

// w* on `support` columns: draw m picks a uniform column and moves to the
// next non-empty one (cyclically); its weight is N(0, 1) and it adds
// w*_j X_j to z64.
__global__ __launch_bounds__(kBlock) void k_gen_truth(int64_t k, int32_t support, uint64_t seed,
                                                      const int64_t *col_ptr, const int32_t *row_idx,
                                                      const float *val, double *z64) {
  const uint64_t key = gen_key(seed, 3, 0);
  for (int32_t m = int32_t(blockIdx.x * kBlock + threadIdx.x); m < support;
       m += int32_t(gridDim.x * kBlock)) {
    int64_t j = int64_t(double(k) * gen_uniform(key, uint64_t(m)));
    if (j >= k) j = k - 1;
    for (int64_t step = 0; step < k && col_ptr[j + 1] == col_ptr[j]; ++step) j = (j + 1) % k;
    if (col_ptr[j + 1] == col_ptr[j]) continue;  // an empty matrix
    const double wj = gen_normal(gen_key(seed, 4, 0), uint64_t(m));
    for (int64_t e = col_ptr[j]; e < col_ptr[j + 1]; ++e)
      atomicAdd(&z64[row_idx[e]], wj * double(val[e]));
  }
}

__global__ __launch_bounds__(kBlock) void k_gen_labels(int64_t n, int32_t loss, uint64_t seed,
                                                       const double *z64, float *y) {
  const uint64_t key = gen_key(seed, 5, 0);
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock) {
    const double z = z64[i];
    if (loss == GENCD_SQUARED) {
      y[i] = float(z + 0.1 * gen_normal(key, uint64_t(i)));
    } else {
      const double p = 1.0 / (1.0 + exp(-z));
      y[i] = gen_uniform(key, 2 * uint64_t(i)) < p ? 1.0f : -1.0f;
    }
  }
}

static unsigned gen_grid(int64_t m, unsigned cap = 4096) {
  int64_t b = (m + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return unsigned(b);
}

static bool gen_args_ok(int64_t n, int64_t k, double density) {
  return n > 0 && k > 0 && n < INT32_MAX && k < INT32_MAX && density > 0.0 && density < 1.0;
}

}  // namespace gencd

using namespace gencd;

extern "C" {

int gencd_gen_workspace_bytes(int64_t n, int64_t k, size_t *out_bytes) {
  if (!out_bytes || n <= 0 || k <= 0) return GENCD_ERR_INVALID_ARG;
  const size_t cnt = sizeof(int32_t) * size_t(k + 1);
  const size_t off = sizeof(int32_t) * size_t(k + 1);
  const size_t part = sizeof(int32_t) * scan_partials_for(k + 1);
  const size_t z = sizeof(double) * size_t(n);
  *out_bytes = (cnt + 255) / 256 * 256 + (off + 255) / 256 * 256 + (part + 255) / 256 * 256 +
               (z + 255) / 256 * 256 + 256;
  return GENCD_OK;
}

int gencd_gen_count(int64_t n, int64_t k, double density, uint64_t seed, int64_t *col_ptr,
                    int64_t *nnz, void *ws, size_t ws_bytes, hipStream_t stream) {
  size_t need = 0;
  if (!gen_args_ok(n, k, density) || !col_ptr || !nnz) return GENCD_ERR_INVALID_ARG;
  if (gencd_gen_workspace_bytes(n, k, &need) || !ws || ws_bytes < need) return GENCD_ERR_WORKSPACE;
  (void)hipGetLastError();
  char *b = static_cast<char *>(ws);
  b += (256 - reinterpret_cast<uintptr_t>(b) % 256) % 256;
  int32_t *cnt = reinterpret_cast<int32_t *>(b);
  int32_t *off = cnt + (k + 1 + 63) / 64 * 64;
  int32_t *part = off + (k + 1 + 63) / 64 * 64;
  hipLaunchKernelGGL(k_gen_cols<false>, dim3(gen_grid(k)), dim3(kBlock), 0, stream, n, k,
                     std::log1p(-density), seed, cnt, nullptr, nullptr, nullptr);
  int st = scan_exclusive(cnt, off, k, part, stream);
  if (st) return st;
  hipLaunchKernelGGL(k_gen_widen, dim3(gen_grid(k + 1)), dim3(kBlock), 0, stream, off, k, col_ptr);
  GENCD_HIP(hipGetLastError());
  int64_t total = 0;
  GENCD_HIP(hipMemcpyAsync(&total, col_ptr + k, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
  GENCD_HIP(hipStreamSynchronize(stream));
  if (total < 0 || total >= INT32_MAX) return GENCD_ERR_UNSUPPORTED;
  *nnz = total;
  return GENCD_OK;
}

int gencd_gen_fill(int64_t n, int64_t k, double density, uint64_t seed, int32_t loss,
                   int32_t support, const int64_t *col_ptr, int32_t *row_idx, float *val, float *y,
                   void *ws, size_t ws_bytes, hipStream_t stream) {
  size_t need = 0;
  if (!gen_args_ok(n, k, density) || !col_ptr || !y || support < 0 ||
      (loss != GENCD_SQUARED && loss != GENCD_LOGISTIC))
    return GENCD_ERR_INVALID_ARG;
  if (gencd_gen_workspace_bytes(n, k, &need) || !ws || ws_bytes < need) return GENCD_ERR_WORKSPACE;
  (void)hipGetLastError();
  char *b = static_cast<char *>(ws);
  b += (256 - reinterpret_cast<uintptr_t>(b) % 256) % 256;
  size_t zoff = need - 256 - (sizeof(double) * size_t(n) + 255) / 256 * 256;
  double *z64 = reinterpret_cast<double *>(b + zoff);
  hipLaunchKernelGGL(k_gen_cols<true>, dim3(gen_grid(k)), dim3(kBlock), 0, stream, n, k,
                     std::log1p(-density), seed, nullptr, col_ptr, row_idx, val);
  int st = fill_f64(z64, n, 0.0, stream);
  if (st) return st;
  if (support > 0)
    hipLaunchKernelGGL(k_gen_truth, dim3(gen_grid(support, 64)), dim3(kBlock), 0, stream, k, support,
                       seed, col_ptr, row_idx, val, z64);
  hipLaunchKernelGGL(k_gen_labels, dim3(gen_grid(n)), dim3(kBlock), 0, stream, n, loss, seed, z64, y);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

}  // extern "C"
