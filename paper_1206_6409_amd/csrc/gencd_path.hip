// Batched regularisation path: many lambda values of Eq. (1) on one matrix.
//
// B "slots" (B in {16, 32, 64}) are solved together with a shared selected
// set J (Shotgun windows of the per-epoch permutation, section 2.1): a group
// of B lanes owns one column of J and lane s works for slot s, so every read
// of the slot-interleaved state W[k][B], Z[n][B] is one coalesced B-wide row
// and the CSC entries of X are read once for all slots.  Propose (Algorithm
// 4) and Update (Algorithm 3) are the single-problem ones applied per lane
// with the lane's own lambda; the FP64 check (objective, KKT, re-sync) runs
// per slot.  A slot whose KKT test passes is retired on the host and the
// next lambda (decreasing order) is admitted into it, warm-started from the
// latest iterate of its predecessor.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "gencd_common.hpp"
#include "gencd_kernels.hpp"

namespace gencd {

struct PathWs {
  float *W;              // [k][B]
  float *zh, *zl;        // [n][B]
  float *lam;            // [B] lambda of each slot for the FP32 Propose arithmetic
  double *lam64;         // [B] the same lambda in FP64 for the check
  int32_t *active;       // [B]
  float *delta;          // [S][B] deltas of the current window
  double *z64, *r64;     // [n][B]
  double *g64;           // [k][B]
  double *red;           // [B][8]: loss, l1, kkt bits, nnz, gmax bits, dual
  double *rep;           // [kRedRep][B][8]: the same, one partial per replica
};

// The check's per-slot reductions go to kRedRep replicas (workgroup b adds
// into replica b % kRedRep) and k_path_fold combines them: with one address
// per slot, every workgroup's FP64 atomic on it would be serialised.
constexpr int kRedRep = 64;

static size_t path_layout(int64_t n, int64_t k, int64_t S, int B, void *base, PathWs *o) {
  const size_t al = 256;
  size_t off = 0;
  char *b = static_cast<char *>(base);
  auto take = [&](size_t bytes) -> void * {
    off = (off + al - 1) / al * al;
    void *p = b ? b + off : nullptr;
    off += bytes > 0 ? bytes : 1;
    return p;
  };
  PathWs w{};
  w.W = static_cast<float *>(take(sizeof(float) * k * B));
  w.zh = static_cast<float *>(take(sizeof(float) * n * B));
  w.zl = static_cast<float *>(take(sizeof(float) * n * B));
  w.lam = static_cast<float *>(take(sizeof(float) * B));
  w.lam64 = static_cast<double *>(take(sizeof(double) * B));
  w.active = static_cast<int32_t *>(take(sizeof(int32_t) * B));
  w.delta = static_cast<float *>(take(sizeof(float) * S * B));
  w.z64 = static_cast<double *>(take(sizeof(double) * n * B));
  w.r64 = static_cast<double *>(take(sizeof(double) * n * B));
  w.g64 = static_cast<double *>(take(sizeof(double) * k * B));
  w.red = static_cast<double *>(take(sizeof(double) * 8 * B));
  w.rep = static_cast<double *>(take(sizeof(double) * 8 * B * kRedRep));
  if (o) *o = w;
  return off + al;
}

// ---------------------------------------------------------------------------
// Batched Propose / Update over one window of shared J
// ---------------------------------------------------------------------------
struct PathArgs {
  const int64_t *col_ptr;
  const int32_t *row_idx;
  const float *val;
  const float *y;
  const float *c;
  const int32_t *col_of_pos;
  const int4 *pdesc;  // per position of the epoch order: {first entry, column, length, 0}
  int32_t win_lo, win_hi;
  float n_f;
  int32_t loss;
  float *W, *zh, *zl;
  const float *lam;
  const int32_t *active;
  float *delta;
  int32_t improve;  // "improve delta_j" steps per column and slot (0: off)
};

// One 256-thread block per column of the window: thread (r, s) = (row lane,
// slot), s = threadIdx % B, r = threadIdx / B, R = 256 / B row lanes.  Row
// lane r takes the column entries r, r + R, ...; for each it reads the
// B-wide row Z[row][0..B) (one coalesced segment per row lane) and the
// entry itself (the same address for all B slot lanes).  Loads are issued in
// batches of R * PU entries so that a short column costs one round of
// dependent loads.  Partial sums are reduced across row lanes in a fixed
// order (shuffles inside a wave, then LDS across the waves), so the result
// does not depend on scheduling.
template <int B>
struct PathShape {
  static constexpr int R = kBlock / B;   // row lanes per column
  static constexpr int PU = 32 / R > 1 ? 32 / R : 2;  // entries per row lane per batch
  static constexpr int NW = kBlock / kWave;
};

// "Improve delta_j" (Algorithm 3, section 4.1) for every slot of one
// column: up to a.improve further Eq. 7 steps on the slot's 1-D objective
//   f_s(d) = (1/n) sum_i l(y_i, Z[i][s] + d x_ij) + lambda_s |W[j][s] + d|
// from the increment in sdel[s] and the z of the first step.  This form
// serves columns longer than one batch: the whole workgroup takes each step
// with the first step's thread shape and arithmetic, re-reading the entries,
// z and y (in the fused launch other columns may have moved z meanwhile).
// A slot whose step no longer changes d keeps it (every later step would
// repeat it), and the loop ends once no slot changed.  Slot lanes hold the
// slot's w_j, c_j, lambda; the improved increments are left in sdel.
template <int B, int R, int PU, int NW>
__device__ __forceinline__ void path_improve(const PathArgs &a, int64_t cb, int64_t ce, int s,
                                             int r, float wj, float cj, float lam,
                                             float (&sred)[NW][B], float *sdel) {
  for (int32_t t = 0; t < a.improve; ++t) {
    const float d = sdel[s];
    float acc = 0.0f;
    if (d != 0.0f) {
      for (int64_t base = cb; base < ce; base += int64_t(R) * PU) {
        int32_t rj[PU];
        float vj[PU], zj[PU], yj[PU];
#pragma unroll
        for (int q = 0; q < PU; ++q) {
          const int64_t e = base + int64_t(q) * R + r;
          rj[q] = e < ce ? a.row_idx[e] : -1;
          vj[q] = e < ce ? a.val[e] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < PU; ++q) {
          const int64_t i = rj[q] >= 0 ? rj[q] : 0;
          zj[q] = a.zh[i * B + s] + a.zl[i * B + s];
          yj[q] = a.y[i];
        }
#pragma unroll
        for (int q = 0; q < PU; ++q)
          if (rj[q] >= 0) acc += vj[q] * dloss_f32(a.loss, yj[q], zj[q] + d * vj[q]);
      }
    }
#pragma unroll
    for (int off = B; off < kWave; off <<= 1) acc += __shfl_xor(acc, off);
    if (int(threadIdx.x) % kWave < B) sred[threadIdx.x / kWave][s] = acc;
    __syncthreads();
    int changed = 0;
    if (int(threadIdx.x) < B && d != 0.0f) {
      float g = 0.0f;
#pragma unroll
      for (int w = 0; w < NW; ++w) g += sred[w][s];
      g /= a.n_f;
      float inc, ph;
      propose_f32(g, cj, wj + d, lam, inc, ph);
      const float dn = d + inc;
      if (dn != d) {
        sdel[s] = dn;
        changed = 1;
      }
    }
    // every read of sdel and sred of this step precedes the barrier
    if (!__syncthreads_or(changed)) break;
  }
}

// l'(y, t) for the improve steps of a column held in one batch: the two
// signs of m = y t are selected instead of branched on (lanes of one wave
// see both), m >= 0: e = exp(-m), s = e / (1 + e); m < 0: e = exp(m),
// s = 1 / (1 + e), with the hardware exponential and reciprocal (about one
// ulp each) in place of the correctly rounded forms.  The steps are
// VALU-bound, and they only refine an increment whose effect the FP64 check
// judges.
__device__ __forceinline__ float dloss_fast_f32(int loss, float y, float t) {
  if (loss == GENCD_SQUARED) return t - y;
  const float m = y * t;
  const float e = __expf(-fabsf(m));
  return -y * ((m >= 0.0f ? e : 1.0f) * __builtin_amdgcn_rcpf(1.0f + e));
}

// Sum over an aligned group of N = 4, 8 or 16 lanes with DPP moves inside
// a row (xor 1, xor 2, half-row mirror, row mirror): every stage adds the
// partner's partial to the lane's own, and the partner adds the same two
// values, so every lane of the group ends with the same bits.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int N>
__device__ __forceinline__ float row_group_sum(float x) {
  static_assert(N == 4 || N == 8 || N == 16, "groups inside one DPP row");
  x += dpp_move<0xB1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_move<0x4E>(x);   // quad_perm [2, 3, 0, 1]
  if constexpr (N >= 8) x += dpp_move<0x141>(x);   // row_half_mirror
  if constexpr (N >= 16) x += dpp_move<0x140>(x);  // row_mirror
  return x;
}

// One column of at most 64 entries (two batches) in LDS for
// path_improve_wave; the first step's batch loop stages it.
constexpr int kImproveMax = 64;

template <int B>
struct ImproveLds {
  float z[kImproveMax][B + 1];  // padded: lanes of one slot read a column of this
  float v[kImproveMax], y[kImproveMax];
  float w[B], lam[B];
  float c;
};

// Stage one batch of the first step (thread (r, s) holds entries
// boff + q R + r of the column) for the improve steps; padding gets v = 0,
// z = 0, y = 1, so that it adds 0 * l'(1, 0).
template <int B, int R, int PU>
__device__ __forceinline__ void improve_stage(ImproveLds<B> &L, int boff, int s, int r,
                                              const int32_t (&ri)[PU], const float (&vv)[PU],
                                              const float (&zb)[PU], const float (&yb)[PU]) {
#pragma unroll
  for (int q = 0; q < PU; ++q) {
    const int e = boff + q * R + r;
    const bool ok = ri[q] >= 0;
    L.z[e][s] = ok ? zb[q] : 0.0f;
    if (s == 0) {
      L.v[e] = ok ? vv[q] : 0.0f;
      L.y[e] = ok ? yb[q] : 1.0f;
    }
  }
}

// The same steps for a column of at most NQ * R entries (one or two
// batches, staged in LDS by the first step), without workgroup barriers
// between steps: wave v takes the slots [v B/4, (v+1) B/4), R lanes per slot
// and NQ entries per lane (the first step's thread shape with slots and row
// lanes swapped), sums over its R lanes with DPP moves (every lane gets the
// same bits) and repeats until none of its slots changed or the steps run
// out.  The loss derivative takes the fast forms above, and 1/n and 1/c
// are formed once.
template <int B, int R, int NQ>
__device__ __forceinline__ void path_improve_wave(const PathArgs &a, int s, float wj, float cj,
                                                  float lam, float *sdel, ImproveLds<B> &L) {
  static_assert(NQ * R <= kImproveMax, "the column fits the staging");
  constexpr int SPW = B / (kBlock / kWave);  // slots per wave
  static_assert(SPW * R == kWave, "a wave holds SPW slots of R lanes");
  if (int(threadIdx.x) < B) {
    L.w[s] = wj;
    L.lam[s] = lam;
    if (s == 0) L.c = cj;
  }
  __syncthreads();  // the staged column and the slots' scalars are in LDS
  const int lane = int(threadIdx.x) % kWave;
  const int sl = lane / R, rl = lane % R;
  const int s2 = int(threadIdx.x) / kWave * SPW + sl;
  float v[NQ], z[NQ], y[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = q * R + rl;
    v[q] = L.v[e];
    z[q] = L.z[e][s2];
    y[q] = L.y[e];
  }
  const float w2 = L.w[s2], lam2 = L.lam[s2], c2 = L.c;
  // Eq. 7 at w + d: d <- d - clamp(w + d, (g - lambda) / c, (g + lambda) / c),
  // with 1/n and 1/c formed once
  const float rn = 1.0f / a.n_f, rc = c2 > 0.0f ? 1.0f / c2 : 0.0f;
  float d = c2 > 0.0f ? sdel[s2] : 0.0f;
  for (int32_t t = 0; t < a.improve; ++t) {
    float acc = 0.0f;
    if (d != 0.0f) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc += v[q] * dloss_fast_f32(a.loss, y[q], z[q] + d * v[q]);
    }
    acc = row_group_sum<R>(acc);
    int changed = 0;
    if (d != 0.0f) {
      const float g = acc * rn;
      const float lo = (g - lam2) * rc, hi = (g + lam2) * rc, wd = w2 + d;
      const float dn = d - (wd < lo ? lo : (wd > hi ? hi : wd));
      changed = dn != d;
      d = dn;
    }
    if (!__any(changed)) break;  // every slot of the wave keeps its increment
  }
  __syncthreads();  // every lane has read sdel before it is rewritten
  if (rl == 0) sdel[s2] = d;
  __syncthreads();
}

// The improve steps of one column, by its length: staged columns of one or
// two batches in waves, longer ones as a workgroup.
template <int B, int R, int PU, int NW>
__device__ __forceinline__ void improve_column(const PathArgs &a, int64_t cb, int64_t ce, int s,
                                               int r, float wj, float cj, float lam,
                                               float (&sred)[NW][B], float *sdel,
                                               ImproveLds<B> &L) {
  const int64_t len = ce - cb;
  if (len <= int64_t(R) * PU)
    path_improve_wave<B, R, PU>(a, s, wj, cj, lam, sdel, L);
  else if (len <= int64_t(kImproveMax))
    path_improve_wave<B, R, kImproveMax / R>(a, s, wj, cj, lam, sdel, L);
  else
    path_improve<B, R, PU, NW>(a, cb, ce, s, r, wj, cj, lam, sred, sdel);
}

template <int B, bool IMP>
__global__ __launch_bounds__(kBlock) void k_path_propose(PathArgs a) {
  using SH = PathShape<B>;
  constexpr int R = SH::R, PU = SH::PU, NW = SH::NW;
  __shared__ float sred[NW][B];
  __shared__ float sdel[B];
  __shared__ std::conditional_t<IMP, ImproveLds<B>, char> simp;
  const int s = int(threadIdx.x) % B, r = int(threadIdx.x) / B;
  const int64_t npos = a.win_hi - a.win_lo;
  for (int64_t p = blockIdx.x; p < npos; p += gridDim.x) {
    const int4 pd = a.pdesc[a.win_lo + p];
    const int32_t j = pd.y;
    const int64_t cb = int64_t(uint32_t(pd.x)), ce = cb + pd.z;
    // the slot's weight, curvature, lambda and activity: issued with the
    // entries' loads, consumed after the reduction
    float wj = 0.0f, cj = 0.0f, lam = 0.0f;
    int32_t act = 0;
    if (int(threadIdx.x) < B) {
      wj = a.W[int64_t(j) * B + s];
      cj = a.c[j];
      lam = a.lam[s];
      act = a.active[s];
    }
    float acc = 0.0f;
    int32_t ri[PU];
    float vv[PU], zb[PU], yb[PU];  // the last batch (the whole column if it fits one)
#pragma unroll
    for (int q = 0; q < PU; ++q) {
      ri[q] = -1;
      vv[q] = zb[q] = yb[q] = 0.0f;
    }
    for (int64_t base = cb; base < ce; base += int64_t(R) * PU) {
#pragma unroll
      for (int q = 0; q < PU; ++q) {
        const int64_t e = base + int64_t(q) * R + r;
        ri[q] = e < ce ? a.row_idx[e] : -1;
        vv[q] = e < ce ? a.val[e] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < PU; ++q) {
        const int64_t i = ri[q] >= 0 ? ri[q] : 0;  // row 0 stands in for padding
        zb[q] = a.zh[i * B + s] + a.zl[i * B + s];
        yb[q] = a.y[i];
      }
#pragma unroll
      for (int q = 0; q < PU; ++q)
        if (ri[q] >= 0) acc += vv[q] * dloss_f32(a.loss, yb[q], zb[q]);
      if constexpr (IMP)
        if (ce - cb <= int64_t(kImproveMax))
          improve_stage<B, R, PU>(simp, int(base - cb), s, r, ri, vv, zb, yb);
    }
#pragma unroll
    for (int off = B; off < kWave; off <<= 1) acc += __shfl_xor(acc, off);
    if (int(threadIdx.x) % kWave < B) sred[threadIdx.x / kWave][s] = acc;
    __syncthreads();
    if (int(threadIdx.x) < B) {
      float g = 0.0f;
#pragma unroll
      for (int w = 0; w < NW; ++w) g += sred[w][s];
      float d = 0.0f;
      if (act != 0) {
        g /= a.n_f;
        float ph;
        propose_f32(g, cj, wj, lam, d, ph);
      }
      sdel[s] = d;
    }
    __syncthreads();
    if constexpr (IMP)  // uniform: the whole workgroup takes the steps
      improve_column<B, R, PU, NW>(a, cb, ce, s, r, wj, cj, lam, sred, sdel, simp);
    if (int(threadIdx.x) < B) {
      const float d = sdel[s];
      if (d != 0.0f) a.W[int64_t(j) * B + s] = wj + d;
      a.delta[p * B + s] = d;
    }
    __syncthreads();  // sred and sdel are reused by the next column
  }
}

// Same thread shape: row lane r scatters delta_s * x_ij of its entries into
// the low words Z_lo[row][s] (non-returning float atomics; the high words
// absorb them at the end of the epoch).
template <int B>
__global__ __launch_bounds__(kBlock) void k_path_update(PathArgs a) {
  using SH = PathShape<B>;
  constexpr int R = SH::R, PU = SH::PU;
  const int s = int(threadIdx.x) % B, r = int(threadIdx.x) / B;
  const int64_t npos = a.win_hi - a.win_lo;
  for (int64_t p = blockIdx.x; p < npos; p += gridDim.x) {
    const float d = a.delta[p * B + s];
    const int4 pd = a.pdesc[a.win_lo + p];
    const int64_t cb = int64_t(uint32_t(pd.x)), ce = cb + pd.z;
    for (int64_t base = cb; base < ce; base += int64_t(R) * PU) {
      int32_t ri[PU];
      float vv[PU];
#pragma unroll
      for (int q = 0; q < PU; ++q) {
        const int64_t e = base + int64_t(q) * R + r;
        ri[q] = e < ce ? a.row_idx[e] : -1;
        vv[q] = e < ce ? a.val[e] : 0.0f;
      }
      if (d != 0.0f) {
#pragma unroll
        for (int q = 0; q < PU; ++q)
          if (ri[q] >= 0) atomicAdd(&a.zl[int64_t(ri[q]) * B + s], d * vv[q]);
      }
    }
  }
}

// Fused asynchronous form (GENCD_FUSED): the same thread shape as
// k_path_propose; after the slot's step the workgroup scatters delta_s x_ij
// from the entries it still holds in registers, so Propose and Update of a
// window are one launch.  Columns of a window read Z while others update it.
// A workgroup that takes several positions (grid stride; all of them with
// GENCD_FUSED_EPOCH) loads the next position's descriptor, first batch of
// entries, weight, curvature, lambda and activity while it works on the
// current one: the matrix, the order, c, lambda and activity do not change
// during the launch, and column j's weights are written only by the
// workgroup that holds position of j in this epoch.
template <int B, int PU, int R>
__device__ __forceinline__ void path_batch(const PathArgs &a, int64_t base, int64_t ce, int r,
                                           int32_t (&ri)[PU], float (&vv)[PU]) {
#pragma unroll
  for (int q = 0; q < PU; ++q) {
    const int64_t e = base + int64_t(q) * R + r;
    ri[q] = e < ce ? a.row_idx[e] : -1;
    vv[q] = e < ce ? a.val[e] : 0.0f;
  }
}

template <int B, bool IMP>
__global__ __launch_bounds__(kBlock) void k_path_fused(PathArgs a) {
  using SH = PathShape<B>;
  constexpr int R = SH::R, PU = SH::PU, NW = SH::NW;
  __shared__ float sred[NW][B];
  __shared__ float sdel[B];
  __shared__ std::conditional_t<IMP, ImproveLds<B>, char> simp;
  const int s = int(threadIdx.x) % B, r = int(threadIdx.x) / B;
  const bool slot_lane = int(threadIdx.x) < B;
  const int64_t npos = a.win_hi - a.win_lo;
  int64_t p = blockIdx.x;
  if (p >= npos) return;  // uniform over the workgroup
  // the current position's descriptor, first batch and per-slot scalars
  int4 pd = a.pdesc[a.win_lo + p];
  int32_t ri[PU];
  float vv[PU];
  path_batch<B, PU, R>(a, int64_t(uint32_t(pd.x)), int64_t(uint32_t(pd.x)) + pd.z, r, ri, vv);
  float wj = 0.0f, cj = 0.0f, lam = 0.0f;
  int32_t act = 0;
  if (slot_lane) {
    wj = a.W[int64_t(pd.y) * B + s];
    cj = a.c[pd.y];
    lam = a.lam[s];
    act = a.active[s];
  }
  for (; p < npos; p += gridDim.x) {
    const int32_t j = pd.y;
    const int64_t cb = int64_t(uint32_t(pd.x)), ce = cb + pd.z;
    const bool one = ce - cb <= int64_t(R) * PU;  // the whole column in one batch
    const int64_t pn = p + gridDim.x;
    const bool more = pn < npos;
    const int4 pdn = more ? a.pdesc[a.win_lo + pn] : make_int4(0, 0, 0, 0);
    float acc = 0.0f;
    float zb[PU], yb[PU];
    for (int64_t base = cb; base < ce; base += int64_t(R) * PU) {
      if (base != cb) path_batch<B, PU, R>(a, base, ce, r, ri, vv);
      float zh[PU], zl[PU];
#pragma unroll
      for (int q = 0; q < PU; ++q) {
        const int64_t i = ri[q] >= 0 ? ri[q] : 0;
        zh[q] = a.zh[i * B + s];
        zl[q] = a.zl[i * B + s];
        yb[q] = a.y[i];
      }
#pragma unroll
      for (int q = 0; q < PU; ++q) {
        zb[q] = zh[q] + zl[q];
        if (ri[q] >= 0) acc += vv[q] * dloss_f32(a.loss, yb[q], zb[q]);
      }
      if constexpr (IMP)
        if (ce - cb <= int64_t(kImproveMax))
          improve_stage<B, R, PU>(simp, int(base - cb), s, r, ri, vv, zb, yb);
    }
#pragma unroll
    for (int off = B; off < kWave; off <<= 1) acc += __shfl_xor(acc, off);
    if (int(threadIdx.x) % kWave < B) sred[threadIdx.x / kWave][s] = acc;
    __syncthreads();
    if (slot_lane) {
      float g = 0.0f;
#pragma unroll
      for (int w = 0; w < NW; ++w) g += sred[w][s];
      float d = 0.0f;
      if (act != 0) {
        g /= a.n_f;
        float ph;
        propose_f32(g, cj, wj, lam, d, ph);
      }
      sdel[s] = d;
    }
    __syncthreads();
    if constexpr (IMP)  // uniform: the whole workgroup takes the steps
      improve_column<B, R, PU, NW>(a, cb, ce, s, r, wj, cj, lam, sred, sdel, simp);
    const float d = sdel[s];
    if (slot_lane && d != 0.0f) a.W[int64_t(j) * B + s] = wj + d;
    // the next position's loads go out before this column's atomics
    int32_t rn[PU];
    float vn[PU];
    float wn = 0.0f, cn = 0.0f;
    if (more) {
      path_batch<B, PU, R>(a, int64_t(uint32_t(pdn.x)), int64_t(uint32_t(pdn.x)) + pdn.z, r, rn, vn);
      if (slot_lane) {
        wn = a.W[int64_t(pdn.y) * B + s];
        cn = a.c[pdn.y];
      }
    }
    if (d != 0.0f) {
      if (one) {
#pragma unroll
        for (int q = 0; q < PU; ++q)
          if (ri[q] >= 0) atomicAdd(&a.zl[int64_t(ri[q]) * B + s], d * vv[q]);
      } else {
        for (int64_t e = cb + r; e < ce; e += R)
          atomicAdd(&a.zl[int64_t(a.row_idx[e]) * B + s], d * a.val[e]);
      }
    }
    __syncthreads();  // sred / sdel are reused by the next column
    pd = pdn;
#pragma unroll
    for (int q = 0; q < PU; ++q) {
      ri[q] = rn[q];
      vv[q] = vn[q];
    }
    wj = wn;
    cj = cn;
  }
}

// Staged form (used at B = 64): one group of B lanes per column, GPB = 256 / B columns per block;
// the group stages B entries at a time in LDS and issues one B-wide atomic
// row per entry.
template <int B>
__global__ __launch_bounds__(kBlock) void k_path_update_staged(PathArgs a) {
  constexpr int GPB = kBlock / B;
  __shared__ int32_t srow[GPB][B];
  __shared__ float sval[GPB][B];
  const int grp = int(threadIdx.x) / B, s = int(threadIdx.x) % B;
  const int64_t npos = a.win_hi - a.win_lo;
  for (int64_t p0 = int64_t(blockIdx.x) * GPB; p0 < npos; p0 += int64_t(gridDim.x) * GPB) {
    const int64_t p = p0 + grp;
    int64_t cb = 0, ce = 0;
    float d = 0.0f;
    if (p < npos) {
      const int4 pd = a.pdesc[a.win_lo + p];
      cb = int64_t(uint32_t(pd.x));
      ce = cb + pd.z;
      d = a.delta[p * B + s];
    }
    for (int64_t base = cb; base < ce; base += B) {
      const int64_t e = base + s;
      srow[grp][s] = e < ce ? a.row_idx[e] : -1;
      sval[grp][s] = e < ce ? a.val[e] : 0.0f;
      __builtin_amdgcn_wave_barrier();
      const int cnt = int(ce - base < B ? ce - base : B);
      if (d != 0.0f)
        for (int u = 0; u < cnt; ++u)
          atomicAdd(&a.zl[int64_t(srow[grp][u]) * B + s], d * sval[grp][u]);
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// Position descriptors of the epoch order.
__global__ __launch_bounds__(kBlock) void k_path_desc(int64_t m, const int32_t *col_of_pos,
                                                       const int64_t *col_ptr, int4 *pdesc) {
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < m;
       p += int64_t(gridDim.x) * kBlock) {
    const int32_t j = col_of_pos[p];
    const int64_t b = col_ptr[j];
    pdesc[p] = make_int4(int32_t(uint32_t(b)), j, int32_t(col_ptr[j + 1] - b), 0);
  }
}

// ---------------------------------------------------------------------------
// Batched FP64 check (per slot): z64 = X W, loss, r64, g64, KKT, |w|_1, dual
// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(kBlock) void k_path_zero(double *z64, int64_t n, double *g64, int64_t k,
                                                      double *red) {
  const int64_t tid = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t nt = int64_t(gridDim.x) * kBlock;
  for (int64_t i = tid; i < n * B; i += nt) z64[i] = 0.0;
  for (int64_t j = tid; j < k * B; j += nt) g64[j] = 0.0;
  if (tid < 8 * B * kRedRep) red[tid] = 0.0;
}

// rows or columns per lane taken together by the streaming check kernels
constexpr int kChkU = 4;

// one group of B lanes per column: z64[i][s] += W[j][s] * x_ij.  Entries
// are read kSpmvU at a time, so a column costs one load round per kSpmvU
// entries instead of one per entry.
constexpr int kSpmvU = 8;
template <int B>
__global__ __launch_bounds__(kBlock) void k_path_spmv(const int64_t *col_ptr, const int32_t *row_idx,
                                                      const float *val, int64_t k, const float *W,
                                                      double *z64) {
  constexpr int GPB = kBlock / B;
  const int grp = threadIdx.x / B, s = threadIdx.x % B;
  for (int64_t j = int64_t(blockIdx.x) * GPB + grp; j < k; j += int64_t(gridDim.x) * GPB) {
    const int64_t e0 = col_ptr[j], e1 = col_ptr[j + 1];
    const double wj = double(W[j * B + s]);
    if (wj == 0.0) continue;
    for (int64_t e = e0; e < e1; e += kSpmvU) {
      int32_t ri[kSpmvU];
      float v[kSpmvU];
#pragma unroll
      for (int q = 0; q < kSpmvU; ++q) {
        ri[q] = e + q < e1 ? row_idx[e + q] : -1;
        v[q] = e + q < e1 ? val[e + q] : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < kSpmvU; ++q)
        if (ri[q] >= 0) atomicAdd(&z64[int64_t(ri[q]) * B + s], wj * double(v[q]));
    }
  }
}

template <int B>
__global__ __launch_bounds__(kBlock) void k_path_rows(int64_t n, int loss, const float *y,
                                                      const double *z64, double *r64, float *zh,
                                                      float *zl, double *red) {
  constexpr int GPB = kBlock / B;
  __shared__ double sacc[kBlock];
  const int grp = threadIdx.x / B, s = threadIdx.x % B;
  const int64_t stride = int64_t(gridDim.x) * GPB;
  double acc = 0.0;
  for (int64_t i0 = int64_t(blockIdx.x) * GPB + grp; i0 < n; i0 += kChkU * stride) {
    double zt[kChkU], yv[kChkU];
#pragma unroll
    for (int u = 0; u < kChkU; ++u) {  // all loads of the batch before any store
      const int64_t i = i0 + u * stride;
      zt[u] = i < n ? z64[i * B + s] : 0.0;
      yv[u] = i < n ? double(y[i]) : 1.0;
    }
#pragma unroll
    for (int u = 0; u < kChkU; ++u) {
      const int64_t i = i0 + u * stride;
      if (i >= n) break;
      const double t = zt[u];
      acc += loss_f64(loss, yv[u], t);
      r64[i * B + s] = dloss_f64(loss, yv[u], t);
      const float h = float(t);
      zh[i * B + s] = h;
      zl[i * B + s] = float(t - double(h));
    }
  }
  sacc[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < B) {
    double t = 0.0;
    for (int g = 0; g < GPB; ++g) t += sacc[g * B + threadIdx.x];
    atomicAdd(&red[(blockIdx.x % kRedRep) * 8 * B + threadIdx.x * 8 + 0], t);
  }
}

template <int B>
__global__ __launch_bounds__(kBlock) void k_path_cols(const int64_t *col_ptr, const int32_t *row_idx,
                                                      const float *val, int64_t k,
                                                      const double *r64, double *g64) {
  constexpr int GPB = kBlock / B;
  const int grp = threadIdx.x / B, s = threadIdx.x % B;
  for (int64_t j = int64_t(blockIdx.x) * GPB + grp; j < k; j += int64_t(gridDim.x) * GPB) {
    double acc = 0.0;
    int64_t e = col_ptr[j];
    const int64_t ce = col_ptr[j + 1];
    for (; e + kUnroll <= ce; e += kUnroll) {
      double r[kUnroll];
      float v[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        v[q] = val[e + q];
        r[q] = r64[int64_t(row_idx[e + q]) * B + s];
      }
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) acc += double(v[q]) * r[q];
    }
    for (; e < ce; ++e) acc += double(val[e]) * r64[int64_t(row_idx[e]) * B + s];
    g64[j * B + s] = acc;
  }
}

template <int B>
__global__ __launch_bounds__(kBlock) void k_path_kkt(int64_t k, double *g64, const float *W,
                                                     const double *lam, double inv_n, double *red) {
  constexpr int GPB = kBlock / B;
  __shared__ double smax[kBlock], sl1[kBlock], sgm[kBlock], snz[kBlock];
  const int grp = threadIdx.x / B, s = threadIdx.x % B;
  const double l = lam[s];
  const int64_t stride = int64_t(gridDim.x) * GPB;
  double vmax = 0.0, l1 = 0.0, gmax = 0.0, nz = 0.0;
  for (int64_t j0 = int64_t(blockIdx.x) * GPB + grp; j0 < k; j0 += kChkU * stride) {
    double gv[kChkU];
    float wv[kChkU];
#pragma unroll
    for (int u = 0; u < kChkU; ++u) {
      const int64_t j = j0 + u * stride;
      gv[u] = j < k ? g64[j * B + s] : 0.0;
      wv[u] = j < k ? W[j * B + s] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kChkU; ++u) {
      const int64_t j = j0 + u * stride;
      if (j >= k) break;
      const double g = gv[u] * inv_n;
      g64[j * B + s] = g;
      if (!(fabs(g) <= gmax)) gmax = fabs(g);
      const double wj = double(wv[u]);
      double v;
      if (wj != 0.0) {
        v = fabs(g + (wj > 0.0 ? l : -l));
        l1 += fabs(wj);
        nz += 1.0;
      } else {
        v = fabs(g) - l;
        if (v < 0.0) v = 0.0;
      }
      if (!(v <= vmax)) vmax = v;
    }
  }
  smax[threadIdx.x] = vmax;
  sl1[threadIdx.x] = l1;
  sgm[threadIdx.x] = gmax;
  snz[threadIdx.x] = nz;
  __syncthreads();
  if (threadIdx.x < B) {
    double m = 0.0, a1 = 0.0, gm = 0.0, z = 0.0;
    for (int g = 0; g < GPB; ++g) {
      const int t = g * B + threadIdx.x;
      if (!(smax[t] <= m)) m = smax[t];
      if (!(sgm[t] <= gm)) gm = sgm[t];
      a1 += sl1[t];
      z += snz[t];
    }
    double *rr = red + (blockIdx.x % kRedRep) * 8 * B + threadIdx.x * 8;
    unsigned long long *rb = reinterpret_cast<unsigned long long *>(rr);
    atomicMax(rb + 2, (m != m) ? 0x7FF8000000000000ull : (unsigned long long)__double_as_longlong(m));
    atomicMax(rb + 4, (gm != gm) ? 0x7FF8000000000000ull : (unsigned long long)__double_as_longlong(gm));
    atomicAdd(rr + 1, a1);
    atomicAdd(rr + 3, z);
  }
}

template <int B>
__global__ __launch_bounds__(kBlock) void k_path_dual(int64_t n, int loss, const float *y,
                                                      const double *r64, const double *lam,
                                                      const double *fold, double *red) {
  constexpr int GPB = kBlock / B;
  __shared__ double sacc[kBlock];
  const int grp = threadIdx.x / B, s = threadIdx.x % B;
  const double l = lam[s];
  // max |g| of the slot, folded from k_path_kkt's replicas into fold[s][4]
  const double gm = fold[s * 8 + 4];
  const double sc = (gm > l) ? l / gm : 1.0;
  const int64_t stride = int64_t(gridDim.x) * GPB;
  double acc = 0.0;
  for (int64_t i0 = int64_t(blockIdx.x) * GPB + grp; i0 < n; i0 += kChkU * stride) {
    double rv[kChkU], yv[kChkU];
#pragma unroll
    for (int u = 0; u < kChkU; ++u) {
      const int64_t i = i0 + u * stride;
      rv[u] = i < n ? r64[i * B + s] : 0.0;
      yv[u] = i < n ? double(y[i]) : 1.0;
    }
#pragma unroll
    for (int u = 0; u < kChkU; ++u) {
      if (i0 + u * stride >= n) break;
      const double v = sc * rv[u];
      const double yi = yv[u];
      if (loss == GENCD_SQUARED) {
        acc -= v * yi + 0.5 * v * v;
      } else {
        const double pp = -v * yi;
        double h = 0.0;
        if (pp > 0.0) h -= pp * log(pp);
        if (pp < 1.0) h -= (1.0 - pp) * log1p(-pp);
        acc += h;
      }
    }
  }
  sacc[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < B) {
    double t = 0.0;
    for (int g = 0; g < GPB; ++g) t += sacc[g * B + threadIdx.x];
    atomicAdd(&red[(blockIdx.x % kRedRep) * 8 * B + threadIdx.x * 8 + 5], t);
  }
}

// Combine the kRedRep replicas into red[B][8]: maxima (entries 2 and 4, as
// bit patterns of non-negative doubles, NaN above all) and sums.
template <int B>
__global__ __launch_bounds__(8 * B) void k_path_fold(const double *rep, double *red) {
  const int tid = int(threadIdx.x);
  const int q = tid % 8;
  if (q == 2 || q == 4) {
    unsigned long long m = 0;
#pragma unroll 16
    for (int r = 0; r < kRedRep; ++r) {
      const unsigned long long b = reinterpret_cast<const unsigned long long *>(rep)[r * 8 * B + tid];
      m = b > m ? b : m;
    }
    red[tid] = __longlong_as_double((long long)m);
  } else {
    double t = 0.0;
#pragma unroll 16
    for (int r = 0; r < kRedRep; ++r) t += rep[r * 8 * B + tid];
    red[tid] = t;
  }
}

template <int B>
__global__ __launch_bounds__(kBlock) void k_path_renorm(int64_t m, float *zh, float *zl) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < m;
       i += int64_t(gridDim.x) * kBlock) {
    const float h = zh[i], l = zl[i];
    zh[i] = h + l;
    zl[i] = twosum_err(h, l);
  }
}

// copy slot columns: dst[j*ds + so] = src[j*ss + si] for j < k
__global__ __launch_bounds__(kBlock) void k_strided_copy(int64_t k, const float *src, int64_t ss,
                                                         int64_t si, float *dst, int64_t ds,
                                                         int64_t so) {
  for (int64_t j = int64_t(blockIdx.x) * kBlock + threadIdx.x; j < k;
       j += int64_t(gridDim.x) * kBlock)
    dst[j * ds + so] = src ? src[j * ss + si] : 0.0f;
}

// dst[i] = float(src[i * stride + slot]) for i < n: one slot's FP64 fitted values
__global__ __launch_bounds__(kBlock) void k_slot_round(int64_t n, const double *src,
                                                       int64_t stride, int64_t slot, float *dst) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * kBlock)
    dst[i] = float(src[i * stride + slot]);
}

static unsigned g1(int64_t m, unsigned cap = 4096) {
  int64_t b = (m + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return unsigned(b);
}

template <int B>
static int path_check(const gencd_csc *X, const float *y, int loss, const PathWs &w, hipStream_t s,
                      std::vector<double> *red) {
  constexpr int GPB = kBlock / B;
  const int64_t n = X->n, k = X->k;
  hipLaunchKernelGGL(k_path_zero<B>, dim3(g1(std::max<int64_t>(n > k ? n : k, 8 * kRedRep) * B)),
                     dim3(kBlock), 0, s, w.z64, n, w.g64, k, w.rep);
  const unsigned gk = unsigned(std::min<int64_t>((k + GPB - 1) / GPB, 16384));
  const unsigned gn = unsigned(std::min<int64_t>((n + GPB - 1) / GPB, 2048));
  hipLaunchKernelGGL(k_path_spmv<B>, dim3(gk), dim3(kBlock), 0, s, X->col_ptr, X->row_idx, X->val,
                     k, w.W, w.z64);
  hipLaunchKernelGGL(k_path_rows<B>, dim3(gn), dim3(kBlock), 0, s, n, loss, y, w.z64, w.r64, w.zh,
                     w.zl, w.rep);
  hipLaunchKernelGGL(k_path_cols<B>, dim3(gk), dim3(kBlock), 0, s, X->col_ptr, X->row_idx, X->val,
                     k, w.r64, w.g64);
  hipLaunchKernelGGL(k_path_kkt<B>, dim3(std::min<unsigned>(gk, 4096)), dim3(kBlock), 0, s, k,
                     w.g64, w.W, w.lam64, 1.0 / double(n), w.rep);
  // fold once for the maximum |g| that the dual needs, and again after it
  hipLaunchKernelGGL(k_path_fold<B>, dim3(1), dim3(8 * B), 0, s, w.rep, w.red);
  hipLaunchKernelGGL(k_path_dual<B>, dim3(gn), dim3(kBlock), 0, s, n, loss, y, w.r64, w.lam64,
                     w.red, w.rep);
  hipLaunchKernelGGL(k_path_fold<B>, dim3(1), dim3(8 * B), 0, s, w.rep, w.red);
  GENCD_HIP(hipGetLastError());
  red->resize(size_t(8) * B);
  GENCD_HIP(hipMemcpyAsync(red->data(), w.red, sizeof(double) * 8 * B, hipMemcpyDeviceToHost, s));
  GENCD_HIP(hipStreamSynchronize(s));
  return GENCD_OK;
}

struct PathSetup {
  Ws base;
  int piece;
  int32_t n_short, n_lpieces;
  int64_t k_live;
};

int path_setup(const gencd_csc *X, const float *y, const gencd_params *p, void *ws, size_t bytes,
               hipStream_t s, PathSetup *out, size_t *used);

size_t path_workspace_bytes(int64_t n, int64_t k, int64_t nnz, int64_t S, int B, int piece,
                            int short_max) {
  return workspace_layout(n, k, nnz, piece, short_max, false, 0, nullptr, nullptr) + 256 +
         path_layout(n, k, S, B, nullptr, nullptr) + 256;
}

// HIP events of one call, released on every return path.
struct PathEvents {
  std::vector<hipEvent_t> v;
  ~PathEvents() {
    for (auto e : v)
      if (e) (void)hipEventDestroy(e);
  }
};

// A captured epoch and the private stream it was captured on, released on
// every return path.
struct PathGraph {
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cs = nullptr;
  ~PathGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (g) (void)hipGraphDestroy(g);
    if (cs) (void)hipStreamDestroy(cs);
  }
};

template <int B>
int path_run(const gencd_csc *X, const float *y, const gencd_params *p, const double *lambdas,
             int32_t L, float *W_out, float *Z_out, char *path_base, const PathSetup &su,
             hipStream_t s, gencd_stats *stats) {
  const int64_t n = X->n, k = X->k, k_live = su.k_live;
  int64_t S = std::min<int64_t>(p->select_size, std::max<int64_t>(k_live, 1));
  PathWs w{};
  path_layout(n, k, S, B, path_base, &w);
  const Ws &ws = su.base;
  // slots
  std::vector<int32_t> slot_lambda(B, -1);   // lambda index held by each slot
  std::vector<int32_t> lambda_slot(L, -1);
  std::vector<int32_t> done(L, 0);
  std::vector<int64_t> start_epoch(L, 0);
  std::vector<int64_t> end_epoch(L, -1);  // epoch of the check that retired the lambda
  std::vector<char> z_valid(B, 0);         // the slot's z is X times its w
  std::vector<float> lam_host(B, 0.0f);
  std::vector<double> lam64_host(B, 0.0);
  std::vector<int32_t> act_host(B, 0);
  int32_t next = 0;
  int st = fill_f32(w.W, k * B, 0.0f, s);
  if (st) return st;
  // *z_ok: whether the slot's z now equals X times its warm start, so no
  // re-sync is needed.  After a check every slot's (z_hi, z_lo) is the split
  // of its FP64 X w; a predecessor still held in a slot, or retired by this
  // very check (its slot not yet refilled, see below), lends its column of
  // z with its weights.
  auto admit = [&](int slot, int64_t epoch, bool *z_ok) -> int {
    const int32_t t = next++;
    *z_ok = false;
    slot_lambda[slot] = t;
    lambda_slot[t] = slot;
    lam_host[slot] = float(lambdas[t]);
    lam64_host[slot] = lambdas[t];
    act_host[slot] = 1;
    start_epoch[t] = epoch;
    // warm start from the latest iterate of the predecessor (decreasing lambdas)
    const float *src = nullptr;
    int64_t ss = 0, si = 0;
    int32_t zsrc = -1;  // slot whose z column matches the warm start
    if (t > 0 && lambda_slot[t - 1] >= 0 && !done[t - 1]) {
      src = w.W;
      ss = B;
      si = lambda_slot[t - 1];
      if (z_valid[si]) zsrc = int32_t(si);
    } else if (t > 0 && done[t - 1]) {
      src = W_out + int64_t(t - 1) * k;
      ss = 1;
      si = 0;
      // slots are refilled in increasing order with increasing lambdas, so
      // the predecessor's slot still holds its z (or is this slot)
      if (end_epoch[t - 1] == epoch && z_valid[lambda_slot[t - 1]]) zsrc = lambda_slot[t - 1];
    }
    if (src)
      hipLaunchKernelGGL(k_strided_copy, dim3(g1(k)), dim3(kBlock), 0, s, k, src, ss, si, w.W,
                         int64_t(B), int64_t(slot));
    if (zsrc >= 0 && zsrc != slot) {
      hipLaunchKernelGGL(k_strided_copy, dim3(g1(n)), dim3(kBlock), 0, s, n, w.zh, int64_t(B),
                         int64_t(zsrc), w.zh, int64_t(B), int64_t(slot));
      hipLaunchKernelGGL(k_strided_copy, dim3(g1(n)), dim3(kBlock), 0, s, n, w.zl, int64_t(B),
                         int64_t(zsrc), w.zl, int64_t(B), int64_t(slot));
    }
    *z_ok = zsrc >= 0;
    z_valid[slot] = *z_ok;
    return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
  };
  // a lambda may enter once its predecessor has run `stagger` epochs (or is
  // done), so that it starts from a partly converged iterate
  const int64_t stagger = p->stagger > 0 ? p->stagger : 0;
  auto may_admit = [&](int64_t e) {
    return next < L && (stagger == 0 || next == 0 || done[next - 1] ||
                        e - start_epoch[next - 1] >= stagger);
  };
  for (int slot = 0; slot < B && may_admit(0); ++slot) {
    bool z_ok;  // the first check re-syncs every slot anyway
    st = admit(slot, 0, &z_ok);
    if (st) return st;
  }
  auto push_slots = [&]() -> int {
    GENCD_HIP(hipMemcpyAsync(w.lam, lam_host.data(), sizeof(float) * B, hipMemcpyHostToDevice, s));
    GENCD_HIP(hipMemcpyAsync(w.lam64, lam64_host.data(), sizeof(double) * B,
                             hipMemcpyHostToDevice, s));
    GENCD_HIP(hipMemcpyAsync(w.active, act_host.data(), sizeof(int32_t) * B,
                             hipMemcpyHostToDevice, s));
    return GENCD_OK;
  };
  st = push_slots();
  if (st) return st;

  int64_t *epoch_dev = reinterpret_cast<int64_t *>(ws.red + 12);
  st = fill_f64(ws.red + 12, 1, 0.0, s);
  if (st) return st;
  PathArgs a{};
  a.col_ptr = X->col_ptr;
  a.row_idx = X->row_idx;
  a.val = X->val;
  a.y = y;
  a.c = ws.c;
  a.col_of_pos = ws.col_of_pos;
  a.pdesc = ws.desc_s;  // the single-problem descriptors are not used here
  a.n_f = float(n);
  a.loss = p->loss;
  a.W = w.W;
  a.zh = w.zh;
  a.zl = w.zl;
  a.lam = w.lam;
  a.active = w.active;
  a.delta = w.delta;
  a.improve = p->improve_steps;
  const int64_t check_every = p->check_every;  // 0: adaptive, on the youngest slot's age
  int64_t next_check = 0;
  // measured on the 64-lambda binary workload: the staged update wins at
  // B = 64 (one full wave per column row), the block update below that
  constexpr bool upd_staged = B == 64;
  const bool fused = (p->flags & GENCD_FUSED) != 0;
  const bool fused_epoch = fused && (p->flags & GENCD_FUSED_EPOCH) != 0;
  // the kernel instances with "improve delta_j" steps, or without
  const bool imp = p->improve_steps > 0;
  void (*const kfused)(PathArgs) = imp ? k_path_fused<B, true> : k_path_fused<B, false>;
  void (*const kpropose)(PathArgs) = imp ? k_path_propose<B, true> : k_path_propose<B, false>;
  std::vector<double> red;
  const int64_t T = (k_live + S - 1) / S;
  // One epoch: selection order (section 2.1), the shared windows' launches,
  // the renormalisation of (z_hi, z_lo) and the epoch counter.  No argument
  // depends on the epoch or on which lambdas the slots hold (those live in
  // device arrays), so GENCD_USE_GRAPH captures it once and replays it.
  // GENCD_PROFILE (plain launches only): an event pair around every fused
  // launch, or around every Propose and every Update launch; the totals of
  // the call go to stats[0].  Algorithmic bytes per nonzero of a launch's
  // columns: fused 12 + 16 B (row index, value, y; each slot's z_hi and z_lo
  // read and z_lo read-modify-write), Propose 12 + 8 B, Update 8 + 8 B; per
  // column: fused and Propose 20 + 8 B (descriptor, c; each slot's weight
  // read and written, or read and its delta written), Update 16 + 4 B.
  const bool use_graph = (p->flags & GENCD_USE_GRAPH) != 0;
  const bool prof = (p->flags & GENCD_PROFILE) != 0 && !use_graph;
  PathEvents pev;
  size_t ev_used = 0;
  std::vector<int> ev_kind;  // 0: fused or Propose pair, 1: Update pair
  std::vector<double> ev_bytes;
  double prof_ms[2] = {0.0, 0.0}, prof_by[2] = {0.0, 0.0};
  int64_t prof_n[2] = {0, 0};
  const size_t ev_cap = prof ? 8192 : 0;
  if (prof) {
    pev.v.assign(ev_cap, nullptr);
    for (auto &ev : pev.v)
      if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess) ev = nullptr;
    ev_kind.assign(ev_cap / 2, 0);
    ev_bytes.assign(ev_cap / 2, 0.0);
  }
  auto harvest = [&]() {  // after a stream synchronisation
    for (size_t u = 0; u + 1 < ev_used; u += 2) {
      float t = 0.0f;
      if (pev.v[u] && pev.v[u + 1] && hipEventElapsedTime(&t, pev.v[u], pev.v[u + 1]) == hipSuccess) {
        prof_ms[ev_kind[u / 2]] += double(t);
        prof_by[ev_kind[u / 2]] += ev_bytes[u / 2];
        ++prof_n[ev_kind[u / 2]];
      }
    }
    ev_used = 0;
  };
  const double nnz_per_col = double(X->nnz) / double(std::max<int64_t>(k_live, 1));
  // record the start of a timed launch; returns the pair's index or -1
  auto tstart = [&](hipStream_t es, int kind, double cols, double per_nnz, double per_col) -> long {
    if (!prof || ev_used + 2 > ev_cap) return -1;
    const size_t u = ev_used;
    ev_used += 2;
    ev_kind[u / 2] = kind;
    ev_bytes[u / 2] = cols * (nnz_per_col * per_nnz + per_col);
    if (pev.v[u]) (void)hipEventRecord(pev.v[u], es);
    return long(u);
  };
  auto tstop = [&](hipStream_t es, long u) {
    if (u >= 0 && pev.v[size_t(u) + 1]) (void)hipEventRecord(pev.v[size_t(u) + 1], es);
  };
  auto enqueue_epoch = [&](hipStream_t es) -> int {
    int rc = launch_epoch_order(ws, k_live, GENCD_SHOTGUN, p->seed, epoch_dev, 0, S, T, es);
    if (rc) return rc;
    hipLaunchKernelGGL(k_path_desc, dim3(g1(k_live)), dim3(kBlock), 0, es, k_live, ws.col_of_pos,
                       X->col_ptr, ws.desc_s);
    if (fused_epoch) {
      // every position of the epoch in one launch: S workgroups, each one
      // column at a time in the order of its positions (grid stride S)
      a.win_lo = 0;
      a.win_hi = int32_t(k_live);
      const long u = tstart(es, 0, double(k_live), 12.0 + 16.0 * B, 20.0 + 8.0 * B);
      hipLaunchKernelGGL(kfused, dim3(unsigned(std::min<int64_t>(S, 65536))), dim3(kBlock), 0, es,
                         a);
      tstop(es, u);
    }
    for (int64_t t = 0; t < (fused_epoch ? 0 : T); ++t) {
      a.win_lo = int32_t(t * S);
      a.win_hi = int32_t(std::min(k_live, (t + 1) * S));
      const int64_t npos = a.win_hi - a.win_lo;
      const unsigned grid = unsigned(std::min<int64_t>(npos > 0 ? npos : 1, 65536));
      if (fused) {
        const long u = tstart(es, 0, double(npos), 12.0 + 16.0 * B, 20.0 + 8.0 * B);
        hipLaunchKernelGGL(kfused, dim3(grid), dim3(kBlock), 0, es, a);
        tstop(es, u);
        continue;
      }
      const long u0 = tstart(es, 0, double(npos), 12.0 + 8.0 * B, 20.0 + 8.0 * B);
      hipLaunchKernelGGL(kpropose, dim3(grid), dim3(kBlock), 0, es, a);
      tstop(es, u0);
      const long u1 = tstart(es, 1, double(npos), 8.0 + 8.0 * B, 16.0 + 4.0 * B);
      if constexpr (upd_staged)
        hipLaunchKernelGGL(k_path_update_staged<B>,
                           dim3(unsigned(std::min<int64_t>((npos + kBlock / B - 1) / (kBlock / B), 16384))),
                           dim3(kBlock), 0, es, a);
      else
        hipLaunchKernelGGL(k_path_update<B>, dim3(grid), dim3(kBlock), 0, es, a);
      tstop(es, u1);
    }
    hipLaunchKernelGGL(k_path_renorm<B>, dim3(g1(n * B)), dim3(kBlock), 0, es, n * B, w.zh, w.zl);
    rc = launch_inc_epoch(epoch_dev, es);
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
  };
  PathGraph graph;
  int64_t e = 0;
  bool resync = true;
  int remaining = L;
  while (remaining > 0) {
    if (resync || e >= next_check) {
      st = path_check<B>(X, y, p->loss, w, s, &red);
      if (st) return st;
      if (prof) harvest();  // the check synchronised the stream
      resync = false;
      std::fill(z_valid.begin(), z_valid.end(), 1);  // the check re-synced every slot's z
      bool admitted = false;
      for (int slot = 0; slot < B; ++slot) {
        const int32_t t = slot_lambda[slot];
        if (t < 0 || done[t]) continue;
        const double lsum = red[slot * 8 + 0], l1 = red[slot * 8 + 1], dsum = red[slot * 8 + 5];
        unsigned long long kb;
        std::memcpy(&kb, &red[slot * 8 + 2], 8);
        double kkt;
        std::memcpy(&kkt, &kb, 8);
        const double obj = lsum / double(n) + lam64_host[slot] * l1;
        gencd_stats &so = stats[t];
        so.objective = obj;
        so.kkt_max = kkt;
        so.gap = obj - dsum / double(n);
        so.nnz_w = int64_t(red[slot * 8 + 3]);
        so.epochs = e - start_epoch[t];
        so.lambda_max = 0.0;
        if (!std::isfinite(obj)) return GENCD_ERR_DIVERGED;
        const bool conv = kkt <= p->kkt_tol &&
                          (p->gap_tol <= 0.0 || so.gap <= p->gap_tol * std::fabs(obj));
        const bool out_of_epochs = so.epochs >= p->max_epochs;
        if (conv || out_of_epochs) {
          so.converged = conv ? 1 : 0;
          hipLaunchKernelGGL(k_strided_copy, dim3(g1(k)), dim3(kBlock), 0, s, k, w.W, int64_t(B),
                             int64_t(slot), W_out + int64_t(t) * k, int64_t(1), int64_t(0));
          if (Z_out)  // the check just formed z64 = X W of this slot
            hipLaunchKernelGGL(k_slot_round, dim3(g1(n)), dim3(kBlock), 0, s, n, w.z64,
                               int64_t(B), int64_t(slot), Z_out + int64_t(t) * n);
          GENCD_HIP(hipGetLastError());
          done[t] = 1;
          end_epoch[t] = e;
          --remaining;
          slot_lambda[slot] = -1;
          act_host[slot] = 0;
          lam_host[slot] = 0.0f;
          lam64_host[slot] = 0.0;
        }
      }
      bool stale = false;  // some admitted slot's z is not X w
      for (int slot = 0; slot < B && may_admit(e); ++slot) {
        if (slot_lambda[slot] >= 0) continue;
        bool z_ok;
        st = admit(slot, e, &z_ok);
        if (st) return st;
        admitted = true;
        stale |= !z_ok;
      }
      st = push_slots();
      if (st) return st;
      if (remaining == 0) break;
      // next check: from the age of the youngest slot (adaptive interval)
      int64_t young = -1;
      for (int slot = 0; slot < B; ++slot) {
        const int32_t t = slot_lambda[slot];
        if (t >= 0 && !done[t]) young = young < 0 ? e - start_epoch[t] : std::min(young, e - start_epoch[t]);
      }
      next_check = e + check_interval(check_every, young < 0 ? 0 : young);
      bool free_slot = false;
      for (int slot = 0; slot < B; ++slot) free_slot |= slot_lambda[slot] < 0;
      if (free_slot && stagger > 0 && next < L && !done[next - 1])
        next_check = std::min(next_check, start_epoch[next - 1] + stagger);  // the next entry
      if (admitted && stale) {
        resync = true;  // z of an admitted slot must be recomputed from W
        continue;
      }
    }
    // one epoch over the live columns with shared windows
    if (use_graph) {
      if (!graph.exec) {
        // capture on a private stream (the caller's may be the legacy
        // default stream, which cannot be captured); replay on the caller's
        if (!graph.cs) GENCD_HIP(hipStreamCreateWithFlags(&graph.cs, hipStreamNonBlocking));
        GENCD_HIP(hipStreamBeginCapture(graph.cs, hipStreamCaptureModeRelaxed));
        st = enqueue_epoch(graph.cs);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(graph.cs, &g);
        graph.g = g;
        if (st) return st;
        if (ce != hipSuccess || !g) return GENCD_ERR_HIP;
        GENCD_HIP(hipGraphInstantiate(&graph.exec, g, nullptr, nullptr, 0));
      }
      GENCD_HIP(hipGraphLaunch(graph.exec, s));
    } else {
      if (prof && ev_used + 4 * size_t(T) + 2 > ev_cap) {  // room for one more epoch
        GENCD_HIP(hipStreamSynchronize(s));
        harvest();
      }
      st = enqueue_epoch(s);
      if (st) return st;
    }
    for (int slot = 0; slot < B; ++slot) {
      const int32_t t = slot_lambda[slot];
      if (t >= 0 && !done[t]) {
        stats[t].iters += T;
        stats[t].coord_updates += k_live;
        stats[t].nnz_visits += X->nnz;
        stats[t].nnz_updates += X->nnz;
      }
    }
    ++e;
  }
  GENCD_HIP(hipStreamSynchronize(s));
  if (prof) {
    harvest();
    stats[0].prof_launches = prof_n[0];
    stats[0].prof_kernel_ms = prof_ms[0];
    stats[0].prof_bytes = prof_by[0];
    stats[0].prof_update_launches = prof_n[1];
    stats[0].prof_update_ms = prof_ms[1];
    stats[0].prof_update_bytes = prof_by[1];
  }
  return GENCD_OK;
}

}  // namespace gencd

using namespace gencd;

extern "C" {

int gencd_path_workspace_bytes(const gencd_csc *X, const gencd_params *p, int32_t B,
                               size_t *out_bytes) {
  if (!X || !p || !out_bytes || X->n <= 0 || X->k <= 0 || X->nnz < 0) return GENCD_ERR_INVALID_ARG;
  if (B != 16 && B != 32 && B != 64) return GENCD_ERR_INVALID_ARG;
  if (p->select_size <= 0) return GENCD_ERR_INVALID_ARG;
  const int piece = p->piece ? p->piece : kDefaultPiece;
  const int group = p->group ? p->group : kDefaultGroup;
  *out_bytes = path_workspace_bytes(X->n, X->k, X->nnz, std::min<int64_t>(p->select_size, X->k), B,
                                    piece, group * kUnroll) + 256;
  return GENCD_OK;
}

int gencd_solve_path(const gencd_csc *X, const float *y, const gencd_params *p,
                     const double *lambdas, int32_t L, int32_t B, float *W, float *Z, void *ws,
                     size_t ws_bytes, hipStream_t stream, gencd_stats *stats) {
  (void)hipGetLastError();
  auto t0 = std::chrono::steady_clock::now();
  if (!X || !p || !lambdas || L <= 0 || !W || !stats) return GENCD_ERR_INVALID_ARG;
  if (B != 16 && B != 32 && B != 64) return GENCD_ERR_INVALID_ARG;
  if (p->rule != GENCD_SHOTGUN ||
      ((p->flags & GENCD_FUSED) && (p->flags & GENCD_EXACT_ACCUM)) ||
      ((p->flags & GENCD_FUSED_EPOCH) && !(p->flags & GENCD_FUSED)))
    return GENCD_ERR_UNSUPPORTED;
  if (p->select_size <= 0 || !(p->kkt_tol >= 0.0) || !(p->gap_tol >= 0.0) || p->max_epochs < 0 ||
      p->improve_steps < 0 || p->improve_steps > 1000000)
    return GENCD_ERR_INVALID_ARG;
  if (p->loss != GENCD_SQUARED && p->loss != GENCD_LOGISTIC) return GENCD_ERR_INVALID_ARG;
  for (int32_t t = 0; t < L; ++t)
    if (!(lambdas[t] >= 0.0) || !std::isfinite(lambdas[t])) return GENCD_ERR_INVALID_ARG;
  std::memset(stats, 0, sizeof(gencd_stats) * size_t(L));
  size_t need = 0;
  int st = gencd_path_workspace_bytes(X, p, B, &need);
  if (st) return st;
  if (!ws || ws_bytes < need) return GENCD_ERR_WORKSPACE;
  PathSetup su{};
  size_t used = 0;
  st = path_setup(X, y, p, ws, ws_bytes, stream, &su, &used);
  if (st) return st;
  char *pb = static_cast<char *>(ws) + used;
  size_t mis = reinterpret_cast<uintptr_t>(pb) % 256;
  if (mis) pb += 256 - mis;
  switch (B) {
    case 16: st = path_run<16>(X, y, p, lambdas, L, W, Z, pb, su, stream, stats); break;
    case 32: st = path_run<32>(X, y, p, lambdas, L, W, Z, pb, su, stream, stats); break;
    default: st = path_run<64>(X, y, p, lambdas, L, W, Z, pb, su, stream, stats); break;
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int all = 1;
  for (int32_t t = 0; t < L; ++t) {
    stats[t].seconds = secs;
    all &= stats[t].converged;
  }
  if (st) return st;
  return all ? GENCD_OK : GENCD_NOT_CONVERGED;
}

}  // extern "C"
