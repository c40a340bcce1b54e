// Host driver of Algorithm 1 and the C-ABI entry points of libgencd.
//
// gencd_solve runs, per epoch: the selection order (section 2.1), then for
// every iteration one Propose launch (Algorithm 2 / 4; for accept-all rules
// it also applies single-piece updates), the Accept launch of the greedy
// rules (section 2.3), an Update launch for the remaining updates
// (Algorithm 3) and a residual refresh.  Every check_every epochs an FP64
// pass recomputes z = Xw, the objective of Eq. (1) and the KKT violations,
// re-synchronises the FP32 state from it and decides convergence on the
// host.
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "gencd_common.hpp"
#include "gencd_kernels.hpp"
#include "gencd_solver.hpp"

namespace gencd {

static constexpr size_t kAlign = 256;

// long pieces: a long column has more than short_max nonzeros, so there are
// at most nnz / (short_max + 1) of them, each with at most one partial piece
int64_t max_lpieces_for(int64_t k, int64_t nnz, int piece, int short_max) {
  (void)k;
  return nnz / piece + nnz / (short_max + 1) + 2;
}

static int short_max_of(int group) { return group * kUnroll; }

namespace {
struct Carver {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(int64_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += size_t(count > 0 ? count : 1) * sizeof(T);
    return p;
  }
};
}  // namespace

size_t workspace_layout(int64_t n, int64_t k, int64_t nnz, int piece, int short_max, bool rho,
                        int64_t nblocks, void *base, Ws *ws) {
  Carver c{static_cast<char *>(base)};
  Ws w{};
  const int64_t ml = max_lpieces_for(k, nnz, piece, short_max);
  const int64_t rl = radix_hist_len(k);
  int64_t scan_len = ml > k + 1 ? ml : k + 1;
  if (rl > scan_len) scan_len = rl;
  w.max_lpieces = ml;
  w.scan_part_len = scan_partials_for(scan_len);
  w.c = c.take<float>(k);
  w.live = c.take<int32_t>(k);
  w.all_soff = c.take<int32_t>(k + 1);
  w.all_loff = c.take<int32_t>(k + 1);
  w.desc_all_s = c.take<int4>(k);
  w.live_rec = c.take<int4>(k);
  w.desc_all_l = c.take<int4>(ml);
  w.tmp_cnt = c.take<int32_t>(k + 1);
  w.tmp_cnt2 = c.take<int32_t>(k + 1);
  w.scan_part = c.take<int32_t>(int64_t(w.scan_part_len));
  w.cls_off = c.take<int32_t>(k + 1);
  w.cls_mem = c.take<int32_t>(k);
  w.rad_h = c.take<int32_t>(rl);
  w.rad_o = c.take<int32_t>(rl);
  w.col_of_pos = c.take<int32_t>(k);
  w.soff = c.take<int32_t>(k + 1);
  w.loff = c.take<int32_t>(k + 1);
  w.desc_s = c.take<int4>(k);
  w.desc_l = c.take<int4>(ml);
  w.win_off = c.take<int32_t>(k + 1);
  w.wbl = c.take<int32_t>(k + 2);
  w.delta = c.take<float>(k);
  w.phi = c.take<float>(k);
  w.gacc = c.take<float>(ml);
  w.wsnap = c.take<float>(k);
  w.acc = c.take<int32_t>(k);
  w.zs = c.take<float4>(n);
  w.w_ckpt = c.take<float>(k);
  w.rs = c.take<float>(n);
  w.z64 = c.take<double>(n);
  w.r64 = c.take<double>(n);
  w.g64 = c.take<double>(k);
  w.red = c.take<double>(16);
  w.rrep = c.take<double>(int64_t(kChkRep) * 16);
  w.scat = c.take<unsigned long long>(int64_t(kChkRep) * 16);
  if (rho || nblocks > 0) {
    w.rho_dinv = c.take<double>(k);
    w.rho_x = c.take<double>(k);
    w.rho_hist = c.take<double>(kRhoMaxIters);
  }
  w.nblocks = nblocks;
  if (nblocks > 0) {
    w.bbase = c.take<int32_t>(k);
    w.bcol = c.take<int32_t>(k);
    w.bp = c.take<int32_t>(nblocks);
    w.bstart = c.take<int32_t>(nblocks + 1);
    w.bwin = c.take<int32_t>(nblocks + 1);
    w.bs = c.take<double>(n * nblocks);
    w.bhist = c.take<double>(int64_t(kBlockRhoMaxIters) * nblocks);
  }
  if (ws) *ws = w;
  return c.off + kAlign;
}

bool csc_ok(const gencd_csc *X) {
  if (!X || X->n <= 0 || X->k <= 0 || X->nnz < 0) return false;
  if (X->n > INT32_MAX || X->k >= INT32_MAX) return false;
  if (!X->col_ptr) return false;
  if (X->nnz > 0 && (!X->row_idx || !X->val)) return false;
  return true;
}

// Block Shotgun: number of preset blocks the workspace holds.
int64_t blocks_of(const gencd_params *p) {
  return (p && p->rule == GENCD_BLOCK_SHOTGUN && p->block > 0) ? p->block : 0;
}

// Shotgun and Thread-Greedy with select_size 0 take |J| from the estimate.
bool wants_rho(const gencd_params *p) {
  return p &&
         (p->rule == GENCD_SHOTGUN || p->rule == GENCD_THREAD_GREEDY || p->rule == GENCD_TOP_GREEDY) &&
         p->select_size == 0;
}

int resolve_schedule(const gencd_params *p, int *piece, int *group) {
  int g = (p && p->group) ? p->group : kDefaultGroup;
  if (g != 4 && g != 8 && g != 16 && g != 32) return GENCD_ERR_INVALID_ARG;
  int pc = (p && p->piece) ? p->piece : kDefaultPiece;
  if (pc < 64 || pc % 64 != 0 || pc > (1 << 22)) return GENCD_ERR_INVALID_ARG;
  *piece = pc;
  *group = g;
  return GENCD_OK;
}

int params_ok(const gencd_params *p, bool need_rule) {
  if (!p) return GENCD_ERR_INVALID_ARG;
  if (p->loss != GENCD_SQUARED && p->loss != GENCD_LOGISTIC) return GENCD_ERR_INVALID_ARG;
  if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return GENCD_ERR_INVALID_ARG;
  if (p->improve_steps < 0 || p->improve_steps > 1000000) return GENCD_ERR_INVALID_ARG;
  if (p->residual < 0 || p->residual > 2) return GENCD_ERR_INVALID_ARG;
  if (!need_rule) return GENCD_OK;
  if (p->rule < GENCD_CYCLIC || p->rule > GENCD_BLOCK_SHOTGUN) return GENCD_ERR_INVALID_ARG;
  if (p->rule == GENCD_BLOCK_SHOTGUN && (p->block < 1 || p->block > kMaxBlocks))
    return GENCD_ERR_INVALID_ARG;
  if ((p->rule == GENCD_SHOTGUN || p->rule == GENCD_THREAD_GREEDY ||
       p->rule == GENCD_TOP_GREEDY) &&
      p->select_size < 0)
    return GENCD_ERR_INVALID_ARG;
  if ((p->rule == GENCD_THREAD_GREEDY || p->rule == GENCD_TOP_GREEDY) && p->block <= 0)
    return GENCD_ERR_INVALID_ARG;
  if (p->rule == GENCD_COLORING && (!p->color || p->num_colors <= 0)) return GENCD_ERR_INVALID_ARG;
  if ((p->flags & GENCD_FUSED) &&
      ((p->rule != GENCD_CYCLIC && p->rule != GENCD_STOCHASTIC && p->rule != GENCD_SHOTGUN &&
        p->rule != GENCD_BLOCK_SHOTGUN) ||
       (p->flags & GENCD_EXACT_ACCUM) || p->improve_steps > 0))
    return GENCD_ERR_UNSUPPORTED;
  if (!(p->kkt_tol >= 0.0) || !(p->gap_tol >= 0.0) || p->max_epochs < 0 ||
      p->check_every < -1000)
    return GENCD_ERR_INVALID_ARG;
  return GENCD_OK;
}

// Device -> host copy of the reduction block, then wait for the stream.
int read_red(const Ws &w, hipStream_t s, Red *out) {
  GENCD_HIP(hipMemcpyAsync(out, w.red, sizeof(Red), hipMemcpyDeviceToHost, s));
  GENCD_HIP(hipStreamSynchronize(s));
  return GENCD_OK;
}

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, sizeof d);
  return d;
}

// |J| = P* = floor(k_live / (2 rho)) clamped to [1, k_live] (section 4.1).
int64_t pstar_of(int64_t k_live, double rho) {
  if (!(rho > 0.0)) return 1;
  const double q = std::floor(double(k_live) / (2.0 * rho));
  if (q < 1.0) return 1;
  if (q > double(k_live)) return k_live > 0 ? k_live : 1;
  return int64_t(q);
}

int setup(const gencd_csc *X, const float *y, int loss, const gencd_params *p, void *ws_base,
          size_t ws_bytes, bool validate_matrix, hipStream_t s, Setup *out, int rho_iters,
          bool need_y, int64_t nblocks, int block_iters) {
  if (!csc_ok(X) || (need_y && !y)) return GENCD_ERR_INVALID_ARG;
  if (rho_iters < 0 || rho_iters > kRhoMaxIters) return GENCD_ERR_INVALID_ARG;
  if (nblocks < 0 || nblocks > kMaxBlocks || block_iters < 1 || block_iters > kBlockRhoMaxIters)
    return GENCD_ERR_INVALID_ARG;
  int st = resolve_schedule(p, &out->piece, &out->group);
  if (st) return st;
  const int smax = short_max_of(out->group);
  if (max_lpieces_for(X->k, X->nnz, out->piece, smax) >= INT32_MAX ||
      X->nnz >= (int64_t(1) << 32))
    return GENCD_ERR_UNSUPPORTED;
  size_t need = workspace_layout(X->n, X->k, X->nnz, out->piece, smax, rho_iters > 0, nblocks, nullptr, nullptr);
  if (!ws_base || ws_bytes < need) return GENCD_ERR_WORKSPACE;
  // align the carve base
  char *base = static_cast<char *>(ws_base);
  size_t mis = reinterpret_cast<uintptr_t>(base) % kAlign;
  if (mis) base += kAlign - mis;
  workspace_layout(X->n, X->k, X->nnz, out->piece, smax, rho_iters > 0, nblocks, base, &out->ws);
  const Ws &w = out->ws;
  st = fill_f64(w.red, 16, 0.0, s);
  if (st) return st;
  st = launch_validate(X, y, loss, validate_matrix, reinterpret_cast<unsigned long long *>(w.red) + 10, s);
  if (st) return st;
  st = launch_preprocess(X, loss, out->piece, smax, w, s);
  if (st) return st;
  int32_t host[3] = {0, 0, 0};
  Red r{};
  GENCD_HIP(hipMemcpyAsync(&host[0], w.all_soff + X->k, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GENCD_HIP(hipMemcpyAsync(&host[1], w.soff + X->k, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  GENCD_HIP(hipMemcpyAsync(&host[2], w.all_loff + X->k, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  st = read_red(w, s, &r);
  if (st) return st;
  if (r.bad & 1ull) return GENCD_ERR_BAD_MATRIX;
  if (r.bad & 2ull) return GENCD_ERR_BAD_LABELS;
  out->n_short = host[0];
  out->k_live = host[1];
  out->n_lpieces = host[2];
  st = launch_curvature(X, loss, out->n_short, out->n_lpieces, w, s);
  if (st) return st;
  if (rho_iters > 0) {
    // power iteration; reads the column sums of squares that the curvature
    // pass left in g64
    out->rho_hist.assign(size_t(rho_iters), 0.0);
    if (out->k_live > 0) {
      st = launch_rho(X, out->n_short, out->n_lpieces, w, out->k_live, rho_iters, s);
      if (st) return st;
      GENCD_HIP(hipMemcpyAsync(out->rho_hist.data(), w.rho_hist, sizeof(double) * size_t(rho_iters),
                               hipMemcpyDeviceToHost, s));
      GENCD_HIP(hipStreamSynchronize(s));
      for (double &h : out->rho_hist) h = std::sqrt(h);
    }
    out->rho = out->rho_hist.back();
  }
  if (nblocks > 0 && out->k_live > 0) {
    // preset blocks and P_b* = floor(k_b / (2 rho_b)) clamped to [1, k_b]
    const int64_t nb = std::min<int64_t>(nblocks, out->k_live);
    out->ws.nblocks = nb;
    st = launch_block_setup(X, out->n_short, out->n_lpieces, out->ws, out->k_live,
                            p ? p->seed : 0, block_iters, s);
    if (st) return st;
    std::vector<double> h(size_t(block_iters) * size_t(nb));
    GENCD_HIP(hipMemcpyAsync(h.data(), w.bhist, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    GENCD_HIP(hipStreamSynchronize(s));
    out->brho.resize(size_t(nb));
    out->bp.resize(size_t(nb));
    for (int64_t b = 0; b < nb; ++b) {
      const double r = std::sqrt(h[size_t(block_iters - 1) * size_t(nb) + size_t(b)]);
      const int64_t kb = block_lo(b + 1, out->k_live, nb) - block_lo(b, out->k_live, nb);
      int64_t pb = 1;
      if (r > 0.0) {
        const double f = std::floor(double(kb) / (2.0 * r));
        pb = f < 1.0 ? 1 : (f > double(kb) ? kb : int64_t(f));
      }
      out->brho[size_t(b)] = r;
      out->bp[size_t(b)] = int32_t(pb);
    }
    GENCD_HIP(hipMemcpyAsync(out->ws.bp, out->bp.data(), sizeof(int32_t) * size_t(nb),
                             hipMemcpyHostToDevice, s));
    GENCD_HIP(hipStreamSynchronize(s));
  }
  st = fill_f32(w.gacc, w.max_lpieces, 0.0f, s);
  if (st) return st;
  return fill_i32(w.acc, X->k, 0, s);
}

int enqueue_check(const gencd_csc *X, const float *y, int loss, double lam, const float *w,
                  const Setup &su, bool resync, hipStream_t s, double *host_rep, Red *host_red) {
  int st = launch_check(X, y, loss, lam, w, su.n_short, su.n_lpieces, su.ws, resync, s);
  if (st) return st;
  GENCD_HIP(hipMemcpyAsync(host_rep, su.ws.rrep, sizeof(double) * kChkRep * 16,
                           hipMemcpyDeviceToHost, s));
  GENCD_HIP(hipMemcpyAsync(host_red, su.ws.red, sizeof(Red), hipMemcpyDeviceToHost, s));
  return GENCD_OK;
}

void fold_check(const double *rep, const Red &red, int64_t n, double lam, CheckOut *out) {
  Red r = red;
  r.loss_sum = r.l1 = r.dual_sum = 0.0;
  r.kkt_bits = r.nnz_w = r.gmax_bits = 0ull;
  unsigned long long drift_bits = 0ull;
  double zsq = 0.0;
  for (int i = 0; i < kChkRep; ++i) {  // fold in replica order
    const double *f = rep + i * 16;
    unsigned long long u[8];
    std::memcpy(u, f, sizeof(u));
    r.loss_sum += f[0];
    r.l1 += f[1];
    r.kkt_bits = std::max(r.kkt_bits, u[2]);
    r.nnz_w += u[3];
    r.gmax_bits = std::max(r.gmax_bits, u[4]);
    r.dual_sum += f[5];
    drift_bits = std::max(drift_bits, u[6]);
    zsq += f[7];
  }
  const double rms = std::sqrt(zsq / double(n));
  out->drift_rel = rms > 0.0 ? bits_to_double(drift_bits) / rms : 0.0;
  out->objective = r.loss_sum / double(n) + lam * r.l1;
  out->kkt = bits_to_double(r.kkt_bits);
  out->gap = out->objective - r.dual_sum / double(n);
  out->nnz_w = int64_t(r.nnz_w);
  out->acc_nnz = r.acc_nnz;
  out->acc_cnt = r.acc_cnt;
}

int run_check(const gencd_csc *X, const float *y, int loss, double lam, const float *w,
              const Setup &su, bool resync, hipStream_t s, CheckOut *out) {
  double rep[kChkRep * 16];
  Red r{};
  int st = enqueue_check(X, y, loss, lam, w, su, resync, s, rep, &r);
  if (st) return st;
  GENCD_HIP(hipStreamSynchronize(s));
  fold_check(rep, r, X->n, lam, out);
  return GENCD_OK;
}

namespace {

bool converged(const gencd_params *p, const CheckOut &ck) {
  if (!(ck.kkt <= p->kkt_tol)) return false;
  return p->gap_tol <= 0.0 || ck.gap <= p->gap_tol * std::fabs(ck.objective);
}

int mode_of(int rule) {
  if (rule == GENCD_COLORING) return 1;
  if (rule == GENCD_THREAD_GREEDY || rule == GENCD_GREEDY || rule == GENCD_TOP_GREEDY) return 2;
  return 0;
}

IterArgs base_args(const gencd_csc *X, const float *y, const gencd_params *p, const Setup &su,
                   float *w, float4 *zs) {
  const Ws &ws = su.ws;
  IterArgs a{};
  a.piece = su.piece;
  a.accept_top = p->rule == GENCD_TOP_GREEDY ? p->block : 0;
  a.improve = p->improve_steps;
  a.nrows = X->n;
  a.col_ptr = X->col_ptr;
  a.row_idx = X->row_idx;
  a.val = X->val;
  a.n_f = float(X->n);
  a.loss = p->loss;
  a.lam = float(p->lambda);
  a.c = ws.c;
  a.w = w;
  a.zs = zs;
  a.col_of_pos = ws.col_of_pos;
  a.loff = ws.loff;
  a.desc_s = ws.desc_s;
  a.desc_l = ws.desc_l;
  a.delta = ws.delta;
  a.phi = ws.phi;
  a.gacc = ws.gacc;
  a.gout = nullptr;
  a.wsnap = ws.wsnap;
  a.wbl = ws.wbl;
  a.acc = ws.acc;
  a.bw_pos = ws.tmp_cnt;  // free once the epoch order is built
  a.bw_phi = ws.tmp_cnt2;
  a.counters = reinterpret_cast<unsigned long long *>(ws.red) + 8;
  a.exact_accum = (p->flags & GENCD_EXACT_ACCUM) ? 1 : 0;
  a.scat = nullptr;
  return a;
}

// Colour classes: the live columns stably sorted by colour (members of a
// class in column order, though any order gives the same iteration: the
// members' rows are disjoint), and the class offsets read off the sorted
// keys.  No counter is shared between columns.
__global__ void k_class_keys(const int32_t *live, int64_t k_live, const int32_t *color, int32_t C,
                             uint32_t *keys, int32_t *vals, unsigned long long *bad) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < k_live;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int32_t j = live[t];
    int32_t c = color[j];
    if (c < 0 || c >= C) {
      atomicOr(bad, 4ull);  // reported as INVALID_ARG
      c = 0;
    }
    keys[t] = uint32_t(c);
    vals[t] = j;
  }
}

// off[c] = first sorted position with colour >= c, for c in [0, C]
__global__ void k_class_bounds(const uint32_t *keys, int64_t k_live, int32_t C, int32_t *off) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t <= k_live;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t lo = t == 0 ? 0 : int64_t(keys[t - 1]) + 1;
    const int64_t hi = t == k_live ? int64_t(C) : int64_t(keys[t]);
    for (int64_t c = lo; c <= hi; ++c) off[c] = int32_t(t);
  }
}

int build_classes(const Setup &su, const int32_t *color, int32_t C, hipStream_t s,
                  std::vector<int32_t> *sizes) {
  const Ws &w = su.ws;
  // sort buffers: set-up scratch that the epoch order overwrites later
  uint32_t *k0 = reinterpret_cast<uint32_t *>(w.tmp_cnt), *k1 = reinterpret_cast<uint32_t *>(w.col_of_pos);
  int32_t *v0 = w.tmp_cnt2, *v1 = w.soff;
  unsigned grid = unsigned(std::min<int64_t>((su.k_live + 255) / 256 + 1, 4096));
  hipLaunchKernelGGL(k_class_keys, dim3(grid), dim3(256), 0, s, w.live, su.k_live, color, C, k0,
                     v0, reinterpret_cast<unsigned long long *>(w.red) + 10);
  int ob = 0;
  int st = radix_sort_pairs(k0, v0, k1, v1, su.k_live, bits_for(uint64_t(C - 1)), w.rad_h, w.rad_o,
                            w.scan_part, s, &ob);
  if (st) return st;
  st = copy_i32(w.cls_mem, ob ? v1 : v0, su.k_live, s);
  if (st) return st;
  hipLaunchKernelGGL(k_class_bounds, dim3(grid), dim3(256), 0, s, ob ? k1 : k0, su.k_live, C,
                     w.cls_off);
  GENCD_HIP(hipGetLastError());
  std::vector<int32_t> off(size_t(C) + 1);
  GENCD_HIP(hipMemcpyAsync(off.data(), w.cls_off, sizeof(int32_t) * (C + 1),
                           hipMemcpyDeviceToHost, s));
  Red r{};
  st = read_red(w, s, &r);
  if (st) return st;
  if (r.bad & 4ull) return GENCD_ERR_INVALID_ARG;
  sizes->resize(size_t(C));
  for (int32_t c = 0; c < C; ++c) (*sizes)[c] = off[c + 1] - off[c];
  return GENCD_OK;
}

__global__ void k_check_list(const int32_t *J, int64_t m, int64_t k, unsigned long long *bad) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < m;
       t += int64_t(gridDim.x) * blockDim.x)
    if (J[t] < 0 || J[t] >= k) atomicOr(bad, 8ull);
}

// A captured epoch, released on every return path.
struct GraphHolder {
  hipGraph_t g = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cs = nullptr;  // capture stream
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (g) (void)hipGraphDestroy(g);
    exec = nullptr;
    g = nullptr;
  }
  ~GraphHolder() {
    reset();
    if (cs) (void)hipStreamDestroy(cs);
  }
};

// GENCD_PROFILE on plain launches: one thread waits on the device's
// constant-rate clock for `ticks` before an epoch's launches, so that the
// host has queued the whole epoch when the first of them starts and no
// event pair spans a wait for the host.  The wait ends by the clock or
// after `max_polls` polls, whichever comes first.
__global__ void k_host_lead(int64_t ticks, int64_t max_polls) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t t0 = wall_clock64();
  for (int64_t i = 0; i < max_polls && wall_clock64() - t0 < ticks; ++i)
    __builtin_amdgcn_s_sleep(8);
}

// HIP events owned by one solve call, released on every return path.
struct EventPool {
  std::vector<hipEvent_t> v;
  ~EventPool() {
    for (auto e : v)
      if (e) (void)hipEventDestroy(e);
  }
};

// Whether Propose reads a refreshed residual vector for a window of
// `positions` columns: forced by p->residual, or when the window's expected
// nonzeros reach 4 n (then one pass over the rows costs little next to the
// 12-byte row gathers it replaces with 4-byte ones).
bool wants_rs(const gencd_params *p, int64_t positions, int64_t nnz, int64_t k_live, int64_t n) {
  if (p->residual == 1) return false;
  if (p->residual == 2) return true;
  if (k_live <= 0) return false;
  return double(positions) * double(nnz) / double(k_live) >= 4.0 * double(n);
}

// Expected long pieces in a window of `positions` columns (sizes the grid;
// the kernels stride over the actual count).
int64_t long_bound_for(const Setup &su, int64_t positions) {
  if (su.n_lpieces <= 0 || su.k_live <= 0) return 0;
  const double per = double(su.n_lpieces) * double(positions) / double(su.k_live);
  int64_t b = int64_t(2.0 * per) + 32;
  return b < su.n_lpieces ? b : su.n_lpieces;
}

}  // namespace

struct PathSetup {
  Ws base;
  int piece;
  int32_t n_short, n_lpieces;
  int64_t k_live;
};

// Preprocessing shared with the batched path: the single-problem workspace
// occupies the front of `ws`; *used is its size.
int path_setup(const gencd_csc *X, const float *y, const gencd_params *p, void *ws, size_t bytes,
               hipStream_t s, PathSetup *out, size_t *used) {
  int st = params_ok(p, false);
  if (st) return st;
  Setup su;
  st = setup(X, y, p->loss, p, ws, bytes, (p->flags & GENCD_VALIDATE_DEVICE) != 0, s, &su);
  if (st) return st;
  out->base = su.ws;
  out->piece = su.piece;
  out->n_short = su.n_short;
  out->n_lpieces = su.n_lpieces;
  out->k_live = su.k_live;
  *used = workspace_layout(X->n, X->k, X->nnz, su.piece, short_max_of(su.group), false, 0, nullptr,
                           nullptr) +
          kAlign;
  return GENCD_OK;
}

// ---------------------------------------------------------------------------
// Solve
// ---------------------------------------------------------------------------
int solve_impl(const gencd_csc *X, const float *y, const gencd_params *p, float *w, float *z,
               void *ws_base, size_t ws_bytes, hipStream_t s, gencd_stats *stats) {
  (void)hipGetLastError();  // launch checks below must not see an earlier error
  auto t0 = std::chrono::steady_clock::now();
  gencd_stats loc{};
  gencd_stats *st_out = stats ? stats : &loc;
  std::memset(st_out, 0, sizeof(*st_out));
  int st = params_ok(p, true);
  if (st) return st;
  if (!w) return GENCD_ERR_INVALID_ARG;
  Setup su;
  st = setup(X, y, p->loss, p, ws_base, ws_bytes, (p->flags & GENCD_VALIDATE_DEVICE) != 0, s, &su,
             wants_rho(p) ? kRhoIters : 0, true, blocks_of(p));
  if (st) return st;
  const Ws &ws = su.ws;
  const int rule = p->rule;
  const int mode = mode_of(rule);
  const int64_t k_live = su.k_live;
  std::vector<int32_t> cls_sizes;
  int64_t C = 0;
  if (rule == GENCD_COLORING) {
    C = p->num_colors;
    if (C > X->k) return GENCD_ERR_INVALID_ARG;
    st = build_classes(su, p->color, int32_t(C), s, &cls_sizes);
    if (st) return st;
  }
  if (!(p->flags & GENCD_WARM_START)) {
    st = fill_f32(w, X->k, 0.0f, s);
    if (st) return st;
  }
  // start: z = Xw (FP64), FP32 state, objective, KKT
  CheckOut ck{};
  st = run_check(X, y, p->loss, p->lambda, w, su, true, s, &ck);
  if (st) return st;
  st = copy_f32(ws.w_ckpt, w, X->k, s);
  if (st) return st;
  double best = ck.objective;
  if (!std::isfinite(best)) return GENCD_ERR_DIVERGED;
  st_out->objective = ck.objective;
  st_out->kkt_max = ck.kkt;
  st_out->gap = ck.gap;
  st_out->nnz_w = ck.nnz_w;
  st_out->num_colors = int32_t(C);
  int status = GENCD_NOT_CONVERGED;
  if (converged(p, ck)) {
    status = GENCD_OK;
    st_out->converged = 1;
  }

  int64_t S;
  if (rule == GENCD_CYCLIC || rule == GENCD_STOCHASTIC) S = 1;
  else if (rule == GENCD_GREEDY) S = k_live;
  else if (p->select_size == 0) S = pstar_of(k_live, su.rho);
  else S = p->select_size;
  if (S > k_live) S = k_live;
  if (S < 1) S = 1;
  st_out->rho = su.rho;
  // Block Shotgun: windows of P_b* inside every block; T_blk windows per epoch
  int64_t T_blk = 0, max_pb = 0;
  if (rule == GENCD_BLOCK_SHOTGUN) {
    const int64_t nb = int64_t(su.bp.size());
    double rmax = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t kb = block_lo(b + 1, k_live, nb) - block_lo(b, k_live, nb);
      T_blk += (kb + su.bp[size_t(b)] - 1) / su.bp[size_t(b)];
      max_pb = std::max<int64_t>(max_pb, su.bp[size_t(b)]);
      rmax = std::max(rmax, su.brho[size_t(b)]);
    }
    S = std::max<int64_t>(max_pb, 1);
    st_out->rho = rmax;
  }
  st_out->select_size = S;
  const int64_t check_every = p->check_every;  // 0: adaptive (check_interval)
  int64_t next_check = check_interval(check_every, 0);
  int64_t max_class = 0;
  for (int32_t sz : cls_sizes) max_class = std::max<int64_t>(max_class, sz);
  int64_t *epoch_dev = reinterpret_cast<int64_t *>(ws.red + 12);
  st = fill_f64(ws.red + 12, 1, 0.0, s);  // epoch counter = 0
  if (st) return st;
  IterArgs a = base_args(X, y, p, su, w, ws.zs);
  unsigned long long acc_nnz_seen = 0, acc_cnt_seen = 0;
  // GENCD_PROFILE: one event pair per Propose launch between two checks
  const bool use_graph = (p->flags & GENCD_USE_GRAPH) != 0;
  const bool fused = (p->flags & GENCD_FUSED) != 0;
  const bool prof = (p->flags & GENCD_PROFILE) != 0 && !use_graph && !fused;
  EventPool pool;
  std::vector<hipEvent_t> &evs = pool.v;  // per iteration: Propose pair, Update pair
  size_t ev_used = 0;
  double prof_bytes_pending = 0.0, prof_ubytes_pending = 0.0;
  double lead_ticks_per_us = 0.0;  // device wall-clock ticks per microsecond
  if (prof) {
    a.scat = ws.scat;
    st = fill_i32(reinterpret_cast<int32_t *>(ws.scat), int64_t(kChkRep) * 32, 0, s);
    if (st) return st;
  }
  auto harvest = [&]() {
    // called after a stream synchronisation: every recorded pair is complete
    double ms = 0.0, ums = 0.0;
    for (size_t u = 0; u + 3 < ev_used; u += 4) {
      float t = 0.0f;
      if (evs[u] && evs[u + 1] && hipEventElapsedTime(&t, evs[u], evs[u + 1]) == hipSuccess)
        ms += double(t);
      t = 0.0f;
      if (evs[u + 2] && evs[u + 3] &&
          hipEventElapsedTime(&t, evs[u + 2], evs[u + 3]) == hipSuccess)
        ums += double(t);
    }
    st_out->prof_kernel_ms += ms;
    st_out->prof_launches += int64_t(ev_used / 4);
    st_out->prof_bytes += prof_bytes_pending;
    st_out->prof_update_ms += ums;
    st_out->prof_update_launches += int64_t(ev_used / 4);
    st_out->prof_update_bytes += prof_ubytes_pending;
    prof_bytes_pending = prof_ubytes_pending = 0.0;
    ev_used = 0;
  };
  GraphHolder graph;
  int64_t graph_S = -1;

  // Enqueue one epoch: selection order (section 2.1), then every iteration
  // of Algorithm 1, then the epoch counter increment.  Every argument is
  // independent of the epoch number, so the sequence can be captured once.
  auto enqueue_epoch = [&](int64_t T, int64_t e_host, bool record, hipStream_t es) -> int {
    int rc = rule == GENCD_BLOCK_SHOTGUN
                 ? launch_block_order(ws, k_live, p->seed, epoch_dev, T, es)
                 : launch_epoch_order(ws, k_live, rule, p->seed, epoch_dev, C, S, T, es);
    if (rc) return rc;
    PermKey cpk{};
    if (rule == GENCD_COLORING && !use_graph) cpk = make_perm_key(C, p->seed, e_host);
    for (int64_t t = 0; t < T; ++t) {
      int64_t positions;
      if (rule == GENCD_COLORING) {
        a.win_off = ws.win_off;
        positions = use_graph ? max_class : cls_sizes[size_t(perm_apply(cpk, uint64_t(t)))];
      } else if (rule == GENCD_BLOCK_SHOTGUN) {
        a.win_off = ws.win_off;  // windows of at most max_pb positions
        positions = max_pb;
      } else {
        a.win_off = nullptr;
        a.win_lo = int32_t(t * S);
        a.win_hi = int32_t(std::min(k_live, (t + 1) * S));
        positions = a.win_hi - a.win_lo;
      }
      if (positions == 0) continue;
      a.t = int32_t(t);
      if (fused) {
        // this window's pieces and the previous window's split pieces
        rc = launch_fused(a, su.group, positions, 2 * long_bound_for(su, positions), false, es);
        if (rc) return rc;
        continue;
      }
      const int64_t B = (rule == GENCD_THREAD_GREEDY) ? p->block : positions;
      a.rs = wants_rs(p, positions, X->nnz, k_live, X->n) ? ws.rs : nullptr;
      hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
      if (record && !evs.empty() && ev_used + 4 <= evs.size()) {
        e0 = evs[ev_used];
        e1 = evs[ev_used + 1];
        e2 = evs[ev_used + 2];
        e3 = evs[ev_used + 3];
        ev_used += 4;
      }
      rc = launch_iteration(a, su.group, mode, B, positions, long_bound_for(su, positions),
                            (positions + B - 1) / B, es, e0, e1, e2, e3);
      if (rc) return rc;
    }
    if (fused && T > 0) {  // the last window's split columns
      a.t = int32_t(T);
      const int64_t last = rule == GENCD_BLOCK_SHOTGUN ? max_pb : S;
      rc = launch_fused(a, su.group, 0, long_bound_for(su, last), true, es);
      if (rc) return rc;
    }
    if (mode != 1 && !a.exact_accum) {
      rc = launch_renorm(X->n, ws.zs, es);
      if (rc) return rc;
    }
    return launch_inc_epoch(epoch_dev, es);
  };

  for (int64_t e = 0; status != GENCD_OK && e < p->max_epochs && k_live > 0; ++e) {
    const int64_t T = (rule == GENCD_COLORING)         ? C
                      : (rule == GENCD_BLOCK_SHOTGUN) ? T_blk
                                                      : (k_live + S - 1) / S;
    if (prof && evs.empty()) {
      int rate_khz = 0;
      int dev = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess)
        lead_ticks_per_us = double(rate_khz) / 1000.0;
      const int64_t want = 4 * std::max<int64_t>(T, 1) * (check_every > 0 ? check_every : 64);
      if (want <= 4 * 65536) {
        evs.resize(size_t(want));
        // timing-only events: no system-scope fence when they complete, so
        // the stamped dispatch ends without a cache writeback of its own
        // (they are read only after the stream has been synchronised)
        for (auto &ev : evs)
          if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess) ev = nullptr;
      }
    }
    if (use_graph) {
      if (graph_S != S) {
        // capture on a private stream (the caller's may be the legacy
        // default stream, which cannot be captured); replay on the caller's
        graph.reset();
        if (!graph.cs) GENCD_HIP(hipStreamCreateWithFlags(&graph.cs, hipStreamNonBlocking));
        GENCD_HIP(hipStreamBeginCapture(graph.cs, hipStreamCaptureModeRelaxed));
        st = enqueue_epoch(T, e, false, graph.cs);
        hipGraph_t g = nullptr;
        hipError_t ce = hipStreamEndCapture(graph.cs, &g);
        if (st) {
          if (g) (void)hipGraphDestroy(g);
          return st;
        }
        if (ce != hipSuccess) return GENCD_ERR_HIP;
        graph.g = g;
        GENCD_HIP(hipGraphInstantiate(&graph.exec, g, nullptr, nullptr, 0));
        graph_S = S;
      }
      GENCD_HIP(hipGraphLaunch(graph.exec, s));
    } else {
      if (prof && lead_ticks_per_us > 0.0) {
        // about 15 us of host work per profiled iteration, at most 4 ms
        const double us = std::min(4000.0, 15.0 * double(std::max<int64_t>(T, 1)));
        hipLaunchKernelGGL(k_host_lead, dim3(1), dim3(64), 0, s, int64_t(us * lead_ticks_per_us),
                           int64_t(1) << 22);
      }
      st = enqueue_epoch(T, e, true, s);
      if (st) return st;
    }
    int64_t iters = T;
    if (rule == GENCD_COLORING) {
      iters = 0;
      for (int32_t sz : cls_sizes) iters += sz > 0;
    }
    st_out->iters += iters;
    if (mode != 2) st_out->coord_updates += k_live;
    st_out->epochs = e + 1;
    if (!evs.empty()) {
      prof_bytes_pending += 12.0 * double(X->nnz) + 28.0 * double(k_live);
      // accept-all rules: every live column is accepted once per epoch
      if (mode != 2) prof_ubytes_pending += 24.0 * double(X->nnz) + 8.0 * double(k_live);
    }
    st_out->nnz_visits += X->nnz;
    if (mode != 2) st_out->nnz_updates += X->nnz;
    if (e + 1 >= next_check || e + 1 == p->max_epochs) {
      next_check = e + 1 + check_interval(check_every, e + 1);
      st = run_check(X, y, p->loss, p->lambda, w, su, true, s, &ck);
      if (st) return st;
      if (std::isfinite(ck.drift_rel))
        st_out->z_drift = std::max(st_out->z_drift, ck.drift_rel);
      else
        st_out->z_drift = ck.drift_rel;
      if (mode == 2) {
        if (!evs.empty())
          prof_ubytes_pending += 24.0 * double(ck.acc_nnz - acc_nnz_seen) +
                                 8.0 * double(ck.acc_cnt - acc_cnt_seen);
        st_out->coord_updates += int64_t(ck.acc_cnt - acc_cnt_seen);
        st_out->nnz_updates += int64_t(ck.acc_nnz - acc_nnz_seen);
        acc_cnt_seen = ck.acc_cnt;
        acc_nnz_seen = ck.acc_nnz;
      }
      if (!evs.empty()) harvest();
      const bool bad = !std::isfinite(ck.objective) ||
                       ck.objective > best + 1e-3 * std::fabs(best) + 1e-12;
      if (bad &&
          (rule == GENCD_SHOTGUN || rule == GENCD_THREAD_GREEDY || rule == GENCD_TOP_GREEDY) &&
          S > 1) {
        // Divergence guard: restore the last checked point, halve |J|.
        st = copy_f32(w, ws.w_ckpt, X->k, s);
        if (st) return st;
        st = run_check(X, y, p->loss, p->lambda, w, su, true, s, &ck);
        if (st) return st;
        S = (S + 1) / 2;
        st_out->select_size = S;
        continue;
      }
      if (!std::isfinite(ck.objective)) return GENCD_ERR_DIVERGED;
      st_out->objective = ck.objective;
      st_out->kkt_max = ck.kkt;
      st_out->gap = ck.gap;
      st_out->nnz_w = ck.nnz_w;
      if (ck.objective <= best) {
        best = ck.objective;
        st = copy_f32(ws.w_ckpt, w, X->k, s);
        if (st) return st;
      }
      if (converged(p, ck)) {
        status = GENCD_OK;
        st_out->converged = 1;
      }
    }
  }
  if (k_live == 0 && converged(p, ck)) status = GENCD_OK;
  if (z) {
    st = launch_round_f32(ws.z64, z, X->n, s);
    if (st) return st;
  }
  if (prof) {
    unsigned long long sc[kChkRep * 16];
    GENCD_HIP(hipMemcpyAsync(sc, ws.scat, sizeof(sc), hipMemcpyDeviceToHost, s));
    GENCD_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < kChkRep; ++i) st_out->nnz_scattered += int64_t(sc[i * 16]);
  }
  GENCD_HIP(hipStreamSynchronize(s));
  st_out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return status;
}

// ---------------------------------------------------------------------------
// One step on a given J
// ---------------------------------------------------------------------------
int step_impl(const gencd_csc *X, const float *y, const gencd_params *p, const int32_t *J,
              int64_t nJ, float *w, float *z_hi, float *z_lo, float *g, float *delta, float *phi,
              int32_t *accepted, void *ws_base, size_t ws_bytes, hipStream_t s) {
  (void)hipGetLastError();  // launch checks below must not see an earlier error
  int st = params_ok(p, false);
  if (st) return st;
  if (p->rule < GENCD_CYCLIC || p->rule > GENCD_BLOCK_SHOTGUN) return GENCD_ERR_INVALID_ARG;
  if ((p->rule == GENCD_THREAD_GREEDY || p->rule == GENCD_TOP_GREEDY) && p->block <= 0)
    return GENCD_ERR_INVALID_ARG;
  if (!w || !z_hi || !z_lo || nJ < 0 || (nJ > 0 && !J)) return GENCD_ERR_INVALID_ARG;
  if (nJ > X->k) return GENCD_ERR_INVALID_ARG;
  Setup su;
  st = setup(X, y, p->loss, p, ws_base, ws_bytes, (p->flags & GENCD_VALIDATE_DEVICE) != 0, s, &su);
  if (st) return st;
  if (nJ == 0) return GENCD_OK;
  const Ws &ws = su.ws;
  {
    unsigned grid = unsigned(std::min<int64_t>((nJ + 255) / 256, 1024));
    hipLaunchKernelGGL(k_check_list, dim3(grid), dim3(256), 0, s, J, nJ, X->k,
                       reinterpret_cast<unsigned long long *>(ws.red) + 10);
    Red r{};
    st = read_red(ws, s, &r);
    if (st) return st;
    if (r.bad & 8ull) return GENCD_ERR_INVALID_ARG;
  }
  st = launch_list_order(ws, J, nJ, s);
  if (st) return st;
  const int mode = mode_of(p->rule);
  st = launch_pack_state(X->n, z_hi, z_lo, y, ws.zs, s);
  if (st) return st;
  IterArgs a = base_args(X, y, p, su, w, ws.zs);
  a.win_off = nullptr;
  a.win_lo = 0;
  a.win_hi = int32_t(nJ);
  a.t = 0;
  a.gout = g;
  const int64_t B = (p->rule == GENCD_THREAD_GREEDY) ? p->block : nJ;
  a.rs = wants_rs(p, nJ, X->nnz, su.k_live, X->n) ? su.ws.rs : nullptr;
  st = launch_iteration(a, su.group, mode, B, nJ, std::max<int64_t>(long_bound_for(su, nJ), 1),
                        (nJ + B - 1) / B, s);
  if (st) return st;
  st = launch_unpack_state(X->n, ws.zs, z_hi, z_lo, s);
  if (st) return st;
  if (delta) st = copy_f32(delta, ws.delta, nJ, s);
  if (st) return st;
  if (phi) st = copy_f32(phi, ws.phi, nJ, s);
  if (st) return st;
  if (accepted) st = (mode == 2) ? copy_i32(accepted, ws.acc, nJ, s) : fill_i32(accepted, nJ, 1, s);
  if (st) return st;
  GENCD_HIP(hipStreamSynchronize(s));
  return GENCD_OK;
}

int check_impl(const gencd_csc *X, const float *y, int loss, double lambda, const float *w,
               double *z64, double *g64, gencd_stats *stats, void *ws_base, size_t ws_bytes,
               hipStream_t s) {
  (void)hipGetLastError();  // launch checks below must not see an earlier error
  gencd_params p{};
  p.loss = loss;
  p.lambda = lambda;
  int st = params_ok(&p, false);
  if (st) return st;
  Setup su;
  st = setup(X, y, loss, &p, ws_base, ws_bytes, false, s, &su);
  if (st) return st;
  CheckOut ck{};
  st = run_check(X, y, loss, lambda, w, su, false, s, &ck);
  if (st) return st;
  if (z64) GENCD_HIP(hipMemcpyAsync(z64, su.ws.z64, sizeof(double) * X->n, hipMemcpyDeviceToDevice, s));
  if (g64) GENCD_HIP(hipMemcpyAsync(g64, su.ws.g64, sizeof(double) * X->k, hipMemcpyDeviceToDevice, s));
  GENCD_HIP(hipStreamSynchronize(s));
  if (stats) {
    stats->objective = ck.objective;
    stats->kkt_max = ck.kkt;
    stats->gap = ck.gap;
    stats->nnz_w = ck.nnz_w;
  }
  return GENCD_OK;
}

}  // namespace gencd

// ---------------------------------------------------------------------------
// Allocation-free solve.  Its workspace is this fixed device array: every
// device the library runs on holds one copy until the process ends, and
// every allocation-free call on that device shares it.
// ---------------------------------------------------------------------------
namespace gencd {
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxScratchDevices = 64;
}  // namespace gencd

static __device__ __align__(256) unsigned char scratch[gencd::kScratchBytes];

namespace gencd {
namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current) and kept.  The array's name is only
// a host-side stand-in, never a device address.
int scratch_ptr(void **out) {
  int dev = -1;
  GENCD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return GENCD_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GENCD_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GENCD_OK;
}
}  // namespace
}  // namespace gencd

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace gencd;

extern "C" {

const char *gencd_status_string(int status) {
  switch (status) {
    case GENCD_OK: return "ok";
    case GENCD_NOT_CONVERGED: return "not converged (max_epochs reached)";
    case GENCD_ERR_INVALID_ARG: return "invalid argument";
    case GENCD_ERR_BAD_MATRIX: return "invalid CSC matrix";
    case GENCD_ERR_BAD_LABELS: return "logistic labels must be -1 or +1";
    case GENCD_ERR_WORKSPACE: return "workspace missing or too small";
    case GENCD_ERR_UNSUPPORTED: return "unsupported option";
    case GENCD_ERR_DIVERGED: return "diverged (non-finite objective)";
    case GENCD_ERR_HIP: return "HIP runtime error";
    case GENCD_ERR_BUDGET: return "request exceeds the memory budget";
    case GENCD_ERR_TOO_LARGE: return "problem exceeds the static scratch of the allocation-free call";
    default: return "unknown status";
  }
}

int gencd_workspace_bytes(const gencd_csc *X, const gencd_params *p, size_t *out_bytes) {
  if (!out_bytes || !X || X->n <= 0 || X->k <= 0 || X->nnz < 0) return GENCD_ERR_INVALID_ARG;
  int piece, group;
  int st = resolve_schedule(p, &piece, &group);
  if (st) return st;
  *out_bytes = workspace_layout(X->n, X->k, X->nnz, piece, short_max_of(group), wants_rho(p),
                               blocks_of(p), nullptr, nullptr) +
               kAlign;
  return GENCD_OK;
}

int gencd_lambda_max(const gencd_csc *X, const float *y, int32_t loss, double *out, void *ws,
                     size_t ws_bytes, hipStream_t stream) {
  if (!out) return GENCD_ERR_INVALID_ARG;
  gencd_stats st{};
  int rc = check_impl(X, y, loss, 0.0, nullptr, nullptr, nullptr, &st, ws, ws_bytes, stream);
  if (rc) return rc;
  *out = st.kkt_max;
  return GENCD_OK;
}

int gencd_solve(const gencd_csc *X, const float *y, const gencd_params *p, float *w, float *z,
                void *ws, size_t ws_bytes, hipStream_t stream, gencd_stats *stats) {
  return solve_impl(X, y, p, w, z, ws, ws_bytes, stream, stats);
}

int gencd_solve_noalloc(const gencd_csc *X, const float *y, const gencd_params *p, float *w,
                        float *z, hipStream_t stream, gencd_stats *stats) {
  // host checks first: a problem that does not fit is rejected before any
  // HIP call
  if (!p || !w) return GENCD_ERR_INVALID_ARG;
  if (p->flags & (GENCD_USE_GRAPH | GENCD_PROFILE)) return GENCD_ERR_UNSUPPORTED;
  size_t need = 0;
  int st = gencd_workspace_bytes(X, p, &need);
  if (st) return st;
  if (need > kScratchBytes) return GENCD_ERR_TOO_LARGE;
  void *base = nullptr;
  st = scratch_ptr(&base);
  if (st) return st;
  return solve_impl(X, y, p, w, z, base, kScratchBytes, stream, stats);
}

int gencd_step(const gencd_csc *X, const float *y, const gencd_params *p, const int32_t *J,
               int64_t nJ, float *w, float *z_hi, float *z_lo, float *g, float *delta,
               float *phi, int32_t *accepted, void *ws, size_t ws_bytes, hipStream_t stream) {
  return step_impl(X, y, p, J, nJ, w, z_hi, z_lo, g, delta, phi, accepted, ws, ws_bytes, stream);
}

int gencd_check(const gencd_csc *X, const float *y, int32_t loss, double lambda, const float *w,
                double *z64, double *g64, gencd_stats *stats, void *ws, size_t ws_bytes,
                hipStream_t stream) {
  if (!w) return GENCD_ERR_INVALID_ARG;
  return check_impl(X, y, loss, lambda, w, z64, g64, stats, ws, ws_bytes, stream);
}

int gencd_rho_workspace_bytes(const gencd_csc *X, const gencd_params *p, size_t *out_bytes) {
  if (!out_bytes || !X || X->n <= 0 || X->k <= 0 || X->nnz < 0) return GENCD_ERR_INVALID_ARG;
  int piece, group;
  int st = resolve_schedule(p, &piece, &group);
  if (st) return st;
  *out_bytes = workspace_layout(X->n, X->k, X->nnz, piece, short_max_of(group), true, 0, nullptr,
                                nullptr) +
               kAlign;
  return GENCD_OK;
}

int gencd_estimate_rho(const gencd_csc *X, const gencd_params *p, int32_t iters, double *rho_hist,
                       int64_t *k_live, int64_t *select_size, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  (void)hipGetLastError();
  if (!rho_hist || iters < 1 || iters > kRhoMaxIters) return GENCD_ERR_INVALID_ARG;
  gencd_params q{};
  if (p) q = *p;
  q.loss = GENCD_SQUARED;  // no labels: nothing to validate
  Setup su;
  int st = setup(X, nullptr, GENCD_SQUARED, &q, ws, ws_bytes, (q.flags & GENCD_VALIDATE_DEVICE) != 0,
                 stream, &su, iters, false);
  if (st) return st;
  for (int32_t t = 0; t < iters; ++t) rho_hist[t] = su.rho_hist[size_t(t)];
  if (k_live) *k_live = su.k_live;
  if (select_size) *select_size = pstar_of(su.k_live, su.rho);
  return GENCD_OK;
}

int gencd_block_rho_workspace_bytes(const gencd_csc *X, const gencd_params *p, int64_t num_blocks,
                                    size_t *out_bytes) {
  if (!out_bytes || !X || X->n <= 0 || X->k <= 0 || X->nnz < 0 || num_blocks < 1 ||
      num_blocks > kMaxBlocks)
    return GENCD_ERR_INVALID_ARG;
  int piece, group;
  int st = resolve_schedule(p, &piece, &group);
  if (st) return st;
  *out_bytes = workspace_layout(X->n, X->k, X->nnz, piece, short_max_of(group), false, num_blocks,
                                nullptr, nullptr) +
               kAlign;
  return GENCD_OK;
}

int gencd_estimate_block_rho(const gencd_csc *X, const gencd_params *p, int64_t num_blocks,
                             int32_t iters, double *rho_out, int64_t *pstar_out, void *ws,
                             size_t ws_bytes, hipStream_t stream) {
  (void)hipGetLastError();
  if (!rho_out || !pstar_out || num_blocks < 1 || num_blocks > kMaxBlocks || iters < 1 ||
      iters > kBlockRhoMaxIters)
    return GENCD_ERR_INVALID_ARG;
  gencd_params q{};
  if (p) q = *p;
  q.loss = GENCD_SQUARED;  // no labels: nothing to validate
  Setup su;
  int st = setup(X, nullptr, GENCD_SQUARED, &q, ws, ws_bytes, (q.flags & GENCD_VALIDATE_DEVICE) != 0,
                 stream, &su, 0, false, num_blocks, iters);
  if (st) return st;
  if (num_blocks > su.k_live) return GENCD_ERR_INVALID_ARG;
  for (int64_t b = 0; b < num_blocks; ++b) {
    rho_out[b] = su.brho[size_t(b)];
    pstar_out[b] = su.bp[size_t(b)];
  }
  return GENCD_OK;
}

int gencd_select_perm(int64_t m, uint64_t seed, int64_t epoch, int32_t *out, hipStream_t stream) {
  if (m < 0 || m >= INT32_MAX || (m > 0 && !out)) return GENCD_ERR_INVALID_ARG;
  int st = launch_select_perm(m, seed, epoch, out, stream);
  if (st) return st;
  return hipStreamSynchronize(stream) == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

}  // extern "C"
