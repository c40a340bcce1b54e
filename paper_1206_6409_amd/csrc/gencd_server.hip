// Continuous-batching solve server.
//
// Requests are Shotgun solves of Eq. (1) (section 4.1; each request has its
// own matrix, labels, loss, lambda and |J|, or |J| = P* from the spectral
// radius).  They are admitted in arrival order whenever a slot is free and
// their state fits in the caller-owned device arena.  Admitted requests
// advance together: every round is ONE Propose launch and ONE Update launch
// over a device work table of (request slot, window position range) items,
// so a single dispatch carries one Jacobi iteration (Algorithm 2 / 4, then
// Algorithm 3) of every admitted request.  A request's state (w, packed
// z_hi/z_lo/y, curvature, epoch order, FP64 check arrays) stays resident in
// the arena from admission to retirement.
//
// Threads.  An admission thread prepares requests on a stream of its own
// (preprocessing, |J| from the power iteration, the initial FP64 check and
// the first epoch order) while rounds run; a driver thread launches the
// rounds on the caller's stream and, at each request's epoch end, enqueues
// its FP64 check (z = Xw re-sync, objective, KKT) with an asynchronous
// read-back, so no round waits for the host.  A request whose check meets
// its tolerance is retired: its checked iterate (kept at check time) is
// copied back to the caller's w (and Xw to z), its arena range is freed and
// the next waiting request is admitted.
//
// The admission policy (Admission) is plain host logic with no HIP calls; it
// also backs gencd_server_plan, a discrete-event replay of the policy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "gencd_common.hpp"
#include "gencd_kernels.hpp"
#include "gencd_solver.hpp"

namespace gencd {

// First-fit range allocator over [0, size).
class Arena {
 public:
  explicit Arena(size_t size = 0) : size_(size) {
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t roff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }

 private:
  size_t size_;
  size_t used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Waiting {
  int64_t ticket;
  size_t bytes;
};

// FIFO admission by free slots and arena space (head-of-line: a request that
// does not fit yet blocks the ones behind it, so large requests are never
// starved).
class Admission {
 public:
  Admission(size_t arena_bytes, int max_slots) : arena_(arena_bytes), max_slots_(max_slots) {}
  bool fits_ever(size_t bytes) const { return (bytes + 255) / 256 * 256 <= arena_.size(); }
  void enqueue(int64_t ticket, size_t bytes) { queue_.push_back({ticket, bytes}); }
  // the head request, if a slot is free and it fits
  bool pump_one(int64_t *ticket, size_t *off) {
    if (queue_.empty() || busy_ >= max_slots_) return false;
    if (!arena_.alloc(queue_.front().bytes, off)) return false;
    *ticket = queue_.front().ticket;
    queue_.pop_front();
    ++busy_;
    return true;
  }
  // admitted (ticket, offset) pairs, in order
  std::vector<std::pair<int64_t, size_t>> pump() {
    std::vector<std::pair<int64_t, size_t>> out;
    while (!queue_.empty() && busy_ < max_slots_) {
      size_t off;
      if (!arena_.alloc(queue_.front().bytes, &off)) break;
      out.push_back({queue_.front().ticket, off});
      queue_.pop_front();
      ++busy_;
    }
    return out;
  }
  void finish(size_t off, size_t bytes) {
    arena_.release(off, bytes);
    --busy_;
  }
  int busy() const { return busy_; }
  size_t waiting() const { return queue_.size(); }
  size_t used() const { return arena_.used(); }

 private:
  Arena arena_;
  int max_slots_;
  int busy_ = 0;
  std::deque<Waiting> queue_;
};

// ---------------------------------------------------------------------------
// Multi-request round kernels
// ---------------------------------------------------------------------------

// One admitted request as the round kernels see it.
struct MpSlot {
  const int64_t *col_ptr;
  const int32_t *row_idx;
  const float *val;
  const float *c;          // curvature beta ||X_j||^2 / n
  float *w;                // the caller's weights (the live iterate)
  float4 *zs;              // {z_hi, z_lo, y, 0} per row
  const int32_t *col_of_pos;  // current epoch order of the live columns
  float *delta;            // increments of the current window
  int64_t r0;              // round at which the slot's epoch 0 started
  int64_t T;               // windows per epoch
  float lam, n_f;
  int32_t loss, G;         // G: lanes per column (4..64, from the mean column length)
  int32_t S, k_live;       // |J| and the live column count
  int32_t fused, pad_;     // fused: Propose scatters each step at once (GENCD_FUSED)
};

// Work item (one wave): slot, window-relative positions [lo, hi).  A wave
// takes one batch of 64 / G columns, so a round's dependence chain is one
// column long; a slot gets more positions per item only when its window
// would exceed its share of the item table.
constexpr int kMpRoundsPerItem = 1;
constexpr int32_t kMpMaxItems = 262144;  // work items of one round (4 MiB table)

// Round r of every slot: window t = (r - r0) mod T of its epoch order.
// Propose (UPD = false) writes delta and w_j += delta_j; Update (UPD = true)
// scatters delta_j x_ij into the low words z_lo (non-returning atomics; the
// FP64 check at the epoch end re-syncs the pair).  A fused slot
// (GENCD_FUSED, section 4.1) scatters each column's step in its Propose
// launch, as soon as the group has it, and leaves delta at zero, so the
// Update launch passes over it; its columns read z while others of the
// window update it.
template <bool UPD>
__global__ __launch_bounds__(kBlock) void k_mp_round(const MpSlot *slots, const int4 *items,
                                                     int32_t nitems, int64_t round) {
  const int64_t wid = int64_t(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
  if (wid >= nitems) return;  // whole waves: no barrier in this kernel
  const int lane = int(threadIdx.x) & (kWave - 1);
  const int4 it = items[wid];
  const MpSlot &sl = slots[it.x];
  if (UPD && sl.fused) return;  // its steps were scattered by Propose
  const int64_t t = (round - sl.r0) % sl.T;
  const int32_t P0 = int32_t(t * sl.S);
  const int32_t P1 = min(P0 + sl.S, sl.k_live);
  const int G = sl.G, per = kWave / G, gl = lane & (G - 1);
  const int32_t hi = min(P0 + it.z, P1);
  for (int32_t p = P0 + it.y + lane / G; p < hi; p += per) {
    const int32_t j = sl.col_of_pos[p];
    const int64_t b = sl.col_ptr[j];
    const int32_t len = int32_t(sl.col_ptr[j + 1] - b);
    int32_t ri[kUnroll];
    float vv[kUnroll];
    if constexpr (!UPD) {
      const float wj = sl.w[j], cj = sl.c[j];
      float s = 0.0f;
      for (int32_t base = 0; base < len; base += G * kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int32_t e = base + u * G + gl;
          ri[u] = e < len ? sl.row_idx[b + e] : -1;
          vv[u] = e < len ? sl.val[b + e] : 0.0f;
        }
        float4 zr[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) zr[u] = sl.zs[ri[u] >= 0 ? ri[u] : 0];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (ri[u] >= 0) s += vv[u] * dloss_f32(sl.loss, zr[u].z, zr[u].x + zr[u].y);
      }
      // butterfly: every lane of the group holds the same sum, hence the same step
      for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, kWave);
      float d, ph;
      propose_f32(s / sl.n_f, cj, wj, sl.lam, d, ph);
      if (gl == 0) {
        sl.delta[p - P0] = sl.fused ? 0.0f : d;
        if (d != 0.0f) sl.w[j] = wj + d;
      }
      if (!sl.fused || d == 0.0f) continue;
      if (len <= G * kUnroll) {  // the only batch is still in registers
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (ri[u] >= 0) atomicAdd(&sl.zs[ri[u]].y, d * vv[u]);
        continue;
      }
      for (int32_t base = 0; base < len; base += G * kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int32_t e = base + u * G + gl;
          ri[u] = e < len ? sl.row_idx[b + e] : -1;
          vv[u] = e < len ? sl.val[b + e] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (ri[u] >= 0) atomicAdd(&sl.zs[ri[u]].y, d * vv[u]);
      }
    } else {
      const float d = sl.delta[p - P0];
      if (d == 0.0f) continue;
      for (int32_t base = 0; base < len; base += G * kUnroll) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int32_t e = base + u * G + gl;
          ri[u] = e < len ? sl.row_idx[b + e] : -1;
          vv[u] = e < len ? sl.val[b + e] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (ri[u] >= 0) atomicAdd(&sl.zs[ri[u]].y, d * vv[u]);
      }
    }
  }
}

// Epoch order of one slot: position p holds live column live[pi_e(p)], the
// same keyed Feistel permutation (section 2.1's random subsets) as the
// single-problem solve.
__global__ __launch_bounds__(kBlock) void k_mp_order(const int32_t *live, int64_t k_live, PermKey pk,
                                                     int32_t *col_of_pos) {
  for (int64_t p = int64_t(blockIdx.x) * kBlock + threadIdx.x; p < k_live;
       p += int64_t(gridDim.x) * kBlock)
    col_of_pos[p] = live[perm_apply(pk, uint64_t(p))];
}

static unsigned grid_of(int64_t m, unsigned cap = 4096) {
  int64_t b = (m + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return unsigned(b);
}

static int enqueue_order(const Setup &su, uint64_t seed, int64_t epoch, hipStream_t s) {
  if (su.k_live <= 0) return GENCD_OK;
  const PermKey pk = make_perm_key(su.k_live, seed, epoch);
  hipLaunchKernelGGL(k_mp_order, dim3(grid_of(su.k_live)), dim3(kBlock), 0, s, su.ws.live,
                     su.k_live, pk, su.ws.col_of_pos);
  return hipGetLastError() == hipSuccess ? GENCD_OK : GENCD_ERR_HIP;
}

// Lanes per column from the mean column length: about 4 entries per lane.
static int32_t group_for(int64_t nnz, int64_t k_live) {
  const double mean = k_live > 0 ? double(nnz) / double(k_live) : 1.0;
  int32_t g = 4;
  while (g < kWave && double(g) * kUnroll < mean) g *= 2;
  return g;
}

// Extra arena bytes per request beyond the single-solve workspace: the best
// checked iterate (divergence guard).
static size_t slot_extra(int64_t k) { return (size_t(k) * sizeof(float) + 511) / 256 * 256; }

}  // namespace gencd

using namespace gencd;

struct gencd_server {
  int device = 0;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  int max_slots = 0;
  hipStream_t stream = nullptr;      // rounds (the caller's)
  hipStream_t adm_stream = nullptr;  // admission work
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_adm, cv_drv, cv_done;
  Admission adm{0, 0};

  enum State { FREE, ADMITTING, ACTIVE };
  struct Slot {
    State state = FREE;
    int64_t ticket = -1;
    gencd_request req{};
    size_t off = 0, bytes = 0;
    Setup su;
    float *w_best = nullptr;
    MpSlot dev{};
    int64_t S = 1, T = 1, epoch = 0, in_epoch = 0, next_check = 1;
    double best = 0.0;
    bool check_pending = false;
    bool retiring = false;
    hipEvent_t ev_check = nullptr, ev_final = nullptr;
    double *h_rep = nullptr;  // pinned: kChkRep * 16 replica words, then the Red block
    gencd_result res{};
  };
  std::vector<Slot> slots;
  std::map<int64_t, gencd_server::Slot> pending_req;  // submitted, not admitted (req + times)
  std::deque<int> ready;                 // slots set up by the admission thread
  std::deque<gencd_result> results;      // finished, not yet polled
  int64_t next_ticket = 0, in_flight = 0;
  bool stop = false;
  std::thread adm_thread, drv_thread;
  // device tables of the driver, filled from a ring of pinned host stages
  MpSlot *d_slots = nullptr;
  int4 *d_items = nullptr;
  int32_t max_items = 0, cur_items = 0;
  struct Stage {
    MpSlot *slots = nullptr;
    int4 *items = nullptr;
    hipEvent_t ev = nullptr;
  };
  std::vector<Stage> stage;
  std::vector<hipEvent_t> ev_round;
  int64_t rounds = 0, slot_rounds = 0, shared_rounds = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void admission_loop();
  void driver_loop();
  void publish(Slot &sl, int status);
  void release() {  // HIP objects and pinned buffers (threads already joined)
    for (auto &e : ev_round)
      if (e) (void)hipEventDestroy(e);
    for (auto &sg : stage) {
      if (sg.ev) (void)hipEventDestroy(sg.ev);
      if (sg.slots) (void)hipHostFree(sg.slots);
      if (sg.items) (void)hipHostFree(sg.items);
    }
    for (auto &sl : slots) {
      if (sl.ev_check) (void)hipEventDestroy(sl.ev_check);
      if (sl.ev_final) (void)hipEventDestroy(sl.ev_final);
      if (sl.h_rep) (void)hipHostFree(sl.h_rep);
    }
    if (adm_stream) (void)hipStreamDestroy(adm_stream);
  }
};

namespace {
void stats_from_check(gencd_stats &st, const CheckOut &ck) {
  st.objective = ck.objective;
  st.kkt_max = ck.kkt;
  st.gap = ck.gap;
  st.nnz_w = ck.nnz_w;
}
bool conv_of(const gencd_params &p, const CheckOut &ck) {
  if (!(ck.kkt <= p.kkt_tol)) return false;
  return p.gap_tol <= 0.0 || ck.gap <= p.gap_tol * std::fabs(ck.objective);
}
}  // namespace

// Result of a finished slot to the results queue (caller holds mu).
void gencd_server::publish(Slot &sl, int status) {
  sl.res.ticket = sl.ticket;
  sl.res.user_tag = sl.req.user_tag;
  sl.res.status = status;
  sl.res.finish_s = now();
  sl.res.stats.seconds = sl.res.finish_s - sl.res.start_s;
  results.push_back(sl.res);
  adm.finish(sl.off, sl.bytes);
  sl.state = FREE;
  sl.retiring = false;
  sl.check_pending = false;
  --in_flight;
  cv_adm.notify_all();
  cv_done.notify_all();
}

// Admission: waiting requests into free slots, each prepared on the
// admission stream while rounds of the others run.
void gencd_server::admission_loop() {
  (void)hipSetDevice(device);
  for (;;) {
    int si = -1;
    int64_t ticket = -1;
    size_t off = 0;
    {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        if (stop) return;
        if (adm.pump_one(&ticket, &off)) break;
        cv_adm.wait(lk);
      }
      for (int i = 0; i < max_slots; ++i)
        if (slots[size_t(i)].state == FREE) {
          si = i;
          break;
        }
      Slot &sl = slots[size_t(si)];
      Slot &pr = pending_req[ticket];
      sl.state = ADMITTING;
      sl.ticket = ticket;
      sl.req = pr.req;
      sl.bytes = pr.bytes;
      sl.off = off;
      sl.res = gencd_result{};
      sl.res.submit_s = pr.res.submit_s;
      sl.res.start_s = now();
      pending_req.erase(ticket);
    }
    Slot &sl = slots[size_t(si)];
    const gencd_params &p = sl.req.params;
    const gencd_csc *X = &sl.req.X;
    hipStream_t s = adm_stream;
    char *base = arena + sl.off;
    const size_t ws_bytes = sl.bytes - slot_extra(X->k);
    sl.w_best = reinterpret_cast<float *>(base + ws_bytes);
    sl.su = Setup{};
    int st = setup(X, sl.req.y, p.loss, &p, base, ws_bytes, (p.flags & GENCD_VALIDATE_DEVICE) != 0,
                   s, &sl.su, wants_rho(&p) ? kRhoIters : 0);
    CheckOut ck{};
    if (!st && !(p.flags & GENCD_WARM_START)) st = fill_f32(sl.req.w, X->k, 0.0f, s);
    if (!st) st = run_check(X, sl.req.y, p.loss, p.lambda, sl.req.w, sl.su, true, s, &ck);
    if (!st && !std::isfinite(ck.objective)) st = GENCD_ERR_DIVERGED;
    int64_t S = 1;
    if (!st) {
      S = p.select_size > 0 ? p.select_size : pstar_of(sl.su.k_live, sl.su.rho);
      S = std::max<int64_t>(1, std::min<int64_t>(S, std::max<int64_t>(sl.su.k_live, 1)));
      sl.res.stats.rho = sl.su.rho;
      sl.res.stats.select_size = S;
      stats_from_check(sl.res.stats, ck);
    }
    const bool done_now = !st && (conv_of(p, ck) || sl.su.k_live == 0 || p.max_epochs == 0);
    if (!st && !done_now) {
      st = copy_f32(sl.w_best, sl.req.w, X->k, s);
      if (!st) st = copy_f32(sl.su.ws.w_ckpt, sl.req.w, X->k, s);
      if (!st) st = enqueue_order(sl.su, p.seed, 0, s);
    }
    if (!st && done_now && sl.req.z) st = launch_round_f32(sl.su.ws.z64, sl.req.z, X->n, s);
    if (hipStreamSynchronize(s) != hipSuccess && !st) st = GENCD_ERR_HIP;
    std::lock_guard<std::mutex> lk(mu);
    if (st || done_now) {
      sl.res.stats.converged = (!st && conv_of(p, ck)) ? 1 : 0;
      publish(sl, st ? st : (sl.res.stats.converged ? GENCD_OK : GENCD_NOT_CONVERGED));
      continue;
    }
    sl.S = S;
    sl.T = (sl.su.k_live + S - 1) / S;
    sl.next_check = check_interval(p.check_every, 0);
    sl.epoch = 0;
    sl.in_epoch = 0;
    sl.best = ck.objective;
    ready.push_back(si);
    cv_drv.notify_all();
  }
}

// Driver: rounds on the caller's stream, epoch-end checks, retirements.
void gencd_server::driver_loop() {
  (void)hipSetDevice(device);
  std::vector<int> active;  // slots in the current work table
  int fail = GENCD_OK;
  bool dirty = false;
  bool all_fused = false;  // every slot of the work table is fused: no Update launch
  const int Q = int(ev_round.size());
  int stage_next = 0;

  // Fold slot si's finished check read-back and act on it: keep going,
  // restart from the best iterate with half the window (divergence guard),
  // or retire (converged, out of epochs, diverged).
  enum { KEEP, RESTARTED, RETIRED };
  auto process_check = [&](int si) -> int {
    Slot &sl = slots[size_t(si)];
    sl.check_pending = false;
    CheckOut ck{};
    Red red{};
    std::memcpy(&red, sl.h_rep + kChkRep * 16, sizeof(Red));
    fold_check(sl.h_rep, red, sl.req.X.n, sl.req.params.lambda, &ck);
    const gencd_params &p = sl.req.params;
    gencd_stats &so = sl.res.stats;
    so.z_drift = std::isfinite(ck.drift_rel) ? std::max(so.z_drift, ck.drift_rel) : ck.drift_rel;
    const bool bad = !std::isfinite(ck.objective) ||
                     ck.objective > sl.best + 1e-3 * std::fabs(sl.best) + 1e-12;
    const int64_t k = sl.req.X.k;
    if (bad && sl.S > 1) {
      // back to the best checked iterate with half the window
      fail = copy_f32(sl.req.w, sl.w_best, k, stream);
      if (!fail)
        fail = launch_check(&sl.req.X, sl.req.y, p.loss, p.lambda, sl.req.w, sl.su.n_short,
                            sl.su.n_lpieces, sl.su.ws, true, stream);
      if (!fail) fail = copy_f32(sl.su.ws.w_ckpt, sl.req.w, k, stream);
      if (!fail) fail = enqueue_order(sl.su, p.seed, sl.epoch, stream);
      sl.S = (sl.S + 1) / 2;
      sl.T = (sl.su.k_live + sl.S - 1) / sl.S;
      sl.in_epoch = 0;
      sl.dev.r0 = rounds;
      so.select_size = sl.S;
      dirty = true;
      return RESTARTED;
    }
    bool retire = false;
    if (!std::isfinite(ck.objective)) {
      sl.res.status = GENCD_ERR_DIVERGED;
      retire = true;
    } else {
      stats_from_check(so, ck);
      if (ck.objective <= sl.best) {
        sl.best = ck.objective;
        if (!fail) fail = copy_f32(sl.w_best, sl.su.ws.w_ckpt, k, stream);
      }
      const bool conv = conv_of(p, ck);
      if (conv || so.epochs >= p.max_epochs) {
        so.converged = conv ? 1 : 0;
        sl.res.status = conv ? GENCD_OK : GENCD_NOT_CONVERGED;
        retire = true;
      }
    }
    if (!retire) return KEEP;
    // the checked iterate (w_ckpt) and its FP64 product z64 go back to the caller
    // once the rounds already enqueued have run
    if (!fail) fail = copy_f32(sl.req.w, sl.su.ws.w_ckpt, k, stream);
    if (!fail && sl.req.z) fail = launch_round_f32(sl.su.ws.z64, sl.req.z, sl.req.X.n, stream);
    if (hipEventRecord(sl.ev_final, stream) != hipSuccess && !fail) fail = GENCD_ERR_HIP;
    sl.retiring = true;
    dirty = true;
    return RETIRED;
  };

  for (;;) {
    // 1. newly prepared slots; stop when asked and idle
    {
      std::unique_lock<std::mutex> lk(mu);
      bool retiring = false;
      for (auto &sl : slots) retiring |= sl.retiring;
      if (active.empty() && !retiring) {
        cv_drv.wait(lk, [&] { return stop || !ready.empty(); });
        if (stop && ready.empty()) return;
      }
      while (!ready.empty()) {
        const int si = ready.front();
        ready.pop_front();
        Slot &sl = slots[size_t(si)];
        sl.state = ACTIVE;
        sl.dev.r0 = rounds;  // its epoch 0 starts with the next round
        active.push_back(si);
        dirty = true;
      }
    }
    // 2. finished read-backs; results of retired slots once their copies ran
    for (size_t a = 0; a < active.size();) {
      Slot &sl = slots[size_t(active[a])];
      if (sl.check_pending && hipEventQuery(sl.ev_check) == hipSuccess &&
          process_check(active[a]) == RETIRED) {
        active.erase(active.begin() + long(a));
        continue;
      }
      ++a;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      for (auto &sl : slots)
        if (sl.retiring && hipEventQuery(sl.ev_final) == hipSuccess) publish(sl, sl.res.status);
    }
    if (fail) {
      // a HIP call failed: every admitted request ends with that status
      (void)hipStreamSynchronize(stream);
      std::lock_guard<std::mutex> lk(mu);
      for (int si : active) publish(slots[size_t(si)], fail);
      for (auto &sl : slots)
        if (sl.retiring) publish(sl, fail);
      active.clear();
      fail = GENCD_OK;
      continue;
    }
    if (active.empty()) {
      std::this_thread::sleep_for(std::chrono::microseconds(50));
      continue;
    }
    // 3. the work table, after a change of the slot set or of a window size
    if (dirty) {
      Stage &sg = stage[size_t(stage_next)];
      stage_next = (stage_next + 1) % int(stage.size());
      (void)hipEventSynchronize(sg.ev);  // its previous upload has been consumed
      int32_t nitems = 0;
      const int32_t budget = std::max<int32_t>(1, max_items / max_slots);
      all_fused = true;
      for (int si : active) {
        Slot &sl = slots[size_t(si)];
        const Ws &w = sl.su.ws;
        MpSlot &d = sl.dev;
        d.col_ptr = sl.req.X.col_ptr;
        d.row_idx = sl.req.X.row_idx;
        d.val = sl.req.X.val;
        d.c = w.c;
        d.w = sl.req.w;
        d.zs = w.zs;
        d.col_of_pos = w.col_of_pos;
        d.delta = w.delta;
        d.T = sl.T;
        d.lam = float(sl.req.params.lambda);
        d.n_f = float(sl.req.X.n);
        d.loss = sl.req.params.loss;
        d.G = group_for(sl.req.X.nnz, sl.su.k_live);
        d.S = int32_t(sl.S);
        d.k_live = int32_t(sl.su.k_live);
        d.fused = (sl.req.params.flags & GENCD_FUSED) ? 1 : 0;
        d.pad_ = 0;
        all_fused = all_fused && d.fused;
        sg.slots[si] = d;
        int32_t span = (kWave / d.G) * kMpRoundsPerItem;
        const int32_t need = (d.S + budget - 1) / budget;  // at most `budget` items per slot
        if (span < need) span = need;
        for (int32_t lo = 0; lo < d.S; lo += span)
          sg.items[nitems++] = make_int4(si, lo, std::min<int32_t>(lo + span, d.S), 0);
      }
      if (hipMemcpyAsync(d_slots, sg.slots, sizeof(MpSlot) * size_t(max_slots),
                         hipMemcpyHostToDevice, stream) != hipSuccess ||
          hipMemcpyAsync(d_items, sg.items, sizeof(int4) * size_t(nitems), hipMemcpyHostToDevice,
                         stream) != hipSuccess ||
          hipEventRecord(sg.ev, stream) != hipSuccess) {
        fail = GENCD_ERR_HIP;
        continue;
      }
      cur_items = nitems;
      dirty = false;
    }
    // 4. one round: every active slot advances one window, one launch each
    //    for Propose and Update; at most Q rounds are in flight
    if (rounds >= Q) (void)hipEventSynchronize(ev_round[size_t(rounds % Q)]);
    const unsigned grid = unsigned((cur_items + (kBlock / kWave) - 1) / (kBlock / kWave));
    hipLaunchKernelGGL(k_mp_round<false>, dim3(grid), dim3(kBlock), 0, stream, d_slots, d_items,
                       cur_items, rounds);
    if (!all_fused)  // fused slots scattered their steps in the Propose launch
      hipLaunchKernelGGL(k_mp_round<true>, dim3(grid), dim3(kBlock), 0, stream, d_slots, d_items,
                         cur_items, rounds);
    if (hipGetLastError() != hipSuccess || hipEventRecord(ev_round[size_t(rounds % Q)], stream) != hipSuccess) {
      fail = GENCD_ERR_HIP;
      continue;
    }
    ++rounds;
    slot_rounds += int64_t(active.size());
    shared_rounds += active.size() > 1 ? 1 : 0;
    // 5. epoch ends: fold the previous check first, then the FP64 check of
    //    this epoch (z re-sync) with its read-back, and the next order
    for (size_t a = 0; a < active.size();) {
      const int si = active[a];
      Slot &sl = slots[size_t(si)];
      if (++sl.in_epoch < sl.T) {
        ++a;
        continue;
      }
      sl.in_epoch = 0;
      if (sl.check_pending) {
        (void)hipEventSynchronize(sl.ev_check);
        const int r = process_check(si);
        if (r == RETIRED) {
          active.erase(active.begin() + long(a));
          continue;
        }
        if (r == RESTARTED) {  // the epoch starts over from the best iterate
          ++a;
          continue;
        }
      }
      const gencd_params &p = sl.req.params;
      gencd_stats &so = sl.res.stats;
      so.epochs += 1;
      so.iters += sl.T;
      so.coord_updates += sl.su.k_live;
      so.nnz_visits += sl.req.X.nnz;
      so.nnz_updates += sl.req.X.nnz;
      ++sl.epoch;
      if (sl.epoch >= sl.next_check || sl.epoch >= p.max_epochs) {
        sl.next_check = sl.epoch + check_interval(p.check_every, sl.epoch);
        Red *red = reinterpret_cast<Red *>(sl.h_rep + kChkRep * 16);
        if (!fail)
          fail = enqueue_check(&sl.req.X, sl.req.y, p.loss, p.lambda, sl.req.w, sl.su, true,
                               stream, sl.h_rep, red);
        if (!fail) fail = copy_f32(sl.su.ws.w_ckpt, sl.req.w, sl.req.X.k, stream);
        if (!fail && hipEventRecord(sl.ev_check, stream) != hipSuccess) fail = GENCD_ERR_HIP;
        sl.check_pending = true;
      } else if (!fail) {
        fail = launch_renorm(sl.req.X.n, sl.su.ws.zs, stream);
      }
      if (!fail) fail = enqueue_order(sl.su, p.seed, sl.epoch, stream);
      ++a;
    }
  }
}

extern "C" {

int gencd_server_create(void *arena, size_t arena_bytes, int32_t max_slots, hipStream_t stream,
                        gencd_server **out) {
  if (!out || !arena || arena_bytes == 0 || max_slots <= 0 || max_slots > 256)
    return GENCD_ERR_INVALID_ARG;
  gencd_server *sv = new (std::nothrow) gencd_server();
  if (!sv) return GENCD_ERR_INVALID_ARG;
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return GENCD_ERR_HIP;
  }
  // align the usable arena; the driver's two small tables sit at its end
  char *base = static_cast<char *>(arena);
  size_t mis = reinterpret_cast<uintptr_t>(base) % 256;
  size_t skip = mis ? 256 - mis : 0;
  const size_t tab_bytes = (sizeof(MpSlot) * size_t(max_slots) + 255) / 256 * 256;
  const int32_t max_items = kMpMaxItems;  // each slot gets a share of the table;
                                          // gencd_server_overhead_bytes counts it
  const size_t item_bytes = sizeof(int4) * size_t(max_items);
  if (arena_bytes <= skip + tab_bytes + item_bytes + 256) {
    delete sv;
    return GENCD_ERR_BUDGET;
  }
  base += skip;
  arena_bytes -= skip;
  sv->d_slots = reinterpret_cast<MpSlot *>(base + arena_bytes - tab_bytes - item_bytes);
  sv->d_items = reinterpret_cast<int4 *>(base + arena_bytes - item_bytes);
  sv->max_items = max_items;
  arena_bytes -= tab_bytes + item_bytes;
  arena_bytes = arena_bytes / 256 * 256;
  sv->arena = base;
  sv->arena_bytes = arena_bytes;
  sv->max_slots = max_slots;
  sv->stream = stream;
  sv->t0 = std::chrono::steady_clock::now();
  sv->adm = Admission(arena_bytes, max_slots);
  sv->slots.resize(size_t(max_slots));
  bool ok = hipStreamCreateWithFlags(&sv->adm_stream, hipStreamNonBlocking) == hipSuccess;
  sv->ev_round.assign(8, nullptr);
  for (auto &e : sv->ev_round)
    ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  sv->stage.resize(4);
  for (auto &sg : sv->stage) {
    void *a = nullptr, *b = nullptr;
    ok = ok && hipHostMalloc(&a, sizeof(MpSlot) * size_t(max_slots), hipHostMallocDefault) == hipSuccess;
    sg.slots = static_cast<MpSlot *>(a);
    ok = ok && hipHostMalloc(&b, item_bytes, hipHostMallocDefault) == hipSuccess;
    sg.items = static_cast<int4 *>(b);
    ok = ok && hipEventCreateWithFlags(&sg.ev, hipEventDisableTiming) == hipSuccess;
    if (sg.slots) std::memset(static_cast<void *>(sg.slots), 0, sizeof(MpSlot) * size_t(max_slots));
  }
  for (auto &sl : sv->slots) {
    ok = ok && hipEventCreateWithFlags(&sl.ev_check, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&sl.ev_final, hipEventDisableTiming) == hipSuccess;
    void *h = nullptr;
    ok = ok && hipHostMalloc(&h, sizeof(double) * (kChkRep * 16 + 16), hipHostMallocDefault) ==
                   hipSuccess;
    sl.h_rep = static_cast<double *>(h);
  }
  if (!ok) {
    sv->release();
    delete sv;
    return GENCD_ERR_HIP;
  }
  sv->adm_thread = std::thread([sv] { sv->admission_loop(); });
  sv->drv_thread = std::thread([sv] { sv->driver_loop(); });
  *out = sv;
  return GENCD_OK;
}

int gencd_server_request_bytes(const gencd_csc *X, const gencd_params *p, size_t *out_bytes) {
  if (!X || !p || !out_bytes) return GENCD_ERR_INVALID_ARG;
  size_t bytes = 0;
  const int st = gencd_workspace_bytes(X, p, &bytes);
  if (st) return st;
  *out_bytes = (bytes + slot_extra(X->k) + 255) / 256 * 256;
  return GENCD_OK;
}

size_t gencd_server_overhead_bytes(int32_t max_slots) {
  const size_t tab = (sizeof(MpSlot) * size_t(max_slots > 0 ? max_slots : 1) + 255) / 256 * 256;
  return tab + sizeof(int4) * size_t(kMpMaxItems) + 512;
}

int gencd_server_submit(gencd_server *sv, const gencd_request *req, int64_t *ticket) {
  if (!sv || !req || !ticket) return GENCD_ERR_INVALID_ARG;
  const gencd_params &p = req->params;
  int st = params_ok(&p, true);
  if (st) return st;
  if (!req->w || !req->y || !csc_ok(&req->X)) return GENCD_ERR_INVALID_ARG;
  if (p.rule != GENCD_SHOTGUN || p.improve_steps != 0 ||
      (p.flags & (GENCD_EXACT_ACCUM | GENCD_PROFILE | GENCD_FUSED_EPOCH)))
    return GENCD_ERR_UNSUPPORTED;
  size_t bytes = 0;
  st = gencd_workspace_bytes(&req->X, &p, &bytes);
  if (st) return st;
  bytes += slot_extra(req->X.k);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (!sv->adm.fits_ever(bytes)) return GENCD_ERR_BUDGET;
  const int64_t t = sv->next_ticket++;
  gencd_server::Slot &pr = sv->pending_req[t];
  pr.req = *req;
  pr.bytes = bytes;
  pr.res.submit_s = sv->now();
  ++sv->in_flight;
  sv->adm.enqueue(t, bytes);
  sv->cv_adm.notify_all();
  *ticket = t;
  return GENCD_OK;
}

int gencd_server_poll(gencd_server *sv, gencd_result *out, int32_t max, int32_t wait_for,
                      int32_t *n_out) {
  if (!sv || !n_out || max < 0 || (max > 0 && !out)) return GENCD_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (wait_for > 0) {
    const size_t want = size_t(std::min<int64_t>(wait_for, int64_t(sv->results.size()) + sv->in_flight));
    sv->cv_done.wait(lk, [&] { return sv->results.size() >= want; });
  }
  int32_t n = 0;
  while (n < max && !sv->results.empty()) {
    out[n++] = sv->results.front();
    sv->results.pop_front();
  }
  *n_out = n;
  return GENCD_OK;
}

int gencd_server_info(gencd_server *sv, gencd_server_status *out) {
  if (!sv || !out) return GENCD_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  out->running = sv->adm.busy();
  out->waiting = int32_t(sv->adm.waiting());
  out->finished_unpolled = int32_t(sv->results.size());
  out->arena_used = sv->adm.used();
  out->arena_bytes = sv->arena_bytes;
  out->rounds = sv->rounds;
  out->slot_rounds = sv->slot_rounds;
  out->shared_rounds = sv->shared_rounds;
  return GENCD_OK;
}

int gencd_server_destroy(gencd_server *sv) {
  if (!sv) return GENCD_ERR_INVALID_ARG;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->in_flight == 0; });
    sv->stop = true;
  }
  sv->cv_adm.notify_all();
  sv->cv_drv.notify_all();
  sv->adm_thread.join();
  sv->drv_thread.join();
  (void)hipStreamSynchronize(sv->stream);
  sv->release();
  delete sv;
  return GENCD_OK;
}

// Discrete-event replay of the admission policy: requests arrive at
// arrival[i] needing bytes[i] of arena and holding a slot for service[i]
// seconds.  Returns the start time of every request (or -1 if it can never
// fit: the live server rejects those with GENCD_ERR_BUDGET).
int gencd_server_plan(size_t arena_bytes, int32_t max_slots, int32_t n, const size_t *bytes,
                      const double *arrival, const double *service, double *start) {
  if (max_slots <= 0 || n < 0 || (n > 0 && (!bytes || !arrival || !service || !start)))
    return GENCD_ERR_INVALID_ARG;
  for (int32_t i = 1; i < n; ++i)
    if (arrival[i] < arrival[i - 1]) return GENCD_ERR_INVALID_ARG;
  Admission adm(arena_bytes, max_slots);
  struct Running {
    double end;
    int32_t i;
    size_t off;
  };
  std::vector<Running> run;
  int32_t next = 0;
  double t = 0.0;
  for (int32_t i = 0; i < n; ++i) start[i] = -1.0;
  while (next < n || !run.empty() || adm.waiting() > 0) {
    // next event: an arrival or a completion
    double t_arr = next < n ? arrival[next] : 1e300;
    double t_end = 1e300;
    size_t ri = 0;
    for (size_t r = 0; r < run.size(); ++r)
      if (run[r].end < t_end) {
        t_end = run[r].end;
        ri = r;
      }
    if (t_arr == 1e300 && t_end == 1e300) break;  // waiting requests that can never start
    if (t_end <= t_arr) {
      t = t_end;
      adm.finish(run[ri].off, bytes[run[ri].i]);
      run.erase(run.begin() + long(ri));
    } else {
      t = t_arr;
      if (adm.fits_ever(bytes[next])) adm.enqueue(next, bytes[next]);
      ++next;
    }
    for (auto &a : adm.pump()) {
      const int32_t i = int32_t(a.first);
      start[i] = t;
      run.push_back({t + service[i], i, a.second});
    }
  }
  return GENCD_OK;
}

}  // extern "C"
