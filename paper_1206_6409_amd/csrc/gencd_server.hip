// Continuous-batching solve server.
//
// Requests (Eq. (1) problems of any shape, each with its own loss, lambda
// and rule) are admitted in arrival order whenever a slot is free and their
// workspace fits in the caller-owned device arena (first-fit sub-allocation,
// 256-byte aligned).  Each admitted request runs gencd_solve on a worker
// thread with its own HIP stream, so solves of different requests overlap on
// the device while their state (w, z, residual, workspace) stays resident in
// the arena.  Finished requests free their slot and arena range and the next
// waiting requests are admitted at once.
//
// The admission policy (Admission) is plain host logic with no HIP calls; it
// also backs gencd_server_plan, a discrete-event replay of the policy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/gencd.h"

namespace gencd {

int solve_impl(const gencd_csc *X, const float *y, const gencd_params *p, float *w, float *z,
               void *ws_base, size_t ws_bytes, hipStream_t s, gencd_stats *stats);

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

}  // namespace gencd

using namespace gencd;

struct gencd_server {
  int device = 0;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  int max_slots = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  Admission adm{0, 0};
  struct Job {
    gencd_request req;
    size_t bytes = 0, off = 0;
    double submit_s = 0, start_s = 0;
  };
  std::map<int64_t, Job> jobs;        // submitted, not yet finished
  std::deque<int64_t> ready;          // admitted, waiting for a worker
  std::deque<gencd_result> results;   // finished, not yet polled
  std::vector<std::thread> workers;
  int64_t next_ticket = 0;
  bool stop = false;
  int64_t in_flight = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void admit_locked() {
    for (auto &a : adm.pump()) {
      jobs[a.first].off = a.second;
      ready.push_back(a.first);
    }
    cv_work.notify_all();
  }
  void worker_loop() {
    (void)hipSetDevice(device);
    hipStream_t s = nullptr;
    const bool have_stream = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
      int64_t ticket;
      Job job;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || !ready.empty(); });
        if (ready.empty()) break;  // stop requested and nothing left
        ticket = ready.front();
        ready.pop_front();
        jobs[ticket].start_s = now();
        job = jobs[ticket];
      }
      gencd_result res{};
      res.ticket = ticket;
      res.user_tag = job.req.user_tag;
      if (!have_stream) {
        res.status = GENCD_ERR_HIP;
      } else {
        res.status = solve_impl(&job.req.X, job.req.y, &job.req.params, job.req.w, job.req.z,
                                arena + job.off, job.bytes, s, &res.stats);
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        res.submit_s = job.submit_s;
        res.start_s = jobs[ticket].start_s;
        res.finish_s = now();
        results.push_back(res);
        adm.finish(job.off, job.bytes);
        jobs.erase(ticket);
        --in_flight;
        admit_locked();
      }
      cv_done.notify_all();
    }
    if (have_stream) (void)hipStreamDestroy(s);
  }
};

extern "C" {

int gencd_server_create(void *arena, size_t arena_bytes, int32_t max_slots, gencd_server **out) {
  if (!out || !arena || arena_bytes == 0 || max_slots <= 0 || max_slots > 256)
    return GENCD_ERR_INVALID_ARG;
  gencd_server *sv = new (std::nothrow) gencd_server();
  if (!sv) return GENCD_ERR_INVALID_ARG;
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return GENCD_ERR_HIP;
  }
  // align the usable arena
  char *base = static_cast<char *>(arena);
  size_t mis = reinterpret_cast<uintptr_t>(base) % 256;
  if (mis) {
    if (arena_bytes <= 256 - mis) {
      delete sv;
      return GENCD_ERR_INVALID_ARG;
    }
    arena_bytes -= 256 - mis;
    base += 256 - mis;
  }
  sv->arena = base;
  sv->arena_bytes = arena_bytes;
  sv->max_slots = max_slots;
  sv->t0 = std::chrono::steady_clock::now();
  sv->adm = Admission(arena_bytes, max_slots);
  for (int i = 0; i < max_slots; ++i) sv->workers.emplace_back([sv] { sv->worker_loop(); });
  *out = sv;
  return GENCD_OK;
}

int gencd_server_submit(gencd_server *sv, const gencd_request *req, int64_t *ticket) {
  if (!sv || !req || !ticket) return GENCD_ERR_INVALID_ARG;
  size_t bytes = 0;
  int st = gencd_workspace_bytes(&req->X, &req->params, &bytes);
  if (st) return st;
  if (!req->w || !req->y) return GENCD_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (!sv->adm.fits_ever(bytes)) return GENCD_ERR_BUDGET;
  const int64_t t = sv->next_ticket++;
  gencd_server::Job job;
  job.req = *req;
  job.bytes = bytes;
  job.submit_s = sv->now();
  sv->jobs[t] = job;
  ++sv->in_flight;
  sv->adm.enqueue(t, bytes);
  sv->admit_locked();
  *ticket = t;
  return GENCD_OK;
}

int gencd_server_poll(gencd_server *sv, gencd_result *out, int32_t max, int32_t wait_for,
                      int32_t *n_out) {
  if (!sv || !n_out || max < 0 || (max > 0 && !out)) return GENCD_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (wait_for > 0) {
    const size_t want = size_t(std::min<int64_t>(wait_for, sv->results.size() + sv->in_flight));
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
  return GENCD_OK;
}

int gencd_server_destroy(gencd_server *sv) {
  if (!sv) return GENCD_ERR_INVALID_ARG;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->in_flight == 0; });
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (auto &t : sv->workers) t.join();
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
  std::vector<size_t> off_of(size_t(n), 0);
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
