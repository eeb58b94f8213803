// Serving: continuous batching of factorization jobs on one device.
//
// A context holds one device allocation (the HBM budget), a table of slots
// (each with its own HIP stream at the default priority, a completion event
// and a pinned host copy of its job's round state) and a scheduler thread.
// The scheduler admits queued jobs in submission order whenever a slot is
// free and the job's workspace fits the unallocated part of the budget, keeps
// one batch of rounds in flight per active job (on the job's stream, so the
// rounds of different jobs overlap on the device), and retires a job as soon
// as its state says it is finished, which frees its slot and memory for the
// next one.  Each job runs the same host driver as arpc_factor (make_job), so
// its kernels, launch shapes and results are those of a factorization alone;
// one round of a job is recorded once as a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/arpc.h"
#include "arpc_common.h"
#include "arpc_host.h"

using namespace arpc;
using Clock = std::chrono::steady_clock;

namespace {

// First-fit allocator over [0, size) in 256-byte units.
class Pool {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size >= 256) free_[0] = size / 256 * 256;
  }
  // offset of a block of `bytes`, or SIZE_MAX
  size_t alloc(size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
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

 private:
  std::map<size_t, size_t> free_;  // offset -> size
};

enum JobState { QUEUED, ACTIVE, DONE };

struct ServedJob {
  arpc_job id = 0;
  arpc_problem p{};
  const double* X = nullptr;
  void* F = nullptr;
  int64_t* pivots = nullptr;
  Layout l{};
  JobState state = QUEUED;
  bool cancel = false;
  int slot = -1;
  size_t ws_off = 0;
  arpc_status result = ARPC_OK;
  arpc_stats stats{};
  Clock::time_point t_submit;
  std::unique_ptr<JobBase> run;
  std::unique_ptr<Profiler> prof;
};

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  RoundState* hstate = nullptr;  // pinned
  ServedJob* job = nullptr;
};

bool graphs_enabled() {
  const char* e = getenv("ARPC_SERVE_GRAPHS");
  return !(e && strcmp(e, "0") == 0);
}

}  // namespace

struct arpc_ctx_s {
  int device = 0;
  size_t budget = 0;
  char* base = nullptr;
  Pool pool;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<ServedJob*> queue;
  std::unordered_map<arpc_job, std::unique_ptr<ServedJob>> jobs;
  std::thread worker;
  bool stop = false;
  arpc_job next_id = 1;
  arpc_serving_stats info{};
  bool graphs = true;

  void run();
  void retire(ServedJob* j, arpc_status st, bool have_stats);  // with mu held
};

void arpc_ctx_s::retire(ServedJob* j, arpc_status st, bool have_stats) {
  j->result = st;
  if (!have_stats) std::memset(&j->stats, 0, sizeof(j->stats));
  j->stats.ms_total = std::chrono::duration<double, std::milli>(Clock::now() - j->t_submit).count();
  if (j->slot >= 0) {
    pool.release(j->ws_off, j->l.total);
    info.bytes_in_use -= (int64_t)((j->l.total + 255) / 256 * 256);
    slots[j->slot].job = nullptr;
    info.active -= 1;
    j->slot = -1;
  }
  j->run.reset();
  j->prof.reset();
  j->state = DONE;
  info.completed += 1;
  if (st == ARPC_ECANCELED) info.cancelled += 1;
  cv_done.notify_all();
}

void arpc_ctx_s::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool progress = false;
    // admission, in submission order
    for (;;) {
      if (stop || queue.empty()) break;
      int free_slot = -1;
      for (size_t i = 0; i < slots.size(); ++i)
        if (!slots[i].job) { free_slot = (int)i; break; }
      if (free_slot < 0) break;
      ServedJob* j = queue.front();
      const size_t off = pool.alloc(j->l.total);
      if (off == SIZE_MAX) break;
      queue.pop_front();
      info.queued -= 1;
      Slot& sl = slots[free_slot];
      j->slot = free_slot;
      j->ws_off = off;
      j->state = ACTIVE;
      sl.job = j;
      info.active += 1;
      info.bytes_in_use += (int64_t)((j->l.total + 255) / 256 * 256);
      if (info.active > info.peak_active) info.peak_active = info.active;
      if (info.bytes_in_use > info.peak_bytes) info.peak_bytes = info.bytes_in_use;
      progress = true;
      // start it (the lock is released around HIP calls that may take time)
      lk.unlock();
      Unif un{nullptr, 0, j->p.seed};
      j->prof.reset(new Profiler(sl.s, false));
      j->run = make_job(j->p, j->X, j->F, j->pivots, base + off, j->l, sl.s, un, sl.hstate, j->prof.get());
      std::memset(sl.hstate, 0, sizeof(RoundState));
      arpc_status e = j->run->begin();
      if (e == ARPC_OK && graphs) e = j->run->capture_round();
      if (e == ARPC_OK) e = j->run->enqueue_batch();
      if (e == ARPC_OK && hipEventRecord(sl.ev, sl.s) != hipSuccess) e = ARPC_EDEVICE;
      lk.lock();
      if (e != ARPC_OK) {
        (void)hipStreamSynchronize(sl.s);
        retire(j, e, false);
      }
    }
    // progress of the active jobs
    for (size_t i = 0; i < slots.size(); ++i) {
      Slot& sl = slots[i];
      ServedJob* j = sl.job;
      if (!j) continue;
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipErrorNotReady) continue;
      progress = true;
      if (q != hipSuccess) {
        retire(j, ARPC_EDEVICE, false);
        continue;
      }
      if (j->cancel) {
        retire(j, ARPC_ECANCELED, false);
        continue;
      }
      lk.unlock();
      arpc_status e = ARPC_OK;
      bool finished = false;
      arpc_stats st{};
      if (j->run->running()) {
        e = j->run->enqueue_batch();
        if (e == ARPC_OK && hipEventRecord(sl.ev, sl.s) != hipSuccess) e = ARPC_EDEVICE;
      } else {
        finished = true;
        e = j->run->finish(&st, 0.0);
      }
      lk.lock();
      if (finished) {
        j->stats = st;
        retire(j, e, true);
      } else if (e != ARPC_OK) {
        (void)hipStreamSynchronize(sl.s);
        retire(j, e, false);
      }
    }
    if (stop && info.active == 0) break;
    if (!progress) cv_work.wait_for(lk, std::chrono::microseconds(50));
  }
}

extern "C" {

arpc_status arpc_create(int device, size_t hbm_budget_bytes, int max_slots, arpc_ctx* out) {
  if (!out || max_slots < 1 || max_slots > 64 || hbm_budget_bytes < 4096) return ARPC_EINVAL;
  *out = nullptr;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return ARPC_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return ARPC_EDEVICE;
  std::unique_ptr<arpc_ctx_s> c(new arpc_ctx_s());
  c->device = device;
  c->budget = hbm_budget_bytes / 256 * 256;
  c->graphs = graphs_enabled();
  arpc_status ret = ARPC_OK;
  if (hipMalloc((void**)&c->base, c->budget) != hipSuccess) {
    c->base = nullptr;
    ret = ARPC_EDEVICE;
  }
  c->slots.resize((size_t)max_slots);
  for (auto& sl : c->slots) {
    if (ret != ARPC_OK) break;
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&sl.hstate, sizeof(RoundState), hipHostMallocDefault) != hipSuccess)
      ret = ARPC_EDEVICE;
  }
  if (ret != ARPC_OK) {
    for (auto& sl : c->slots) {
      if (sl.s) (void)hipStreamDestroy(sl.s);
      if (sl.ev) (void)hipEventDestroy(sl.ev);
      if (sl.hstate) (void)hipHostFree(sl.hstate);
    }
    if (c->base) (void)hipFree(c->base);
    (void)hipSetDevice(prev);
    return ret;
  }
  c->pool.reset(c->budget);
  c->info.budget_bytes = (int64_t)c->budget;
  c->info.slots = max_slots;
  arpc_ctx_s* raw = c.get();
  c->worker = std::thread([raw] { raw->run(); });
  (void)hipSetDevice(prev);
  *out = c.release();
  return ARPC_OK;
}

arpc_status arpc_destroy(arpc_ctx ctx) {
  if (!ctx) return ARPC_EINVAL;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stop = true;
    while (!ctx->queue.empty()) {
      ServedJob* j = ctx->queue.front();
      ctx->queue.pop_front();
      ctx->info.queued -= 1;
      ctx->retire(j, ARPC_ECANCELED, false);
    }
    for (auto& sl : ctx->slots)
      if (sl.job) sl.job->cancel = true;
  }
  ctx->cv_work.notify_all();
  ctx->worker.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  for (auto& sl : ctx->slots) {
    (void)hipStreamSynchronize(sl.s);
    (void)hipStreamDestroy(sl.s);
    (void)hipEventDestroy(sl.ev);
    (void)hipHostFree(sl.hstate);
  }
  (void)hipFree(ctx->base);
  (void)hipSetDevice(prev);
  delete ctx;
  return ARPC_OK;
}

arpc_status arpc_submit(arpc_ctx ctx, const arpc_problem* problem, const double* X, void* F, int64_t* pivots,
                        arpc_job* job) {
  if (!ctx || !job) return ARPC_EINVAL;
  const arpc_status v = check_factor_args(problem, X, F, pivots);
  if (v != ARPC_OK) return v;
  std::unique_ptr<ServedJob> j(new ServedJob());
  j->p = *problem;
  j->X = X;
  j->F = F;
  j->pivots = pivots;
  j->l = layout_of(*problem);
  if (j->l.ncbt > 0) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    j->l.grid = fused_grid();
    (void)hipSetDevice(prev);
  }
  if (j->l.total > ctx->budget) return ARPC_ENOMEM;
  j->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->stop) return ARPC_ECANCELED;
    j->id = ctx->next_id++;
    *job = j->id;
    ctx->queue.push_back(j.get());
    ctx->jobs.emplace(j->id, std::move(j));
    ctx->info.submitted += 1;
    ctx->info.queued += 1;
  }
  ctx->cv_work.notify_all();
  return ARPC_OK;
}

arpc_status arpc_poll(arpc_ctx ctx, arpc_job job, int* done, arpc_stats* stats) {
  if (!ctx || !done) return ARPC_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->jobs.find(job);
  if (it == ctx->jobs.end()) return ARPC_EINVAL;
  ServedJob* j = it->second.get();
  if (j->state != DONE) {
    *done = 0;
    return ARPC_OK;
  }
  *done = 1;
  if (stats) *stats = j->stats;
  const arpc_status r = j->result;
  ctx->jobs.erase(it);
  return r;
}

arpc_status arpc_wait(arpc_ctx ctx, arpc_job job, arpc_stats* stats) {
  if (!ctx) return ARPC_EINVAL;
  std::unique_lock<std::mutex> lk(ctx->mu);
  auto it = ctx->jobs.find(job);
  if (it == ctx->jobs.end()) return ARPC_EINVAL;
  ServedJob* j = it->second.get();
  ctx->cv_done.wait(lk, [j] { return j->state == DONE; });
  if (stats) *stats = j->stats;
  const arpc_status r = j->result;
  ctx->jobs.erase(job);
  return r;
}

arpc_status arpc_cancel(arpc_ctx ctx, arpc_job job) {
  if (!ctx) return ARPC_EINVAL;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->jobs.find(job);
    if (it == ctx->jobs.end()) return ARPC_EINVAL;
    ServedJob* j = it->second.get();
    if (j->state == QUEUED) {
      for (auto q = ctx->queue.begin(); q != ctx->queue.end(); ++q)
        if (*q == j) {
          ctx->queue.erase(q);
          break;
        }
      ctx->info.queued -= 1;
      ctx->retire(j, ARPC_ECANCELED, false);
    } else if (j->state == ACTIVE) {
      j->cancel = true;
    }
  }
  ctx->cv_work.notify_all();
  return ARPC_OK;
}

arpc_status arpc_serving_info(arpc_ctx ctx, arpc_serving_stats* out) {
  if (!ctx || !out) return ARPC_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  *out = ctx->info;
  return ARPC_OK;
}

}  // extern "C"
