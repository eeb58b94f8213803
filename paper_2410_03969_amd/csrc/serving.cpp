// Serving: continuous batching of factorization jobs on one device.
//
// A context holds one device allocation (the HBM budget), a table of slots
// and a scheduler thread.  The scheduler admits queued jobs in submission
// order whenever a slot is free and the job's workspace fits the unallocated
// part of the budget, and retires a job as soon as it is finished, which
// frees its slot and memory for the next one.  Each job is driven by the same
// host code as arpc_factor (make_job), so its kernels and results are those
// of a factorization alone.  Jobs advance in one of two ways:
//  - Ticks (the BF16 modes with the one-kernel round product: d <= 16 and
//    b <= 256, or one product with d <= 32 and b <= 208).  Every such job's table row
//    (RoundJob) goes into a device table, and one tick advances all of them
//    by one round with one launch per round step (the round product once per
//    group of jobs with the same compiled shape), on the context's tick
//    stream.  A tick ends by copying every row's round state to pinned host
//    memory; up to two ticks are in flight, so the device never waits for
//    the host between rounds.  A finished job leaves the table; its final
//    reductions are enqueued behind the ticks and it is retired when they
//    complete.
//  - Rounds on the job's own slot stream (every other job): batches of
//    rounds, recorded once as a HIP graph and replayed, as in arpc_factor,
//    overlapping with the ticks and with other slots.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <algorithm>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/arpc.h"
#include "arpc_common.h"
#include "arpc_host.h"
#include "arpc_launch.h"
#include "arpc_mfma.h"

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
  bool ticked = false;     // advanced by ticks (else on its slot stream)
  bool finishing = false;  // ticks: final reductions enqueued, waiting for the slot event
  RoundState last{};       // ticks: round state after the latest completed tick
};

struct Slot {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  RoundState* hstate = nullptr;  // pinned
  double* htrace = nullptr;      // pinned: residual trace of a ticked job
  ServedJob* job = nullptr;
};

// Jobs that ticks can advance: the one-kernel round product of the BF16 modes
// with the library's uniform stream.
bool tickable(const arpc_problem& p, const Layout& l) {
  return l.ncbt > 0 && (p.prec == ARPC_BF16 || p.prec == ARPC_BF16X3);
}

constexpr int kTicks = 2;   // ticks in flight

struct Tick {
  hipEvent_t ev = nullptr;
  RoundJob* htab = nullptr;     // pinned copy of the table (read by the copy at run time)
  RoundJob* dtab = nullptr;     // device table
  RoundState* hst = nullptr;    // pinned: states after the tick
  std::vector<ServedJob*> jobs;
  bool inflight = false;
};

bool ticks_enabled() {
  const char* e = getenv("ARPC_SERVE_TICKS");
  return !(e && strcmp(e, "0") == 0);
}

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
  bool use_ticks = true;
  int64_t max_outstanding = 65536;   // submitted and not yet finished
  hipStream_t ts = nullptr;     // tick stream
  Tick ticks[kTicks];
  int next_tick = 0;            // tick buffer of the next launch
  int oldest = 0;               // oldest tick in flight
  int grid2 = 0;                // two workgroups per compute unit
  RoundJob* dtab_base = nullptr;

  void run();
  void retire(ServedJob* j, arpc_status st, bool have_stats);  // with mu held
  bool launch_tick();                                          // without mu
  void complete_tick(Tick& t);                                 // with mu held
  void free_resources();                                       // after the scheduler has stopped
};

void arpc_ctx_s::free_resources() {
  if (ts) (void)hipStreamSynchronize(ts);
  for (auto& sl : slots) {
    if (sl.s) {
      (void)hipStreamSynchronize(sl.s);
      (void)hipStreamDestroy(sl.s);
    }
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.hstate) (void)hipHostFree(sl.hstate);
    if (sl.htrace) (void)hipHostFree(sl.htrace);
    sl = Slot{};
  }
  for (auto& tk : ticks) {
    if (tk.ev) (void)hipEventDestroy(tk.ev);
    if (tk.htab) (void)hipHostFree(tk.htab);
    if (tk.hst) (void)hipHostFree(tk.hst);
    tk = Tick{};
  }
  if (ts) (void)hipStreamDestroy(ts);
  ts = nullptr;
  if (dtab_base) (void)hipFree(dtab_base);
  dtab_base = nullptr;
  if (base) (void)hipFree(base);
  base = nullptr;
}

// One round of every ticked job that is still running, as one launch per
// round step over the device table (rows grouped by compiled shape for the
// round product), then the rows' round states into pinned memory.
bool arpc_ctx_s::launch_tick() {
  Tick& t = ticks[next_tick];
  const int n = (int)t.jobs.size();
  if (n == 0) return false;
  // group by (mode, column blocks, coordinate class, kernel form)
  auto key = [](ServedJob* j) {
    const RoundJob& r = j->run->row();
    return std::make_tuple(j->p.prec, j->l.ncbt, r.d <= 8 ? 8 : (r.d <= 16 ? 16 : 32), r.fa.kf.use_r);
  };
  std::stable_sort(t.jobs.begin(), t.jobs.end(), [&](ServedJob* a, ServedJob* b) { return key(a) < key(b); });
  RoundGrid g{};
  int bmax = 1;
  for (int i = 0; i < n; ++i) {
    t.htab[i] = t.jobs[i]->run->row();
    round_grid_max(g, round_grid_of(t.htab[i]));
    if (t.htab[i].b > bmax) bmax = t.htab[i].b;
  }
  hipStream_t s = ts;
  if (hipMemcpyAsync(t.dtab, t.htab, sizeof(RoundJob) * (size_t)n, hipMemcpyHostToDevice, s) != hipSuccess)
    return false;
  launch_propose_tab(s, t.dtab, n, g);
  launch_gather_tab(s, t.dtab, n, g, false, false);
  launch_reject_tab(s, t.dtab, n, bmax);
  for (int i0 = 0; i0 < n;) {   // per mode: the inverse factor, F(S_r,:)^T chunks, accepted points
    int i1 = i0, ncbt = 0;
    int64_t bd = 1;
    while (i1 < n && t.jobs[i1]->p.prec == t.jobs[i0]->p.prec) {
      ncbt = std::max(ncbt, t.jobs[i1]->l.ncbt);
      bd = std::max(bd, (int64_t)t.htab[i1].b * t.htab[i1].d);
      ++i1;
    }
    launch_fused_prep_tab(s, gemm_prec(t.jobs[i0]->p.prec), t.dtab + i0, i1 - i0, ncbt, bd);
    i0 = i1;
  }
  for (int i0 = 0; i0 < n;) {   // per compiled shape: the round product
    int i1 = i0, tiles = 1;
    while (i1 < n && key(t.jobs[i1]) == key(t.jobs[i0])) {
      tiles = std::max(tiles, t.htab[i1].fa.ntiles);
      ++i1;
    }
    const int prec = gemm_prec(t.jobs[i0]->p.prec);
    FusedArgs any = t.htab[i0].fa;
    any.ntiles = 1 << 30;
    const int budget = fused_grid_of(prec, any, grid2);   // persistent workgroups of a lone job
    const int per = std::max(1, (budget + (i1 - i0) - 1) / (i1 - i0));
    launch_fused_round_tab(s, prec, t.jobs[i0]->l.ncbt, t.htab[i0].d, t.htab[i0].fa, t.dtab + i0, i1 - i0,
                           std::min(per, tiles));
    i0 = i1;
  }
  launch_diag_tab(s, t.dtab, n, g);
  launch_finish_tab(s, t.dtab, n);
  launch_collect_tab(s, t.dtab, n, t.hst);
  if (hipGetLastError() != hipSuccess || hipEventRecord(t.ev, s) != hipSuccess) return false;
  t.inflight = true;
  next_tick = (next_tick + 1) % kTicks;
  return true;
}

// A tick has completed: the states of its rows are in t.hst.  A job that is
// no longer running (or was cancelled) leaves the ticks: its final
// reductions go on the tick stream, behind every tick already launched.
void arpc_ctx_s::complete_tick(Tick& t) {
  for (size_t i = 0; i < t.jobs.size(); ++i) {
    ServedJob* j = t.jobs[i];
    if (j->finishing || j->state != ACTIVE) continue;
    j->last = t.hst[i];
    if (j->last.status == ST_RUNNING && !j->cancel) continue;
    Slot& sl = slots[j->slot];
    j->finishing = true;
    arpc_status e = ARPC_OK;
    if (!j->cancel) e = j->run->finish_enqueue(j->last, sl.htrace);
    if (e == ARPC_OK && hipEventRecord(sl.ev, ts) != hipSuccess) e = ARPC_EDEVICE;
    if (e != ARPC_OK) {
      (void)hipStreamSynchronize(ts);
      retire(j, e, false);
    }
  }
  t.jobs.clear();
  t.inflight = false;
}

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
      j->ticked = use_ticks && tickable(j->p, j->l);
      if (j->ticked) info.ticked_jobs += 1;
      sl.job = j;
      info.active += 1;
      info.bytes_in_use += (int64_t)((j->l.total + 255) / 256 * 256);
      if (info.active > info.peak_active) info.peak_active = info.active;
      if (info.bytes_in_use > info.peak_bytes) info.peak_bytes = info.bytes_in_use;
      progress = true;
      // start it (the lock is released around HIP calls that may take time)
      lk.unlock();
      Unif un{nullptr, 0, j->p.seed};
      hipStream_t js = j->ticked ? ts : sl.s;
      j->prof.reset(new Profiler(js, false));
      j->run = make_job(j->p, j->X, j->F, j->pivots, base + off, j->l, js, un, sl.hstate, j->prof.get());
      std::memset(sl.hstate, 0, sizeof(RoundState));
      arpc_status e = j->run->begin();
      if (!j->ticked) {
        if (e == ARPC_OK && graphs) e = j->run->capture_round();
        if (e == ARPC_OK) e = j->run->enqueue_batch();
        if (e == ARPC_OK && hipEventRecord(sl.ev, sl.s) != hipSuccess) e = ARPC_EDEVICE;
      }
      lk.lock();
      if (e != ARPC_OK) {
        (void)hipStreamSynchronize(js);
        retire(j, e, false);
      }
    }
    // jobs on their own slot streams, and ticked jobs whose final reductions were enqueued
    for (size_t i = 0; i < slots.size(); ++i) {
      Slot& sl = slots[i];
      ServedJob* j = sl.job;
      if (!j || (j->ticked && !j->finishing)) continue;
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipErrorNotReady) continue;
      progress = true;
      if (q != hipSuccess) {
        retire(j, ARPC_EDEVICE, false);
        continue;
      }
      if (j->ticked) {
        arpc_stats st{};
        const arpc_status e = j->cancel ? ARPC_ECANCELED : j->run->finish_stats(j->last, *sl.htrace, &st);
        j->stats = st;
        retire(j, e, !j->cancel);
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
    // ticks: completions in launch order, then a new tick while fewer than
    // kTicks are in flight and some ticked job is still running
    while (ticks[oldest].inflight) {
      const hipError_t q = hipEventQuery(ticks[oldest].ev);
      if (q == hipErrorNotReady) break;
      progress = true;
      if (q != hipSuccess) {
        for (ServedJob* j : ticks[oldest].jobs)
          if (j->state == ACTIVE) retire(j, ARPC_EDEVICE, false);
        ticks[oldest].jobs.clear();
        ticks[oldest].inflight = false;
      } else {
        complete_tick(ticks[oldest]);
      }
      oldest = (oldest + 1) % kTicks;
    }
    if (!ticks[next_tick].inflight) {
      Tick& t = ticks[next_tick];
      t.jobs.clear();
      for (auto& sl : slots)
        if (sl.job && sl.job->ticked && !sl.job->finishing && (sl.job->last.status == ST_RUNNING) && !sl.job->cancel)
          t.jobs.push_back(sl.job);
      // a cancelled ticked job that is not in flight leaves now
      for (auto& sl : slots) {
        ServedJob* j = sl.job;
        if (!j || !j->ticked || j->finishing || !j->cancel) continue;
        bool inflight = false;
        for (auto& tk : ticks)
          if (tk.inflight && std::find(tk.jobs.begin(), tk.jobs.end(), j) != tk.jobs.end()) inflight = true;
        if (inflight) continue;
        j->finishing = true;
        if (hipEventRecord(sl.ev, ts) != hipSuccess) retire(j, ARPC_EDEVICE, false);
        progress = true;
      }
      if (!t.jobs.empty()) {
        lk.unlock();
        const bool ok = launch_tick();
        lk.lock();
        progress = true;
        if (ok) info.ticks += 1;
        if (!ok) {
          (void)hipStreamSynchronize(ts);
          for (ServedJob* j : t.jobs)
            if (j->state == ACTIVE) retire(j, ARPC_EDEVICE, false);
          t.jobs.clear();
          t.inflight = false;
        }
      }
    }
    if (stop && info.active == 0) break;
    if (!progress) cv_work.wait_for(lk, std::chrono::microseconds(20));
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
  c->use_ticks = ticks_enabled();
  c->grid2 = fused_grid();
  arpc_status ret = ARPC_OK;
  if (hipMalloc((void**)&c->base, c->budget) != hipSuccess) {
    c->base = nullptr;
    ret = ARPC_EDEVICE;
  }
  if (ret == ARPC_OK &&
      (hipMalloc((void**)&c->dtab_base, sizeof(RoundJob) * (size_t)max_slots * kTicks) != hipSuccess ||
       hipStreamCreateWithFlags(&c->ts, hipStreamNonBlocking) != hipSuccess))
    ret = ARPC_EDEVICE;
  for (int t = 0; t < kTicks && ret == ARPC_OK; ++t) {
    Tick& tk = c->ticks[t];
    tk.dtab = c->dtab_base + (size_t)t * max_slots;
    if (hipEventCreateWithFlags(&tk.ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&tk.htab, sizeof(RoundJob) * (size_t)max_slots, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&tk.hst, sizeof(RoundState) * (size_t)max_slots, hipHostMallocDefault) != hipSuccess)
      ret = ARPC_EDEVICE;
  }
  c->slots.resize((size_t)max_slots);
  for (auto& sl : c->slots) {
    if (ret != ARPC_OK) break;
    if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&sl.hstate, sizeof(RoundState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.htrace, sizeof(double), hipHostMallocDefault) != hipSuccess)
      ret = ARPC_EDEVICE;
  }
  if (ret != ARPC_OK) {
    c->free_resources();
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
  ctx->free_resources();
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
    if (ctx->info.queued + ctx->info.active >= ctx->max_outstanding) return ARPC_EBUSY;
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

arpc_status arpc_serving_set_limit(arpc_ctx ctx, int64_t max_outstanding) {
  if (!ctx || max_outstanding < 1 || max_outstanding > 2147483647LL) return ARPC_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->max_outstanding = max_outstanding;
  return ARPC_OK;
}

arpc_status arpc_serving_info(arpc_ctx ctx, arpc_serving_stats* out) {
  if (!ctx || !out) return ARPC_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  *out = ctx->info;
  return ARPC_OK;
}

}  // extern "C"
