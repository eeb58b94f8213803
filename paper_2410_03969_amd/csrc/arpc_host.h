// Host-side types shared by the factorization entry points and the
// serving scheduler (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <memory>
#include <vector>

#include "../../include/arpc.h"
#include "arpc_common.h"
#include "arpc_launch.h"

namespace arpc {

// Byte offset of the residual trace inside the round state's slot of the
// workspace; the round history follows that slot at the next 256-byte boundary.
constexpr size_t kTraceOff = 128;

// Offsets of the buffers carved from one factorization's workspace.
struct Layout {
  size_t st, jd, u, csum, cpre, props, acc, hist, Fs, Fs32, Hp, H, Xp, Bt, Bt2, Bm1, Bm2, Fb, C, C0, P, Xq, X8, xn8, Xp8,
      ypn, trace, total;
  bool dist;  // kernel columns precomputed on the matrix cores (two-kernel path, d > 16 or FP8 mode)
  bool packed;  // FP8 mode, d % 4 == 0: the points also as e4m3 codes (X8) with their norms (xn8)
  bool dist8;   // packed, d <= 256, d % 16 == 0: kernel columns in the update GEMM's epilogue
                // (the accepted points as codes in Xp8 with norms ypn; no C0)
  int part_cols;
  bool valu;  // vector-unit GEMM kernels instead of the matrix-core ones
  bool fblk;  // a panel-blocked copy of F (BF16 modes; FP64 and FP32 read F itself)
  int ncbt;   // > 0: one-kernel round product with this column-block count
  int grid;   // persistent workgroups of that kernel (set per call)
};

// Per-kernel-class timing with HIP events on the launch stream.
struct Profiler {
  hipStream_t s;
  bool on;
  unsigned mask;      // timed classes (bit per ARPC_KC_*)
  bool open = false;  // the current class is being timed
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<int, size_t>> marks;  // (class, index of start event)
  size_t used = 0;
  double ms[ARPC_NUM_KC] = {0};
  int64_t n[ARPC_NUM_KC] = {0};
  Profiler(hipStream_t st, unsigned classes) : s(st), on(classes != 0), mask(classes) {}
  ~Profiler() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(int cls) {
    open = on && ((mask >> cls) & 1u);
    if (!open) return;
    marks.push_back({cls, used});
    (void)hipEventRecord(next(), s);
  }
  void end() {
    if (!open) return;
    (void)hipEventRecord(next(), s);
    open = false;
  }
  // called after a stream synchronisation; ARPC_TRACE=1 also prints every
  // launch's time to stderr
  void collect() {
    if (!on) return;
    static const bool trace = getenv("ARPC_TRACE") != nullptr;
    for (auto& m : marks) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, pool[m.second], pool[m.second + 1]) == hipSuccess) {
        ms[m.first] += t;
        n[m.first] += 1;
        if (trace) fprintf(stderr, "arpc-trace class=%d launch=%lld ms=%.4f\n", m.first, (long long)n[m.first], t);
      }
    }
    marks.clear();
    used = 0;
  }
};

// One factorization driven by the host (see Job in api.cpp).
struct JobBase {
  virtual ~JobBase() {}
  virtual const RoundJob& row() const = 0;
  virtual arpc_status begin() = 0;
  virtual arpc_status capture_round() = 0;
  virtual arpc_status enqueue_batch() = 0;
  // look, look_ev: if set, the last round copies the round state into *look
  // after its rejection step and records look_ev
  virtual arpc_status enqueue_rounds(int64_t rounds, RoundState* look = nullptr, hipEvent_t look_ev = nullptr) = 0;
  virtual arpc_status enqueue_end() = 0;
  virtual bool running() = 0;
  virtual arpc_status finish(arpc_stats* stats, double ms_total) = 0;
  virtual arpc_status finish_enqueue(const RoundState& h, double* htrace) = 0;
  virtual arpc_status finish_stats(const RoundState& h, double trace_resid, arpc_stats* stats) = 0;
  // synchronous form: the end of the run (residual trace, zero tails)
  // followed by one copy of the state, trace and round history
  // (end_read_bytes) into host memory
  virtual size_t end_read_bytes() const = 0;
  virtual arpc_status enqueue_end_read(char* dst) = 0;
  virtual arpc_status finish_read(const char* src, arpc_stats* stats, double ms_total) = 0;
};

extern unsigned g_profiling;   // timed kernel classes (arpc_set_profiling*)
arpc_status validate(const arpc_problem* p);
KParams kparams_of(const arpc_problem& p);
Layout layout_of(const arpc_problem& p);
int fused_grid();
arpc_status check_factor_args(const arpc_problem* p, const double* X, const void* F, const int64_t* pivots);
std::unique_ptr<JobBase> make_job(const arpc_problem& p, const double* X, void* F, int64_t* pivots, char* ws,
                                  const Layout& l, hipStream_t s, const Unif& un, RoundState* hstate,
                                  Profiler* prof);
// The round kernels' table row of a factorization whose workspace ws has
// layout l (X: the points the rounds read, the rounded copy in the FP8 mode).
RoundJob round_job_of(const arpc_problem& p, const Layout& l, char* ws, const double* X, void* F,
                      int64_t* pivots, const Unif& un);
int gemm_prec(int prec);
// Checks the arguments, carves the workspace and runs the factorization to
// completion on `stream` (the host waits between batches of rounds).  timed:
// honour the process-wide profiling switch (else no events are created).
arpc_status factor_impl(const arpc_problem* p, const double* X, void* F, int64_t* pivots, void* ws,
                        size_t ws_bytes, void* stream, const Unif& un, arpc_stats* stats, bool timed);

}  // namespace arpc
