// C ABI and host code of the accelerated RPCholesky library.
//
// arpc_factor validates the problem, carves the caller's workspace, and
// enqueues rounds of Alg. 2 (each: proposals, residual submatrix,
// RejectionSampleSubmatrix, update GEMM, triangular solve, diagonal update)
// in batches.  The round state lives on the device; the host only reads it
// between batches to decide whether more rounds are needed.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/arpc.h"
#include "arpc_common.h"
#include "arpc_launch.h"
#include "arpc_mfma.h"
#include "arpc_host.h"

using namespace arpc;

namespace arpc {

unsigned g_profiling = 0;   // timed kernel classes

// The update GEMM and triangular solve run on the matrix cores; setting
// ARPC_GEMM=valu selects the register-tiled vector kernels instead (FP64 and
// FP32 modes only), which serve as a cross-check.
bool use_valu_gemm() {
  const char* e = getenv("ARPC_GEMM");
  return e && strcmp(e, "valu") == 0;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Persistent workgroups of the fused round kernel: two per compute unit of
// the current device.
int fused_grid() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  return 2 * cus;
}

// ARPC_FUSED=0 turns the one-kernel round product of the BF16 modes off (the
// two-kernel matrix-core path then runs, as for FP32), for cross-checks.
bool fused_disabled() {
  const char* e = getenv("ARPC_FUSED");
  return e && strcmp(e, "0") == 0;
}



inline int64_t nchunks_of(int64_t N) { return (N + CHUNK - 1) / CHUNK; }

size_t elem_size(int prec) { return prec == ARPC_FP64 ? sizeof(double) : sizeof(float); }

// The FP8 mode runs the BF16 mode's update GEMM and solve; only the kernel
// columns differ (FP8 contraction of the rounded points).
int gemm_prec(int prec) { return prec == ARPC_FP8 ? ARPC_BF16 : prec; }

Layout layout_of(const arpc_problem& p) {
  Layout l{};
  const size_t es = elem_size(p.prec);
  const int64_t nch = nchunks_of(p.N);
  const int gp = gemm_prec(p.prec);
  const bool valu = use_valu_gemm() && p.prec <= ARPC_FP32;
  l.valu = valu;
  // one kernel per round: the BF16 modes with d <= 16, and the one-product
  // BF16 mode with d <= 32 and b <= 208 (its LDS then holds the accepted
  // points' coordinates beside the resident inverse factor)
  const int fn = fused_ncbt(gp, (int)p.b);
  const bool fuse = !valu && !fused_disabled() && p.prec != ARPC_FP8 && fn > 0 &&
                    (p.d <= 16 || (gp == ARPC_BF16 && p.d <= 32 && fn <= 13));
  l.ncbt = fuse ? fn : -1;
  const bool fused = l.ncbt > 0;
  l.part_cols = valu ? 64 : (fused ? BMAX : mfma_part_cols(gp, (int)p.b));
  const int64_t nparts = (p.b + l.part_cols - 1) / l.part_cols;
  const size_t mb = valu ? 0 : (fused ? fused_operand_bytes(gp, p.k, (int)p.b)
                                      : mfma_operand_bytes(gp, p.k, (int)p.b));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  // the round state, the residual trace beside it and the round history
  // right after: the end of a run reads all three back in one copy
  static_assert(sizeof(RoundState) <= kTraceOff, "round state overlaps the trace slot");
  l.st = take(kTraceOff + sizeof(double));
  l.trace = l.st + kTraceOff;
  l.hist = take(sizeof(int32_t) * (p.k + 1));
  l.jd = take(sizeof(RoundJob));
  l.u = take(sizeof(double) * p.N);
  l.csum = take(sizeof(double) * nch);
  l.cpre = take(sizeof(double) * nch);
  l.props = take(sizeof(int64_t) * p.b);
  l.acc = take(sizeof(int32_t) * p.b);
  l.Fs = take(sizeof(double) * p.b * p.k);
  l.Fs32 = take(es == sizeof(float) ? sizeof(float) * p.b * fs32_ld(p.k) : 0);
  l.Hp = take(sizeof(double) * gather_splits(p.k) * p.b * p.b);
  l.H = take(sizeof(double) * p.b * p.b);
  l.Xp = take(sizeof(double) * p.b * p.d);
  l.Bt = take(valu ? es * p.k * p.b : 0);
  l.Bt2 = take(valu ? es * p.b * p.b : 0);
  l.Bm1 = take(mb);
  l.Bm2 = take(mb);
  // the blocked copy of F: the BF16 modes contract over it; FP64 and FP32 read F itself
  l.fblk = !valu && gp != ARPC_FP64 && gp != ARPC_FP32;
  l.Fb = take(l.fblk ? mfma_blocked_bytes(gp, p.N, p.k) : 0);
  l.C = take(valu ? es * p.N * p.b : (fused ? 0 : mfma_blocked_bytes(gp, p.N, p.b)));
  l.dist = !valu && !fused && (mfma_dist_contraction((int)p.d) || p.prec == ARPC_FP8);
  l.dist8 = l.dist && p.prec == ARPC_FP8 && p.d % 4 == 0 && mfma_dist_in_epilogue((int)p.d);
  l.C0 = take(l.dist && !l.dist8 ? es * p.N * p.b : 0);
  l.P = take(sizeof(double) * nparts * p.N);
  l.Xq = take(p.prec == ARPC_FP8 ? sizeof(double) * p.N * p.d : 0);
  l.packed = p.prec == ARPC_FP8 && l.dist && p.d % 4 == 0;   // e4m3 codes for the distance kernel
  l.X8 = take(l.packed ? (size_t)p.N * p.d : 0);
  l.xn8 = take(l.packed ? sizeof(float) * p.N : 0);
  l.Xp8 = take(l.dist8 ? (size_t)p.b * p.d : 0);
  l.ypn = take(l.dist8 ? sizeof(float) * p.b : 0);
  l.total = off;
  return l;
}

arpc_status validate(const arpc_problem* p) {
  if (!p) return ARPC_EINVAL;
  if (p->N < 1 || p->N > 2147483647LL) return ARPC_EINVAL;
  if (p->d < 1 || p->d > 4096) return ARPC_EINVAL;
  if (p->k < 1 || p->k > p->N) return ARPC_EINVAL;
  if (p->b < 1 || p->b > BMAX) return ARPC_EINVAL;
  if (p->kernel < ARPC_GAUSSIAN || p->kernel > ARPC_MATERN52) return ARPC_EINVAL;
  if (p->prec < ARPC_FP64 || p->prec > ARPC_FP8) return ARPC_EINVAL;
  if (!std::isfinite(p->bandwidth) || !(p->bandwidth > 0.0)) return ARPC_EINVAL;
  if (p->max_rounds < 0) return ARPC_EINVAL;
  if (p->method != ARPC_ACCEL && p->method != ARPC_BLOCK) return ARPC_EINVAL;
  if (p->reserved != 0) return ARPC_EINVAL;
  return ARPC_OK;
}

KParams kparams_of(const arpc_problem& p) {
  KParams kp{};
  kp.kernel = p.kernel;
  kp.sigma = p.bandwidth;
  if (p.kernel == ARPC_GAUSSIAN) kp.c0 = 1.0 / (2.0 * p.bandwidth * p.bandwidth);
  else if (p.kernel == ARPC_MATERN52) kp.c0 = 5.0 / (3.0 * p.bandwidth * p.bandwidth);
  return kp;
}



// Status of a finished run from its final round state.
arpc_status status_of(const arpc_problem& p, const RoundState& h) {
  if (h.nonfinite) return ARPC_ENUMERIC;
  if (h.status == ST_NOUNIF) return ARPC_EINVAL;
  if (h.status == ST_RUNNING) return ARPC_INCOMPLETE;
  return (h.k_r == p.k || (p.max_rounds > 0 && h.round >= p.max_rounds && h.status == ST_DONE)) ? ARPC_OK
                                                                                            : ARPC_EARLY_STOP;
}

// Statistics of a run from its final round state, the accepted count of
// each round (hist, h.round entries) and the residual trace.
void fill_stats(const arpc_problem& p, const Layout& l, const RoundState& h, const int32_t* hist, double trace_resid,
                arpc_stats* stats) {
  if (!stats) return;
  std::memset(stats, 0, sizeof(*stats));
  const arpc_status ret = status_of(p, h);
  const int64_t N = p.N;
  stats->k_out = h.k_r;
  stats->rounds = h.round;
  stats->proposals = h.proposals;
  stats->status = ret;
  stats->trace_A = h.trace_A;
  stats->trace_resid = trace_resid;
  // algorithmic traffic per round and row: the blocked copy of F read over
  // k_r columns at the contraction precision, the points, G written once to
  // F at its storage precision, the row norm; the two-kernel path also writes
  // C (update GEMM) and reads it (solve).  The write of G into the blocked
  // copy (which the next rounds contract over) is counted apart.  What the
  // two-kernel update GEMM reads for the kernel columns: the points in FP64
  // (epilogue from the coordinates), the e4m3 codes and a squared norm
  // (epilogue on the FP8 matrix cores), or the precomputed columns (s_r
  // values per row at the storage precision).
  double kr = 0.0, fg = 0.0, ft = 0.0, bg = 0.0, bt = 0.0, bb = 0.0;
  const double es = (double)elem_size(p.prec);
  const double eb = p.prec == ARPC_FP64 ? 8.0 : (gemm_prec(p.prec) == ARPC_BF16 ? 2.0 : 4.0);
  const bool fused = l.ncbt > 0;
  for (int64_t r = 0; r < h.round; ++r) {
    const double sr = hist[r];
    fg += 2.0 * (double)N * kr * sr;
    ft += (double)N * sr * sr;
    if (sr > 0) {
      if (fused) {
        bg += (double)N * (kr * eb + 8.0 * (double)p.d + sr * es + 8.0);
      } else {
        const double kc = l.dist8 ? (double)p.d + 4.0 : (l.dist ? sr * es : 8.0 * (double)p.d);
        bg += (double)N * (kr * eb + sr * eb + kc);
        bt += (double)N * (sr * (eb + es) + 8.0);
      }
      if (l.fblk) bb += (double)N * sr * eb;
    }
    kr += sr;
  }
  stats->fused = fused ? 1 : 0;
  stats->flops_colgemm = fg;
  stats->flops_trsm = ft;
  stats->bytes_colgemm = bg;
  stats->bytes_trsm = bt;
  stats->bytes_blocked = bb;
}

RoundJob round_job_of(const arpc_problem& p, const Layout& l, char* ws, const double* X, void* F,
                      int64_t* pivots, const Unif& un) {
  RoundJob j{};
  const int b = (int)p.b;
  const int64_t N = p.N, k = p.k;
  j.st = (RoundState*)(ws + l.st);
  j.u = (double*)(ws + l.u);
  j.csum = (double*)(ws + l.csum);
  j.cpre = (double*)(ws + l.cpre);
  j.nchunks = nchunks_of(N);
  j.N = N;
  j.X = X;
  j.d = (int)p.d;
  j.b = b;
  j.un = un;
  j.kp = kparams_of(p);
  j.props = (int64_t*)(ws + l.props);
  j.acc = (int32_t*)(ws + l.acc);
  j.pivots = pivots;
  j.kmax = k;
  j.max_rounds = p.max_rounds;
  j.keep_all = p.method == ARPC_BLOCK ? 1 : 0;
  j.part_cols = l.part_cols;
  j.F = F;
  j.Fs = (double*)(ws + l.Fs);
  j.Fs32 = elem_size(p.prec) == sizeof(float) ? (float*)(ws + l.Fs32) : nullptr;
  j.ldf = k;
  j.Hp = (double*)(ws + l.Hp);
  j.parts = gather_splits(k);
  j.W = gather_width(k);
  j.H = (double*)(ws + l.H);
  j.Xp = (double*)(ws + l.Xp);
  j.P = (const double*)(ws + l.P);
  j.hist = (int32_t*)(ws + l.hist);
  j.Fb = ws + l.Fb;
  j.nkc = (k + 31) / 32;
  j.Bm1 = (unsigned char*)(ws + l.Bm1);
  j.Bm2 = (unsigned char*)(ws + l.Bm2);
  if (l.ncbt > 0) {
    j.CP = 16 * l.ncbt;
    j.nt = (l.ncbt + 1) / 2;
    FusedRound fr{F, ws + l.Fb, j.nkc, N, X, j.d, j.Xp, j.kp, j.Bm1, j.Bm2, (double*)(ws + l.P), b, l.ncbt, l.grid};
    j.fa = fused_args_of(gemm_prec(p.prec), fr, j.st);
  }
  return j;
}

// One round of a factorization.  tab: its table row in device memory (hj:
// the host copy, g: its grids); the steps shared by every mode go through
// the table launchers, the two-kernel and vector-unit products take their
// arguments directly.
template <typename T>
void enqueue_round(hipStream_t s, const arpc_problem& p, const KParams& kp, char* ws, const Layout& l,
                   const double* X, T* F, const RoundJob* tab, const RoundJob& hj, const RoundGrid& g,
                   Profiler& prof, RoundState* look = nullptr, hipEvent_t look_ev = nullptr) {
  const int b = (int)p.b, d = (int)p.d;
  const int64_t N = p.N, k = p.k;
  RoundState* st = (RoundState*)(ws + l.st);
  int64_t* props = (int64_t*)(ws + l.props);
  int32_t* acc = (int32_t*)(ws + l.acc);
  double* Fs = (double*)(ws + l.Fs);
  double* H = (double*)(ws + l.H);
  double* Xp = (double*)(ws + l.Xp);
  T* Bt = (T*)(ws + l.Bt);
  T* Bt2 = (T*)(ws + l.Bt2);
  T* C = (T*)(ws + l.C);
  double* P = (double*)(ws + l.P);

  prof.begin(ARPC_KC_PROPOSE);
  launch_propose_tab(s, tab, 1, g);
  prof.end();
  prof.begin(ARPC_KC_GATHER);
  launch_gather_tab(s, tab, 1, g, sizeof(T) == sizeof(double), d > 32);
  prof.end();
  prof.begin(ARPC_KC_REJECT);
  launch_reject_tab(s, tab, 1, b);
  prof.end();
  if (look) {
    // the state once this round's pivots are known (s_r), read back while
    // the rest of the round runs
    (void)hipMemcpyAsync(look, st, sizeof(RoundState), hipMemcpyDeviceToHost, s);
    (void)hipEventRecord(look_ev, s);
  }
  if (l.ncbt > 0) {  // BF16 modes: one kernel for the update GEMM, the solve and the stores
    prof.begin(ARPC_KC_PREP);
    launch_fused_prep_tab(s, gemm_prec(p.prec), tab, 1, l.ncbt, p.b * p.d);
    prof.end();
    prof.begin(ARPC_KC_COLGEMM);
    launch_fused_round_tab(s, gemm_prec(p.prec), l.ncbt, d, hj.fa, tab, 1, fused_grid_of(gemm_prec(p.prec), hj.fa, l.grid));
    prof.end();
  } else if (l.valu) {  // vector-unit kernels (cross-check path)
    prof.begin(ARPC_KC_PREP);
    launch_prep<T>(s, Fs, k, acc, props, X, d, Bt, b, Xp, H, b, Bt2, k, st);
    prof.end();
    prof.begin(ARPC_KC_COLGEMM);
    launch_colgemm<T>(s, F, N, Bt, b, X, d, Xp, kp, C, b, st);
    prof.end();
    prof.begin(ARPC_KC_TRSM);
    launch_trsm<T>(s, C, N, Bt2, b, F, P, st);
    prof.end();
  } else {
    MfmaRound mr{F, l.fblk ? (void*)(ws + l.Fb) : nullptr, C, N, X, d, Xp, kp, (unsigned char*)(ws + l.Bm1), (unsigned char*)(ws + l.Bm2),
                 (int)((b + 15) / 16 * 16), P, Fs, k, acc, H, b, k,
                 l.dist && !l.dist8 ? (void*)(ws + l.C0) : nullptr,
                 l.packed ? (const unsigned*)(ws + l.X8) : nullptr, l.packed ? (const float*)(ws + l.xn8) : nullptr,
                 l.dist8 ? (const unsigned char*)(ws + l.Xp8) : nullptr,
                 l.dist8 ? (const float*)(ws + l.ypn) : nullptr};
    if (elem_size(p.prec) == sizeof(float)) mr.Fs32 = (const float*)(ws + l.Fs32);
    prof.begin(ARPC_KC_PREP);
    launch_prep_xp_tab(s, tab, 1, p.b * p.d);
    if (l.dist8)   // the accepted points as e4m3 codes for the update GEMM's epilogue
      launch_pack_e4m3(s, Xp, b, d, (unsigned*)(ws + l.Xp8), (float*)(ws + l.ypn));
    launch_mfma_prep(s, gemm_prec(p.prec), mr, st);
    prof.end();
    prof.begin(ARPC_KC_COLGEMM);
    if (mr.C0) launch_dist(s, p.prec, mr, st);
    launch_mfma_colgemm(s, gemm_prec(p.prec), mr, st);
    prof.end();
    prof.begin(ARPC_KC_TRSM);
    launch_mfma_trsm(s, gemm_prec(p.prec), mr, st);
    prof.end();
  }
  prof.begin(ARPC_KC_DIAG);
  launch_diag_tab(s, tab, 1, g);
  prof.end();
  prof.begin(ARPC_KC_FINISH);
  launch_finish_tab(s, tab, 1);
  prof.end();
}

#define HIPCHK(x)                          \
  do {                                     \
    if ((x) != hipSuccess) return ARPC_EDEVICE; \
  } while (0)

// One factorization as a host-side state machine, shared by arpc_factor and
// the serving scheduler: begin() enqueues the initial pass, enqueue_batch() a
// batch of rounds followed by an asynchronous copy of the round state into
// *hstate, running() inspects that copy once the stream has reached it, and
// finish() enqueues the final reductions, waits for them and fills the stats.
template <typename T>
struct Job final : JobBase {
  arpc_problem p;
  const double* X;
  T* F;
  int64_t* pivots;
  char* ws;
  Layout l;
  hipStream_t s;
  Unif un;
  KParams kp;
  RoundState* hstate;
  Profiler* prof;
  int64_t known_k = 0, enqueued = 0;
  hipGraphExec_t round_graph = nullptr;

  const double* Xin;   // the caller's points (X: the points every round reads)
  RoundJob hj;         // the round kernels' table row (host copy; the device copy is at ws + l.jd)
  RoundGrid g;

  Job(const arpc_problem& p_, const double* X_, T* F_, int64_t* piv_, char* ws_, const Layout& l_,
      hipStream_t s_, const Unif& un_, RoundState* h_, Profiler* prof_)
      : p(p_), X(p_.prec == ARPC_FP8 ? (const double*)(ws_ + l_.Xq) : X_), F(F_), pivots(piv_), ws(ws_), l(l_),
        s(s_), un(un_), kp(kparams_of(p_)), hstate(h_), prof(prof_), Xin(X_),
        hj(round_job_of(p_, l_, ws_, X, F_, piv_, un_)), g(round_grid_of(hj)) {}
  const RoundJob& row() const override { return hj; }
  ~Job() override {
    if (round_graph) (void)hipGraphExecDestroy(round_graph);
  }

  arpc_status begin() override {
    RoundState* st = (RoundState*)(ws + l.st);
    const int64_t nch = nchunks_of(p.N);
    HIPCHK(hipMemsetAsync(st, 0, sizeof(RoundState), s));
    launch_store_job(s, hj, (RoundJob*)(ws + l.jd));
    prof->begin(ARPC_KC_INIT);
    // FP8 mode: the rounded points (and, d % 4 == 0, their codes, norms and
    // the non-finite flag in the same pass, so the initialisation scans none)
    if (l.packed)
      launch_round_pack_e4m3(s, Xin, p.N, (int)p.d, (double*)(ws + l.Xq), (unsigned*)(ws + l.X8),
                             (float*)(ws + l.xn8), st);
    else if (p.prec == ARPC_FP8)
      launch_round_e4m3(s, Xin, (double*)(ws + l.Xq), p.N * p.d);
    launch_init(s, (double*)(ws + l.u), (double*)(ws + l.csum), X, p.N, l.packed ? 0 : (int)p.d, kp, st, nch);
    prof->end();
    HIPCHK(hipGetLastError());
    return ARPC_OK;
  }

  // Record one round's kernels as a graph (they read the round state from
  // device memory, so the same graph serves every round of this job).
  arpc_status capture_round() override {
    Profiler off(s, false);
    hipGraph_t gr = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    enqueue_round<T>(s, p, kp, ws, l, X, F, (const RoundJob*)(ws + l.jd), hj, g, off);
    const hipError_t e = hipStreamEndCapture(s, &gr);
    if (e != hipSuccess || !gr) return ARPC_EDEVICE;
    const hipError_t ei = hipGraphInstantiate(&round_graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ei != hipSuccess) {
      round_graph = nullptr;
      return ARPC_EDEVICE;
    }
    return ARPC_OK;
  }

  arpc_status enqueue_batch() override {
    // the fewest rounds that could still be needed (every round accepts <= b)
    int64_t batch = (p.k - known_k + p.b - 1) / p.b;
    if (batch < 1) batch = 1;
    if (p.max_rounds > 0 && enqueued + batch > p.max_rounds) batch = p.max_rounds - enqueued;
    if (batch < 1) batch = 1;
    for (int64_t r = 0; r < batch; ++r) {
      if (round_graph) HIPCHK(hipGraphLaunch(round_graph, s));
      else enqueue_round<T>(s, p, kp, ws, l, X, F, (const RoundJob*)(ws + l.jd), hj, g, *prof);
    }
    enqueued += batch;
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(hstate, ws + l.st, sizeof(RoundState), hipMemcpyDeviceToHost, s));
    return ARPC_OK;
  }

  // Rounds and the end of the run enqueued without reading anything back
  // (the asynchronous entry points): rounds past the end exit on the device.
  arpc_status enqueue_rounds(int64_t rounds, RoundState* look, hipEvent_t look_ev) override {
    for (int64_t r = 0; r < rounds; ++r)
      enqueue_round<T>(s, p, kp, ws, l, X, F, (const RoundJob*)(ws + l.jd), hj, g, *prof,
                       r + 1 == rounds ? look : nullptr, look_ev);
    HIPCHK(hipGetLastError());
    return ARPC_OK;
  }

  arpc_status enqueue_end() override {
    launch_trace(s, (double*)(ws + l.csum), nchunks_of(p.N), (double*)(ws + l.trace));
    launch_zero_tail(s, (const RoundState*)(ws + l.st), p.k, p.N, (int)sizeof(T), F, pivots);
    HIPCHK(hipGetLastError());
    return ARPC_OK;
  }

  bool running() override {
    if (hstate->status != ST_RUNNING) return false;
    known_k = hstate->k_r;
    return true;
  }

  // Batched form of the end of a run (serving ticks): enqueue the residual
  // trace into *htrace and the zero tails of F and pivots for the final
  // state h (read by the caller after the last tick that ran this job);
  // finish_stats then fills the statistics once the stream has passed them.
  arpc_status finish_enqueue(const RoundState& h, double* htrace) override {
    const int64_t N = p.N, nch = nchunks_of(N);
    double* tr = (double*)(ws + l.trace);
    launch_trace(s, (double*)(ws + l.csum), nch, tr);
    HIPCHK(hipMemcpyAsync(htrace, tr, sizeof(double), hipMemcpyDeviceToHost, s));
    // zero tails of F and pivots past k_r, from the device state (which h copies)
    if (h.k_r < p.k && !h.nonfinite)
      launch_zero_tail(s, (const RoundState*)(ws + l.st), p.k, N, (int)sizeof(T), F, pivots);
    HIPCHK(hipGetLastError());
    return ARPC_OK;
  }

  arpc_status finish_stats(const RoundState& h, double trace_resid, arpc_stats* stats) override {
    const arpc_status ret = status_of(p, h);
    if (ret == ARPC_ENUMERIC) return ret;
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->k_out = h.k_r;
      stats->rounds = h.round;
      stats->proposals = h.proposals;
      stats->status = ret;
      stats->fused = l.ncbt > 0 ? 1 : 0;
      stats->trace_A = h.trace_A;
      stats->trace_resid = trace_resid;
    }
    return ret;
  }

  size_t end_read_bytes() const override { return l.hist - l.st + sizeof(int32_t) * (size_t)(p.k + 1); }

  arpc_status enqueue_end_read(char* dst) override {
    arpc_status e = enqueue_end();
    if (e != ARPC_OK) return e;
    HIPCHK(hipMemcpyAsync(dst, ws + l.st, end_read_bytes(), hipMemcpyDeviceToHost, s));
    return ARPC_OK;
  }

  // src: what enqueue_end_read copied, after the stream has passed it
  arpc_status finish_read(const char* src, arpc_stats* stats, double ms_total) override {
    RoundState h;
    std::memcpy(&h, src, sizeof(h));
    if (h.nonfinite) return ARPC_ENUMERIC;
    double trace_resid;
    std::memcpy(&trace_resid, src + (l.trace - l.st), sizeof(double));
    const int32_t* hist = (const int32_t*)(src + (l.hist - l.st));
    const arpc_status ret = status_of(p, h);
    fill_stats(p, l, h, hist, trace_resid, stats);
    if (stats) {
      for (int c = 0; c < ARPC_NUM_KC; ++c) {
        stats->ms_kernel[c] = prof->ms[c];
        stats->launches[c] = prof->n[c];
      }
      stats->ms_total = ms_total;
    }
    return ret;
  }

  arpc_status finish(arpc_stats* stats, double ms_total) override {
    const RoundState h = *hstate;
    if (h.nonfinite) return ARPC_ENUMERIC;
    const int64_t N = p.N, nch = nchunks_of(N);
    // final residual trace and round history
    double* tr = (double*)(ws + l.trace);
    launch_trace(s, (double*)(ws + l.csum), nch, tr);
    double trace_resid = 0.0;
    HIPCHK(hipMemcpyAsync(&trace_resid, tr, sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<int32_t> hist((size_t)h.round + 1, 0);
    if (h.round > 0)
      HIPCHK(hipMemcpyAsync(hist.data(), ws + l.hist, sizeof(int32_t) * h.round, hipMemcpyDeviceToHost, s));
    if (h.k_r < p.k) launch_zero_tail(s, (const RoundState*)(ws + l.st), p.k, N, (int)sizeof(T), F, pivots);
    HIPCHK(hipStreamSynchronize(s));

    const arpc_status ret = status_of(p, h);
    fill_stats(p, l, h, hist.data(), trace_resid, stats);
    if (stats) {
      for (int c = 0; c < ARPC_NUM_KC; ++c) {
        stats->ms_kernel[c] = prof->ms[c];
        stats->launches[c] = prof->n[c];
      }
      stats->ms_total = ms_total;
    }
    return ret;
  }
};


std::unique_ptr<JobBase> make_job(const arpc_problem& p, const double* X, void* F, int64_t* pivots, char* ws,
                                  const Layout& l, hipStream_t s, const Unif& un, RoundState* hstate,
                                  Profiler* prof) {
  if (p.prec == ARPC_FP64)
    return std::unique_ptr<JobBase>(new Job<double>(p, X, (double*)F, pivots, ws, l, s, un, hstate, prof));
  return std::unique_ptr<JobBase>(new Job<float>(p, X, (float*)F, pivots, ws, l, s, un, hstate, prof));
}

arpc_status check_factor_args(const arpc_problem* p, const double* X, const void* F, const int64_t* pivots) {
  arpc_status v = validate(p);
  if (v != ARPC_OK) return v;
  if (!X || !F || !pivots) return ARPC_EINVAL;
  if (((uintptr_t)X & 7) || ((uintptr_t)F & 7) || ((uintptr_t)pivots & 7)) return ARPC_EINVAL;
  if (use_valu_gemm() && p->prec > ARPC_FP32) return ARPC_EINVAL;  // vector kernels: FP64/FP32 only
  return ARPC_OK;
}

}  // namespace arpc

namespace arpc {

// Pinned host memory for the synchronous form's read-backs, one buffer per
// host thread, grown on demand and held until the process ends (a release at
// exit could run after the runtime has been torn down).
static char* sync_staging(size_t bytes) {
  thread_local char* buf = nullptr;
  thread_local size_t cap = 0;
  if (bytes > cap) {
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    const size_t n = (bytes + 65535) & ~size_t(65535);
    if (hipHostMalloc((void**)&buf, n, hipHostMallocDefault) != hipSuccess) {
      buf = nullptr;
      return nullptr;
    }
    cap = n;
  }
  return buf;
}

// Pivots and rounds at a look at the state taken after a round's rejection
// step: what the run will hold once that round ends.
struct Look {
  int64_t pivots = 0, rounds = 0;
};

// Rounds to enqueue after the round in flight, from the state m read back
// after its rejection step (its s_r known) and the previous look: the pivots
// still missing, at the rate the rounds since that look added them, less
// one.  The last of them looks again, so the count never needs to run over:
// it only has to keep the stream from draining.
static int64_t rounds_to_add(const arpc_problem& p, const Look& prev, const RoundState& m, int64_t enqueued) {
  if (m.status != ST_RUNNING || m.s_r == 0) return 0;
  const Look now{m.k_r + m.s_r, m.round + 1};
  if (now.pivots >= p.k) return 0;
  if (p.max_rounds > 0 && enqueued >= p.max_rounds) return 0;
  const int64_t dr = now.rounds - prev.rounds;
  double rate = dr > 0 ? (double)(now.pivots - prev.pivots) / (double)dr : (double)p.b;
  if (rate < 1.0) rate = 1.0;
  int64_t r = (int64_t)std::ceil((double)(p.k - now.pivots) / rate) - 1;
  if (r < 1) r = 1;
  if (p.max_rounds > 0 && enqueued + r > p.max_rounds) r = p.max_rounds - enqueued;
  return r;
}

// The synchronous factorization.  The host never lets the stream drain
// between rounds: the last round of each batch reads the state back after its
// rejection step, and while the rest of that round runs the host enqueues
// more rounds if that round leaves pivots missing, or else the end of the
// run, and waits for it.  No round past the last one is enqueued.
static arpc_status run_sync(const arpc_problem& p, const double* X, void* F, int64_t* pivots, char* ws,
                            const Layout& l, hipStream_t s, const Unif& un, arpc_stats* stats, unsigned classes) {
  const auto t0 = std::chrono::steady_clock::now();
  Profiler prof(s, classes);
  auto job = make_job(p, X, F, pivots, ws, l, s, un, nullptr, &prof);
  char* stg = sync_staging(256 + job->end_read_bytes());
  if (!stg) return ARPC_ENOMEM;
  RoundState* look = (RoundState*)stg;
  char* endb = stg + 256;
  hipEvent_t ev;
  HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t e;
    ~EvGuard() { (void)hipEventDestroy(e); }
  } guard{ev};

  arpc_status e = job->begin();
  if (e != ARPC_OK) return e;
  int64_t enq = 0;
  int64_t want = (p.k + p.b - 1) / p.b;   // the fewest rounds that could suffice
  if (p.max_rounds > 0 && want > p.max_rounds) want = p.max_rounds;
  if (want < 1) want = 1;
  Look prev;
  for (;;) {
    e = job->enqueue_rounds(want - enq, look, ev);
    if (e != ARPC_OK) return e;
    enq = want;
    HIPCHK(hipEventSynchronize(ev));
    const RoundState m = *look;
    const int64_t more = rounds_to_add(p, prev, m, enq);
    if (m.status == ST_RUNNING) prev = Look{m.k_r + m.s_r, m.round + 1};
    if (more > 0) {
      want = enq + more;
      continue;
    }
    e = job->enqueue_end_read(endb);
    if (e != ARPC_OK) return e;
    HIPCHK(hipStreamSynchronize(s));
    RoundState f;
    std::memcpy(&f, endb, sizeof(f));
    if (f.status != ST_RUNNING) break;
    // cannot happen: the look saw the last round's pivots, and the round
    // limit ends the run on the device; one more batch keeps it safe
    want = enq + 1;
  }
  prof.collect();
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return job->finish_read(endb, stats, ms);
}

arpc_status factor_impl(const arpc_problem* p, const double* X, void* F, int64_t* pivots, void* ws,
                        size_t ws_bytes, void* stream, const Unif& un, arpc_stats* stats, bool timed) {
  arpc_status v = check_factor_args(p, X, F, pivots);
  if (v != ARPC_OK) return v;
  if (!ws || ((uintptr_t)ws & 255)) return ARPC_EINVAL;
  Layout l = layout_of(*p);
  if (ws_bytes < l.total) return ARPC_EINVAL;
  if (l.ncbt > 0) l.grid = fused_grid();
  return run_sync(*p, X, F, pivots, (char*)ws, l, (hipStream_t)stream, un, stats, timed ? g_profiling : 0u);
}

}  // namespace arpc

extern "C" {

const char* arpc_status_str(int status) {
  switch (status) {
    case ARPC_OK: return "ok";
    case ARPC_EARLY_STOP: return "early stop: residual reached zero before k pivots";
    case ARPC_INCOMPLETE: return "incomplete: the enqueued rounds ended before k pivots";
    case ARPC_EINVAL: return "invalid argument";
    case ARPC_ENOMEM: return "out of memory";
    case ARPC_EBUSY: return "busy";
    case ARPC_EDEVICE: return "HIP runtime error";
    case ARPC_ENUMERIC: return "non-finite input";
    case ARPC_ECANCELED: return "cancelled";
    default: return "unknown status";
  }
}

const char* arpc_version(void) { return "arpc-gfx950 0.1"; }

arpc_status arpc_workspace_size(const arpc_problem* problem, size_t* bytes) {
  if (!bytes) return ARPC_EINVAL;
  arpc_status v = validate(problem);
  if (v != ARPC_OK) return v;
  *bytes = layout_of(*problem).total;
  return ARPC_OK;
}

arpc_status arpc_factor(const arpc_problem* problem, const double* X, void* F, int64_t* pivots, void* ws,
                        size_t ws_bytes, void* stream, arpc_stats* stats) {
  if (!problem) return ARPC_EINVAL;
  Unif un{nullptr, 0, problem->seed};
  return factor_impl(problem, X, F, pivots, ws, ws_bytes, stream, un, stats, true);
}

arpc_status arpc_factor_uniforms(const arpc_problem* problem, const double* X, void* F, int64_t* pivots,
                                 void* ws, size_t ws_bytes, void* stream, const double* U, int64_t nU,
                                 arpc_stats* stats) {
  if (!problem || !U || nU < 0 || ((uintptr_t)U & 7)) return ARPC_EINVAL;
  Unif un{U, nU, problem->seed};
  return factor_impl(problem, X, F, pivots, ws, ws_bytes, stream, un, stats, true);
}

// Rounds enqueued by arpc_factor_async when the problem sets no round limit:
// the fewest that could suffice, plus half as many again and four.
static int64_t default_async_rounds(const arpc_problem& p) {
  const int64_t need = (p.k + p.b - 1) / p.b;
  int64_t r = need + need / 2 + 4;
  return r < p.k ? r : p.k;
}

arpc_status arpc_factor_async(const arpc_problem* problem, const double* X, void* F, int64_t* pivots, void* ws,
                              size_t ws_bytes, void* stream, int64_t rounds) {
  if (!problem) return ARPC_EINVAL;
  arpc_status v = check_factor_args(problem, X, F, pivots);
  if (v != ARPC_OK) return v;
  if (!ws || ((uintptr_t)ws & 255) || rounds < 0) return ARPC_EINVAL;
  Layout l = layout_of(*problem);
  if (ws_bytes < l.total) return ARPC_EINVAL;
  if (l.ncbt > 0) l.grid = fused_grid();
  if (rounds == 0) rounds = problem->max_rounds > 0 ? problem->max_rounds : default_async_rounds(*problem);
  const Unif un{nullptr, 0, problem->seed};
  hipStream_t s = (hipStream_t)stream;
  Profiler prof(s, 0u);
  auto job = make_job(*problem, X, F, pivots, (char*)ws, l, s, un, nullptr, &prof);
  arpc_status e = job->begin();
  if (e == ARPC_OK) e = job->enqueue_rounds(rounds);
  if (e == ARPC_OK) e = job->enqueue_end();
  return e;
}

arpc_status arpc_factor_continue(const arpc_problem* problem, const double* X, void* F, int64_t* pivots, void* ws,
                                 size_t ws_bytes, void* stream, int64_t rounds) {
  if (!problem) return ARPC_EINVAL;
  arpc_status v = check_factor_args(problem, X, F, pivots);
  if (v != ARPC_OK) return v;
  if (!ws || ((uintptr_t)ws & 255) || rounds < 1) return ARPC_EINVAL;
  Layout l = layout_of(*problem);
  if (ws_bytes < l.total) return ARPC_EINVAL;
  if (l.ncbt > 0) l.grid = fused_grid();
  const Unif un{nullptr, 0, problem->seed};
  hipStream_t s = (hipStream_t)stream;
  Profiler prof(s, 0u);
  auto job = make_job(*problem, X, F, pivots, (char*)ws, l, s, un, nullptr, &prof);
  arpc_status e = job->enqueue_rounds(rounds);
  if (e == ARPC_OK) e = job->enqueue_end();
  return e;
}

arpc_status arpc_factor_query(const arpc_problem* problem, const void* ws, size_t ws_bytes, arpc_stats* stats) {
  arpc_status v = validate(problem);
  if (v != ARPC_OK) return v;
  if (!ws || ((uintptr_t)ws & 255)) return ARPC_EINVAL;
  const Layout l = layout_of(*problem);
  if (ws_bytes < l.total) return ARPC_EINVAL;
  const char* w = (const char*)ws;
  RoundState h{};
  double trace = 0.0;
  if (hipMemcpy(&h, w + l.st, sizeof(RoundState), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&trace, w + l.trace, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return ARPC_EDEVICE;
  if (h.round < 0 || h.round > problem->k) return ARPC_EINVAL;   // not a state this library wrote
  std::vector<int32_t> hist((size_t)h.round + 1, 0);
  if (h.round > 0 &&
      hipMemcpy(hist.data(), w + l.hist, sizeof(int32_t) * (size_t)h.round, hipMemcpyDeviceToHost) != hipSuccess)
    return ARPC_EDEVICE;
  fill_stats(*problem, l, h, hist.data(), trace, stats);
  return status_of(*problem, h);
}

arpc_status arpc_stream_uniforms_host(uint64_t seed, int64_t start, int64_t n, double* out) {
  if (start < 0 || n < 0 || (n > 0 && !out)) return ARPC_EINVAL;
  for (int64_t i = 0; i < n; ++i) out[i] = philox_uniform(seed, (uint64_t)(start + i));
  return ARPC_OK;
}

void arpc_set_profiling(int on) { g_profiling = on ? ~0u : 0u; }

void arpc_set_profiling_classes(unsigned mask) { g_profiling = mask; }

}  // extern "C"
