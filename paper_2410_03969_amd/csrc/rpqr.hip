// Accelerated randomly pivoted QR (Alg. 5, Section 5): kernels and the
// host code of arpc_qr_factor.
//
// B is a dense M x N FP64 matrix (column-major).  A round proposes b columns
// from the residual squared column norms u (the shared proposal kernels),
// forms their residual columns C = B(:,S') - Q F(S',:)^*, keeps a subset by
// RejectionSampleSubmatrix (the shared kernel) on H = C^* C, and extends
//   Q by Q_perp = Orth(C(:,T) - Q (Q^* C(:,T)))   (one extra Gram-Schmidt pass),
//   F by G = B^* Q_perp,  u -= rowsqnorm(G)  (the shared diagonal kernel).
// Orth is Cholesky QR: R^* R = Q_perp^* Q_perp, Q_perp <- Q_perp R^{-1}, the
// QR factorization with a positive diagonal in R (R^{-1} formed explicitly,
// one workgroup per column).  Every product runs on the library's FP64
// matrix-core GEMM (column-major operands, contractions over the M rows split
// over workgroups and summed in a fixed order); the host reads s_r after each
// round's rejection step, since those products take their sizes on the host.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>

#include "../../include/arpc.h"
#include "arpc_common.h"
#include "arpc_dense.h"
#include "arpc_host.h"
#include "arpc_launch.h"

namespace arpc {
namespace {

constexpr int QR_BMAX = 512;

// u(j) = |B(:, j)|^2, one wavefront per column; a non-finite entry sets the flag.
__global__ __launch_bounds__(256) void k_qr_colnorms(const double* __restrict__ B, int64_t M, int64_t N,
                                                     double* __restrict__ u, RoundState* st) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= N) return;
  const double* col = B + j * M;
  double s = 0.0;
  for (int64_t r = lane; r < M; r += 64) s = fma(col[r], col[r], s);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) {
    u[j] = s;
    if (!isfinite(s)) atomicOr(&st->nonfinite, 1);
  }
}

// C(:, i) = B(:, idx[i]) for i < n (M rows).
__global__ __launch_bounds__(256) void k_qr_cols(const double* __restrict__ B, int64_t M,
                                                 const int64_t* __restrict__ idx, int n, double* __restrict__ C) {
  const int i = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n || r >= M) return;
  C[(int64_t)i * M + r] = B[idx[i] * M + r];
}

// Fs(i, t) = F(props[i], t) for i < b, t < kr (column-major, ld b).
__global__ __launch_bounds__(256) void k_qr_rows(const double* __restrict__ F, int64_t N,
                                                 const int64_t* __restrict__ props, int b, int64_t kr,
                                                 double* __restrict__ Fs) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= kr * b) return;
  const int64_t t = e / b;
  const int i = (int)(e % b);
  Fs[e] = F[t * N + props[i]];
}

// Qn(:, a) = C(:, acc[a]) for a < s.
__global__ __launch_bounds__(256) void k_qr_take(const double* __restrict__ C, int64_t M,
                                                 const int32_t* __restrict__ acc, int s, double* __restrict__ Qn) {
  const int a = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (a >= s || r >= M) return;
  Qn[(int64_t)a * M + r] = C[(int64_t)acc[a] * M + r];
}

// P(j) = sum_{c < s} G(j, c)^2 (G column-major, ld N).
__global__ __launch_bounds__(256) void k_qr_rownorms(const double* __restrict__ G, int64_t N, int s,
                                                     double* __restrict__ P) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  double v = 0.0;
  for (int c = 0; c < s; ++c) {
    const double g = G[(int64_t)c * N + j];
    v = fma(g, g, v);
  }
  P[j] = v;
}

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

namespace {

struct QrLayout {
  size_t st, u, csum, cpre, props, acc, hist, Fs, C, H, Tm, Gr, Li, P, part, trace, bad, total;
  size_t part_elems;
};

QrLayout qr_layout(int64_t M, int64_t N, int64_t k, int64_t b) {
  QrLayout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += al256(bytes);
    return o;
  };
  const int64_t nch = (N + CHUNK - 1) / CHUNK;
  l.st = take(sizeof(RoundState));
  l.u = take(sizeof(double) * N);
  l.csum = take(sizeof(double) * nch);
  l.cpre = take(sizeof(double) * nch);
  l.props = take(sizeof(int64_t) * b);
  l.acc = take(sizeof(int32_t) * b);
  l.hist = take(sizeof(int32_t) * (k + 1));
  l.Fs = take(sizeof(double) * b * k);
  l.C = take(sizeof(double) * M * b);
  l.H = take(sizeof(double) * b * b);
  l.Tm = take(sizeof(double) * k * b);
  l.Gr = take(sizeof(double) * b * b);
  l.Li = take(sizeof(double) * b * b);
  l.P = take(sizeof(double) * N);
  // split contractions over the M rows: H = C^* C, Q^* Q_perp, Q_perp^* Q_perp
  size_t pe = dgemm_part_elems(b, b, M);
  if (dgemm_part_elems(k, b, M) > pe) pe = dgemm_part_elems(k, b, M);
  l.part_elems = pe;
  l.part = take(sizeof(double) * pe);
  l.trace = take(sizeof(double));
  l.bad = take(sizeof(int));
  l.total = off;
  return l;
}

arpc_status qr_validate(int64_t M, int64_t N, int64_t k, int64_t b, int64_t max_rounds) {
  if (M < 1 || N < 1 || M > 2147483647LL || N > 2147483647LL) return ARPC_EINVAL;
  if (k < 1 || k > M || k > N) return ARPC_EINVAL;
  if (b < 1 || b > QR_BMAX || max_rounds < 0) return ARPC_EINVAL;
  return ARPC_OK;
}

#define QCHK(x)                               \
  do {                                        \
    if ((x) != hipSuccess) return ARPC_EDEVICE; \
  } while (0)

arpc_status qr_run(int64_t M, int64_t N, int64_t k, int64_t b, uint64_t seed, int64_t max_rounds,
                   const double* B, double* Q, double* F, int64_t* pivots, char* ws, const QrLayout& l,
                   hipStream_t s, arpc_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  Profiler prof(s, g_profiling);
  const Unif un{nullptr, 0, seed};
  const int64_t nch = (N + CHUNK - 1) / CHUNK;
  RoundState* st = (RoundState*)(ws + l.st);
  double* u = (double*)(ws + l.u);
  double* csum = (double*)(ws + l.csum);
  int64_t* props = (int64_t*)(ws + l.props);
  int32_t* acc = (int32_t*)(ws + l.acc);
  double* Fs = (double*)(ws + l.Fs);
  double* C = (double*)(ws + l.C);
  double* H = (double*)(ws + l.H);
  double* Tm = (double*)(ws + l.Tm);
  double* Gr = (double*)(ws + l.Gr);
  double* Li = (double*)(ws + l.Li);
  double* P = (double*)(ws + l.P);
  double* part = (double*)(ws + l.part);
  const size_t pe = l.part_elems;
  int* bad = (int*)(ws + l.bad);
  const int ib = (int)b;
  QCHK(hipMemsetAsync(st, 0, sizeof(RoundState), s));
  QCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
  QCHK(hipMemsetAsync(Q, 0, sizeof(double) * (size_t)M * (size_t)k, s));
  QCHK(hipMemsetAsync(F, 0, sizeof(double) * (size_t)N * (size_t)k, s));
  prof.begin(ARPC_KC_INIT);
  hipLaunchKernelGGL(k_qr_colnorms, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, B, M, N, u, st);
  launch_init_from_diag(s, u, N, csum, st, nch);
  prof.end();
  QCHK(hipGetLastError());
  RoundState hs{};
  int64_t kr = 0;
  for (;;) {
    prof.begin(ARPC_KC_PROPOSE);
    launch_propose(s, u, csum, (double*)(ws + l.cpre), nch, N, ib, un, st, props);
    prof.end();
    prof.begin(ARPC_KC_GATHER);
    hipLaunchKernelGGL(k_qr_cols, dim3((unsigned)((M + 255) / 256), (unsigned)b), dim3(256), 0, s, B, M, props, ib, C);
    if (kr > 0) {
      hipLaunchKernelGGL(k_qr_rows, dim3((unsigned)((kr * b + 255) / 256)), dim3(256), 0, s, F, N, props, ib, kr, Fs);
      QCHK(dgemm(s, false, true, M, ib, kr, -1.0, Q, M, Fs, ib, 1.0, C, M, part, pe));   // C -= Q F(S',:)^*
    }
    QCHK(dgemm(s, true, false, ib, ib, M, 1.0, C, M, C, M, 0.0, H, ib, part, pe));          // H = C^* C
    prof.end();
    prof.begin(ARPC_KC_REJECT);
    launch_reject(s, H, ib, props, un, st, acc, pivots, u, k, false);
    prof.end();
    QCHK(hipGetLastError());
    QCHK(hipMemcpyAsync(&hs, st, sizeof(RoundState), hipMemcpyDeviceToHost, s));
    QCHK(hipStreamSynchronize(s));
    prof.collect();
    if (hs.status != ST_RUNNING) break;
    const int sr = hs.s_r;
    if (sr > 0) {
      double* Qn = Q + kr * M;
      prof.begin(ARPC_KC_PREP);
      hipLaunchKernelGGL(k_qr_take, dim3((unsigned)((M + 255) / 256), (unsigned)sr), dim3(256), 0, s, C, M, acc, sr,
                         Qn);
      if (kr > 0) {   // one extra Gram-Schmidt pass: Q_perp -= Q (Q^* Q_perp)
        QCHK(dgemm(s, true, false, kr, sr, M, 1.0, Q, M, Qn, M, 0.0, Tm, kr, part, pe));
        QCHK(dgemm(s, false, false, M, sr, kr, -1.0, Q, M, Tm, kr, 1.0, Qn, M, part, pe));
      }
      // Cholesky QR: R^* R = Q_perp^* Q_perp (R^* = the lower factor in Gr),
      // Q_perp <- Q_perp R^{-1} = Q_perp (R^{-*})^*, through C as scratch
      QCHK(dgemm(s, true, false, sr, sr, M, 1.0, Qn, M, Qn, M, 0.0, Gr, sr, part, pe));
      launch_chol_block(s, Gr, sr, sr, bad);
      launch_trinv_lower(s, Gr, sr, sr, Li, sr);
      QCHK(dgemm(s, false, true, M, sr, sr, 1.0, Qn, M, Li, sr, 0.0, C, M, part, pe));
      QCHK(hipMemcpyAsync(Qn, C, sizeof(double) * (size_t)M * (size_t)sr, hipMemcpyDeviceToDevice, s));
      prof.end();
      prof.begin(ARPC_KC_COLGEMM);
      QCHK(dgemm(s, true, false, N, sr, M, 1.0, B, M, Qn, M, 0.0, F + kr * N, N, part, pe));   // G = B^* Q_perp
      prof.end();
      prof.begin(ARPC_KC_DIAG);
      hipLaunchKernelGGL(k_qr_rownorms, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, F + kr * N, N, sr, P);
      launch_diag(s, u, csum, P, QR_BMAX, N, nch, st);
      prof.end();
    }
    prof.begin(ARPC_KC_FINISH);
    launch_finish(s, st, ib, k, max_rounds, (int32_t*)(ws + l.hist));
    prof.end();
    QCHK(hipGetLastError());
    QCHK(hipMemcpyAsync(&hs, st, sizeof(RoundState), hipMemcpyDeviceToHost, s));
    QCHK(hipStreamSynchronize(s));
    prof.collect();
    kr = hs.k_r;
    if (hs.status != ST_RUNNING) break;
  }
  if (hs.nonfinite) return ARPC_ENUMERIC;
  int hbad = 0;
  QCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  double* tr = (double*)(ws + l.trace);
  launch_trace(s, csum, nch, tr);
  double trace_resid = 0.0;
  QCHK(hipMemcpyAsync(&trace_resid, tr, sizeof(double), hipMemcpyDeviceToHost, s));
  const int64_t k_out = hs.k_r;
  if (k_out < k) QCHK(hipMemsetAsync(pivots + k_out, 0xff, sizeof(int64_t) * (size_t)(k - k_out), s));
  QCHK(hipStreamSynchronize(s));
  if (hbad) return ARPC_ENUMERIC;
  const arpc_status ret =
      (k_out == k || (max_rounds > 0 && hs.round >= max_rounds && hs.status == ST_DONE)) ? ARPC_OK : ARPC_EARLY_STOP;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->k_out = k_out;
    stats->rounds = hs.round;
    stats->proposals = hs.proposals;
    stats->status = ret;
    stats->trace_A = hs.trace_A;
    stats->trace_resid = trace_resid;
    for (int c = 0; c < ARPC_NUM_KC; ++c) {
      stats->ms_kernel[c] = prof.ms[c];
      stats->launches[c] = prof.n[c];
    }
    stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return ret;
}

}  // namespace
}  // namespace arpc

using namespace arpc;

extern "C" {

arpc_status arpc_qr_workspace_size(int64_t M, int64_t N, int64_t k, int64_t b, size_t* bytes) {
  const arpc_status v = qr_validate(M, N, k, b, 0);
  if (v != ARPC_OK) return v;
  if (!bytes) return ARPC_EINVAL;
  *bytes = qr_layout(M, N, k, b).total;
  return ARPC_OK;
}

arpc_status arpc_qr_factor(int64_t M, int64_t N, int64_t k, int64_t b, uint64_t seed, int64_t max_rounds,
                           const double* B, double* Q, double* F, int64_t* pivots, void* ws, size_t ws_bytes,
                           void* stream, arpc_stats* stats) {
  const arpc_status v = qr_validate(M, N, k, b, max_rounds);
  if (v != ARPC_OK) return v;
  if (!B || !Q || !F || !pivots || !ws) return ARPC_EINVAL;
  if (((uintptr_t)B & 7) || ((uintptr_t)Q & 7) || ((uintptr_t)F & 7) || ((uintptr_t)pivots & 7) ||
      ((uintptr_t)ws & 255))
    return ARPC_EINVAL;
  const QrLayout l = qr_layout(M, N, k, b);
  if (ws_bytes < l.total) return ARPC_EINVAL;
  return qr_run(M, N, k, b, seed, max_rounds, B, Q, F, pivots, (char*)ws, l, (hipStream_t)stream, stats);
}

}  // extern "C"
