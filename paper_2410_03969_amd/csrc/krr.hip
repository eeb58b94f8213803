// Kernel ridge regression (Section 3.2): solve (A + mu I) beta = y by
// preconditioned conjugate gradients with the low-rank preconditioner
// P = F F^* + mu I, F the N x k factor of arpc_factor.
//
// The product with A + mu I regenerates the kernel entries on the fly (one
// thread per row, the other points staged through LDS 64 at a time; FP64,
// direct differences, the diagonal exactly kappa(0)).  P^{-1} r uses the
// Woodbury identity, (r - F (mu I + F^* F)^{-1} F^* r) / mu: the k x k
// matrix mu I + F^* F = L L^* is formed and factored once and L^{-1} is formed
// explicitly, so an application is four matrix-vector products (F^* r,
// L^{-1} t, L^{-*} t, F t), all on the library's FP64 matrix-core GEMM with
// contractions split over workgroups and summed in a fixed order.
// PCG is the textbook iteration from beta = 0 (Golub and Van Loan,
// Alg. 11.5.1) with its scalars kept on the device: dot products reduce in a
// fixed order into device memory, one-thread kernels form alpha and the
// direction update, and a device flag, set when |r| <= tol |y| or after
// max_iter iterations, turns the remaining kernels of the iteration and of
// later iterations into no-ops.  The host enqueues KRR_BATCH iterations at a
// time and reads the flag between batches.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "../../include/arpc.h"
#include "arpc_common.h"
#include "arpc_dense.h"
#include "arpc_host.h"
#include "arpc_launch.h"

namespace arpc {
namespace {

constexpr int KRR_DMAX = 128;   // staged coordinates: 64 points x d doubles in LDS
constexpr int KRR_JC = 64;

constexpr int KRR_PARTS_MAX = 32;   // column partitions of the product with A

// Column partitions for N rows: enough workgroups to fill the chip (one
// thread per row gives only N / 256 of them), each partition at least one
// staged chunk wide.
inline int krr_parts(int64_t N) {
  const int64_t rowblocks = (N + 255) / 256;
  int64_t p = (2048 + rowblocks - 1) / rowblocks;
  const int64_t pmax = (N + KRR_JC - 1) / KRR_JC;
  if (p > pmax) p = pmax;
  if (p > KRR_PARTS_MAX) p = KRR_PARTS_MAX;
  return (int)(p < 1 ? 1 : p);
}

// part(y, i) = sum over columns j of partition y (W columns from W y) of
// A(i, j) v(j), one thread per row.  XR: the row's coordinates in registers
// (d <= 16).
template <bool XR>
__global__ __launch_bounds__(256) void k_krr_matvec(const double* __restrict__ X, int d, KParams kp,
                                                    const double* __restrict__ v, int64_t N, int64_t W,
                                                    double* __restrict__ part) {
  __shared__ double xs[KRR_JC * KRR_DMAX];
  __shared__ double vs[KRR_JC];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  const double* xrow = X + (i < N ? i : N - 1) * d;
  double xr[16];
  if constexpr (XR) {
#pragma unroll
    for (int t = 0; t < 16; ++t) xr[t] = t < d ? xrow[t] : 0.0;
  }
  double acc = 0.0;
  const int64_t jbeg = (int64_t)blockIdx.y * W;
  const int64_t jend = jbeg + W < N ? jbeg + W : N;
  for (int64_t j0 = jbeg; j0 < jend; j0 += KRR_JC) {
    __syncthreads();
    const int64_t nq = (int64_t)KRR_JC * d;
    for (int64_t e = tid; e < nq; e += 256) {
      const int64_t q = j0 * d + e;
      xs[e] = q < jend * d ? X[q] : 0.0;
    }
    if (tid < KRR_JC) vs[tid] = j0 + tid < jend ? v[j0 + tid] : 0.0;
    __syncthreads();
    const int je = jend - j0 < KRR_JC ? (int)(jend - j0) : KRR_JC;
    for (int jj = 0; jj < je; ++jj) {
      const double* xp = xs + jj * d;
      double r2 = 0.0;
      if constexpr (XR) {
#pragma unroll
        for (int t = 0; t < 16; ++t)
          if (t < d) {
            const double e = xr[t] - xp[t];
            r2 += e * e;
          }
      } else {
        for (int t = 0; t < d; ++t) {
          const double e = xrow[t] - xp[t];
          r2 += e * e;
        }
      }
      acc = fma(kappa_r2(r2, kp), vs[jj], acc);
    }
  }
  if (i < N) part[(int64_t)blockIdx.y * N + i] = acc;
}

// out = (A + mu I) v: the partitions' sums added in partition order.
__global__ __launch_bounds__(256) void k_krr_sum(const double* __restrict__ part, int parts,
                                                 const double* __restrict__ v, double mu, int64_t N,
                                                 double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  double acc = 0.0;
  for (int p = 0; p < parts; ++p) acc += part[(int64_t)p * N + i];
  out[i] = fma(mu, v[i], acc);
}

// out(i) = a * x(i) + c * y(i)
__global__ __launch_bounds__(256) void k_krr_axpby(double a, const double* __restrict__ x, double c,
                                                   const double* __restrict__ y, double* __restrict__ out,
                                                   int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = a * x[i] + c * y[i];
}

__global__ __launch_bounds__(256) void k_krr_to_f64(const float* __restrict__ in, double* __restrict__ out,
                                                    int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = (double)in[i];
}

__global__ void k_krr_add_diag(double* __restrict__ M, int k, double mu) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < k) M[(int64_t)i * k + i] += mu;
}

// Device state of the PCG iteration.
struct PcgState {
  double yy, rz, pq, rr, rz_new, alpha, ny, rel;
  int64_t it, max_it;
  double tol;
  int32_t done, pad;
};

// rel and done after the initial residual r = y.
__global__ void k_pcg_start(PcgState* ps, int64_t max_it, double tol) {
  ps->ny = sqrt(ps->yy);
  ps->rel = ps->ny > 0.0 ? 1.0 : 0.0;
  ps->it = 0;
  ps->max_it = max_it;
  ps->tol = tol;
  ps->done = (ps->rel > tol) ? 0 : 1;
}

__global__ void k_pcg_alpha(PcgState* ps) {
  if (ps->done) return;
  ps->alpha = ps->rz / ps->pq;
}

// beta += alpha p, r -= alpha q
__global__ __launch_bounds__(256) void k_pcg_step(const PcgState* ps, const double* __restrict__ p,
                                                  const double* __restrict__ q, double* __restrict__ beta,
                                                  double* __restrict__ r, int64_t n) {
  if (ps->done) return;
  const double a = ps->alpha;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    beta[i] = fma(a, p[i], beta[i]);
    r[i] = fma(-a, q[i], r[i]);
  }
}

__global__ void k_pcg_check(PcgState* ps) {
  if (ps->done) return;
  ps->it += 1;
  ps->rel = sqrt(ps->rr) / ps->ny;
  if (!(ps->rel > ps->tol) || ps->it >= ps->max_it) ps->done = 1;
}

// z = (v - w) / mu  (w = F (mu I + F^* F)^{-1} F^* v), or v / mu without F
__global__ __launch_bounds__(256) void k_pcg_precond_out(const PcgState* ps, const double* __restrict__ v,
                                                         const double* __restrict__ w, double mu,
                                                         double* __restrict__ z, int64_t n) {
  if (ps && ps->done) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) z[i] = w ? (v[i] - w[i]) / mu : v[i] / mu;
}

// p = z + (rz_new / rz) p, rz = rz_new
__global__ __launch_bounds__(256) void k_pcg_dir(PcgState* ps, const double* __restrict__ z, double* __restrict__ p,
                                                 int64_t n) {
  if (ps->done) return;
  const double c = ps->rz_new / ps->rz;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = fma(c, p[i], z[i]);
}

__global__ void k_pcg_rz(PcgState* ps) {
  if (ps->done) return;
  ps->rz = ps->rz_new;
}

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr int KRR_BATCH = 8;   // iterations enqueued between host checks

struct KrrLayout {
  size_t Fd, M, Li, cw, t, t2, w, r, z, p, q, part, gpart, gpe, dpart, ps, bad, total;
};

KrrLayout krr_layout(int64_t N, int64_t k, bool convert) {
  KrrLayout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += al256(bytes);
    return o;
  };
  l.Fd = take(convert ? sizeof(double) * N * k : 0);
  l.M = take(sizeof(double) * k * k);
  l.Li = take(sizeof(double) * k * k);
  l.cw = take(sizeof(double) * chol_work_elems((int)k));
  l.t = take(sizeof(double) * (k > 0 ? k : 1));
  l.t2 = take(sizeof(double) * (k > 0 ? k : 1));
  l.w = take(sizeof(double) * N);
  l.r = take(sizeof(double) * N);
  l.z = take(sizeof(double) * N);
  l.p = take(sizeof(double) * N);
  l.q = take(sizeof(double) * N);
  l.part = take(sizeof(double) * krr_parts(N) * N);
  size_t gpe = 1;
  if (k > 0) {
    const size_t c[4] = {dgemm_part_elems(k, k, N), dgemm_part_elems(k, 1, N), dgemm_part_elems(N, 1, k),
                         dgemm_part_elems(k, 1, k)};
    for (size_t v : c) gpe = v > gpe ? v : gpe;
  }
  l.gpe = gpe;
  l.gpart = take(sizeof(double) * gpe);
  l.dpart = take(sizeof(double) * dot_part_elems(N));
  l.ps = take(sizeof(PcgState));
  l.bad = take(sizeof(int));
  l.total = off;
  return l;
}

arpc_status krr_validate(int64_t N, int64_t d, int32_t kernel, double bw, double mu, int64_t k, double tol,
                         int64_t max_iter) {
  if (N < 1 || N > 2147483647LL || d < 1 || d > KRR_DMAX || k < 0 || k > N || k > 2048) return ARPC_EINVAL;
  if (kernel < ARPC_GAUSSIAN || kernel > ARPC_MATERN52) return ARPC_EINVAL;
  if (!std::isfinite(bw) || !(bw > 0.0) || !std::isfinite(mu) || !(mu > 0.0)) return ARPC_EINVAL;
  if (!(tol > 0.0) || max_iter < 1) return ARPC_EINVAL;
  return ARPC_OK;
}

#define KCHK(x)                               \
  do {                                        \
    if ((x) != hipSuccess) return ARPC_EDEVICE; \
  } while (0)
using clk = std::chrono::steady_clock;
inline double ms_since(clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); }

arpc_status krr_run(int64_t N, int64_t d, int32_t kernel, double bw, double mu, const double* X, const double* y,
                    const void* F, int32_t f_prec, int64_t k, double tol, int64_t max_iter, double* beta, char* ws,
                    const KrrLayout& l, hipStream_t s, arpc_krr_stats* stats) {
  const auto t0 = clk::now();
  arpc_problem pp{};
  pp.kernel = kernel;
  pp.bandwidth = bw;
  const KParams kp = kparams_of(pp);
  // matrix-vector products timed as class colgemm, preconditioner applications as trsm
  Profiler prof(s, (1u << ARPC_KC_COLGEMM) | (1u << ARPC_KC_TRSM));
  const double* Fd = (const double*)F;
  if (k > 0 && f_prec != ARPC_FP64) {
    hipLaunchKernelGGL(k_krr_to_f64, dim3(8192), dim3(256), 0, s, (const float*)F, (double*)(ws + l.Fd), N * k);
    Fd = (const double*)(ws + l.Fd);
  }
  double* M = (double*)(ws + l.M);
  double* Li = (double*)(ws + l.Li);
  double* t = (double*)(ws + l.t);
  double* t2 = (double*)(ws + l.t2);
  double* w = (double*)(ws + l.w);
  double* r = (double*)(ws + l.r);
  double* z = (double*)(ws + l.z);
  double* p = (double*)(ws + l.p);
  double* q = (double*)(ws + l.q);
  double* gpart = (double*)(ws + l.gpart);
  double* dpart = (double*)(ws + l.dpart);
  PcgState* ps = (PcgState*)(ws + l.ps);
  int* bad = (int*)(ws + l.bad);
  const unsigned gN = (unsigned)((N + 255) / 256);
  const int ik = (int)k;
  KCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
  if (k > 0) {   // M = L L^* = mu I + F^* F, then Li = L^{-1}
    KCHK(dgemm(s, true, false, k, k, N, 1.0, Fd, N, Fd, N, 0.0, M, k, gpart, l.gpe));
    hipLaunchKernelGGL(k_krr_add_diag, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, M, ik, mu);
    KCHK(chol_lower(s, M, ik, k, (double*)(ws + l.cw), bad));
    launch_trinv_lower(s, M, ik, k, Li, k);
  }
  // z = P^{-1} v (skipped once the iteration has stopped, when ps is given)
  auto precond = [&](const double* v, double* out, const PcgState* gate) -> arpc_status {
    if (k > 0) {
      KCHK(dgemm(s, true, false, k, 1, N, 1.0, Fd, N, v, N, 0.0, t, k, gpart, l.gpe));     // t = F^* v
      KCHK(dgemm(s, false, false, k, 1, k, 1.0, Li, k, t, k, 0.0, t2, k, gpart, l.gpe));   // L^{-1} t
      KCHK(dgemm(s, true, false, k, 1, k, 1.0, Li, k, t2, k, 0.0, t, k, gpart, l.gpe));    // L^{-*} (L^{-1} t)
      KCHK(dgemm(s, false, false, N, 1, k, 1.0, Fd, N, t, k, 0.0, w, N, gpart, l.gpe));    // F M^{-1} F^* v
    }
    hipLaunchKernelGGL(k_pcg_precond_out, dim3(gN), dim3(256), 0, s, gate, v, k > 0 ? w : nullptr, mu, out, N);
    return ARPC_OK;
  };
  const int parts = krr_parts(N);
  const int64_t pw = ((N + parts - 1) / parts + KRR_JC - 1) / KRR_JC * KRR_JC;   // columns per partition
  double* part = (double*)(ws + l.part);
  auto matvec = [&](const double* v, double* out) {
    if (d <= 16)
      hipLaunchKernelGGL(k_krr_matvec<true>, dim3(gN, parts), dim3(256), 0, s, X, (int)d, kp, v, N, pw, part);
    else
      hipLaunchKernelGGL(k_krr_matvec<false>, dim3(gN, parts), dim3(256), 0, s, X, (int)d, kp, v, N, pw, part);
    hipLaunchKernelGGL(k_krr_sum, dim3(gN), dim3(256), 0, s, part, parts, v, mu, N, out);
  };
  arpc_status e;
  // beta = 0, r = y, z = P^{-1} r, p = z, rz = r.z
  KCHK(hipMemsetAsync(beta, 0, sizeof(double) * N, s));
  KCHK(hipMemcpyAsync(r, y, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  launch_dot(s, y, y, N, dpart, &ps->yy);
  hipLaunchKernelGGL(k_pcg_start, dim3(1), dim3(1), 0, s, ps, max_iter, tol);
  if ((e = precond(r, z, nullptr)) != ARPC_OK) return e;
  KCHK(hipMemcpyAsync(p, z, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  launch_dot(s, r, z, N, dpart, &ps->rz);
  KCHK(hipGetLastError());
  PcgState h{};
  KCHK(hipMemcpyAsync(&h, ps, sizeof(PcgState), hipMemcpyDeviceToHost, s));
  KCHK(hipStreamSynchronize(s));
  const double setup_ms = ms_since(t0);
  while (!h.done) {
    for (int b = 0; b < KRR_BATCH; ++b) {
      prof.begin(ARPC_KC_COLGEMM);
      matvec(p, q);
      prof.end();
      launch_dot(s, p, q, N, dpart, &ps->pq);
      hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(1), 0, s, ps);
      hipLaunchKernelGGL(k_pcg_step, dim3(gN), dim3(256), 0, s, ps, p, q, beta, r, N);
      launch_dot(s, r, r, N, dpart, &ps->rr);
      hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(1), 0, s, ps);
      prof.begin(ARPC_KC_TRSM);
      if ((e = precond(r, z, ps)) != ARPC_OK) return e;
      prof.end();
      launch_dot(s, r, z, N, dpart, &ps->rz_new);
      hipLaunchKernelGGL(k_pcg_dir, dim3(gN), dim3(256), 0, s, ps, z, p, N);
      hipLaunchKernelGGL(k_pcg_rz, dim3(1), dim3(1), 0, s, ps);
    }
    KCHK(hipGetLastError());
    KCHK(hipMemcpyAsync(&h, ps, sizeof(PcgState), hipMemcpyDeviceToHost, s));
    KCHK(hipStreamSynchronize(s));
    prof.collect();
  }
  int hbad = 0;
  KCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  KCHK(hipStreamSynchronize(s));
  const double rel = h.rel;
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->iterations = h.it;
    stats->rel_residual = rel;
    stats->ms_total = ms_since(t0);
    stats->ms_setup = setup_ms;
    stats->ms_matvec = prof.ms[ARPC_KC_COLGEMM];
    stats->ms_precond = prof.ms[ARPC_KC_TRSM];
    stats->status = rel <= tol ? ARPC_OK : ARPC_EARLY_STOP;
  }
  if (hbad || !std::isfinite(rel)) return ARPC_ENUMERIC;
  return rel <= tol ? ARPC_OK : ARPC_EARLY_STOP;
}

}  // namespace
}  // namespace arpc

using namespace arpc;

extern "C" {

arpc_status arpc_krr_workspace_size(int64_t N, int64_t d, int64_t k, int32_t f_prec, size_t* bytes) {
  if (N < 1 || d < 1 || d > KRR_DMAX || k < 0 || k > N || k > 2048 || !bytes) return ARPC_EINVAL;
  *bytes = krr_layout(N, k, f_prec != ARPC_FP64).total;
  return ARPC_OK;
}

arpc_status arpc_krr_pcg(int64_t N, int64_t d, int32_t kernel, double bandwidth, double mu, const double* X,
                         const double* y, const void* F, int32_t f_prec, int64_t k, double tol, int64_t max_iter,
                         double* beta, void* ws, size_t ws_bytes, void* stream, arpc_krr_stats* stats) {
  const arpc_status v = krr_validate(N, d, kernel, bandwidth, mu, k, tol, max_iter);
  if (v != ARPC_OK) return v;
  if (!X || !y || !beta || !ws || (k > 0 && !F)) return ARPC_EINVAL;
  if (((uintptr_t)X & 7) || ((uintptr_t)y & 7) || ((uintptr_t)beta & 7) || ((uintptr_t)ws & 255) ||
      ((uintptr_t)F & 3))
    return ARPC_EINVAL;
  const KrrLayout l = krr_layout(N, k, f_prec != ARPC_FP64);
  if (ws_bytes < l.total) return ARPC_EINVAL;
  return krr_run(N, d, kernel, bandwidth, mu, X, y, F, f_prec, k, tol, max_iter, beta, (char*)ws, l,
                 (hipStream_t)stream, stats);
}

}  // extern "C"
