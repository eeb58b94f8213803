// Kernel ridge regression (Section 3.2): solve (A + mu I) beta = y by
// preconditioned conjugate gradients with the low-rank preconditioner
// P = F F^* + mu I, F the N x k factor of arpc_factor.
//
// The product with A + mu I regenerates the kernel entries on the fly (one
// thread per row, the other points staged through LDS 64 at a time; FP64,
// direct differences, the diagonal exactly kappa(0)).  P^{-1} r uses the
// Woodbury identity, (r - F (mu I + F^* F)^{-1} F^* r) / mu, with the k x k
// matrix formed once (rocBLAS dsyrk) and factored blockwise (the library's
// one-workgroup Cholesky on 64 x 64 diagonal blocks, rocBLAS dtrsm and dsyrk
// for the rest); the plain vector and matrix-vector products are rocBLAS.
// PCG is the textbook iteration from beta = 0 (Golub and Van Loan,
// Alg. 11.5.1); the host reads the scalars of each iteration.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <chrono>
#include <cmath>
#include <cstring>

#include "../../include/arpc.h"
#include "arpc_common.h"
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

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

struct KrrLayout {
  size_t Fd, M, D, t, r, z, p, q, part, bad, total;
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
  l.D = take(sizeof(double) * 64 * 64);
  l.t = take(sizeof(double) * (k > 0 ? k : 1));
  l.r = take(sizeof(double) * N);
  l.z = take(sizeof(double) * N);
  l.p = take(sizeof(double) * N);
  l.q = take(sizeof(double) * N);
  l.part = take(sizeof(double) * krr_parts(N) * N);
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
#define KBCHK(x)                                        \
  do {                                                  \
    if ((x) != rocblas_status_success) return ARPC_EDEVICE; \
  } while (0)

struct KHandle {
  rocblas_handle h = nullptr;
  ~KHandle() {
    if (h) (void)rocblas_destroy_handle(h);
  }
};

using clk = std::chrono::steady_clock;
inline double ms_since(clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); }

arpc_status krr_run(int64_t N, int64_t d, int32_t kernel, double bw, double mu, const double* X, const double* y,
                    const void* F, int32_t f_prec, int64_t k, double tol, int64_t max_iter, double* beta, char* ws,
                    const KrrLayout& l, hipStream_t s, arpc_krr_stats* stats) {
  const auto t0 = clk::now();
  KHandle hb;
  KBCHK(rocblas_create_handle(&hb.h));
  KBCHK(rocblas_set_stream(hb.h, s));
  rocblas_handle h = hb.h;
  arpc_problem pp{};
  pp.kernel = kernel;
  pp.bandwidth = bw;
  const KParams kp = kparams_of(pp);
  const double* Fd = (const double*)F;
  if (k > 0 && f_prec != ARPC_FP64) {
    hipLaunchKernelGGL(k_krr_to_f64, dim3(8192), dim3(256), 0, s, (const float*)F, (double*)(ws + l.Fd), N * k);
    Fd = (const double*)(ws + l.Fd);
  }
  double* M = (double*)(ws + l.M);
  double* t = (double*)(ws + l.t);
  double* r = (double*)(ws + l.r);
  double* z = (double*)(ws + l.z);
  double* p = (double*)(ws + l.p);
  double* q = (double*)(ws + l.q);
  int* bad = (int*)(ws + l.bad);
  const double one = 1.0, zero = 0.0;
  const unsigned gN = (unsigned)((N + 255) / 256);
  KCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
  if (k > 0) {   // M = L L^* = mu I + F^* F
    KBCHK(rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_transpose, (rocblas_int)k, (rocblas_int)N, &one, Fd,
                        (rocblas_int)N, &zero, M, (rocblas_int)k));
    hipLaunchKernelGGL(k_krr_add_diag, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, M, (int)k, mu);
    // blocked right-looking Cholesky, 64 columns at a time: the diagonal
    // block by the one-workgroup kernel (it reads and writes only that block,
    // which has leading dimension k here, so it is factored in a packed copy),
    // the panel below by a triangular solve, the trailing matrix by a
    // symmetric rank-64 update
    constexpr int NBK = 64;
    for (int64_t j = 0; j < k; j += NBK) {
      const int nb = (int)(k - j < NBK ? k - j : NBK);
      double* Ajj = M + j * k + j;
      double* Dp = (double*)(ws + l.D);
      KCHK(hipMemcpy2DAsync(Dp, sizeof(double) * nb, Ajj, sizeof(double) * k, sizeof(double) * nb, nb,
                            hipMemcpyDeviceToDevice, s));
      launch_dense_chol(s, Dp, nb, bad);
      KCHK(hipMemcpy2DAsync(Ajj, sizeof(double) * k, Dp, sizeof(double) * nb, sizeof(double) * nb, nb,
                            hipMemcpyDeviceToDevice, s));
      const int64_t rest = k - j - nb;
      if (rest > 0) {
        double* Aij = M + j * k + j + nb;            // rows below the block, its columns
        KBCHK(rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                            rocblas_diagonal_non_unit, (rocblas_int)rest, nb, &one, Ajj, (rocblas_int)k, Aij,
                            (rocblas_int)k));
        const double mone = -1.0;
        KBCHK(rocblas_dsyrk(h, rocblas_fill_lower, rocblas_operation_none, (rocblas_int)rest, nb, &mone, Aij,
                            (rocblas_int)k, &one, M + (j + nb) * k + j + nb, (rocblas_int)k));
      }
    }
  }
  // z = P^{-1} v
  auto precond = [&](const double* v, double* out) -> arpc_status {
    if (k == 0) {
      hipLaunchKernelGGL(k_krr_axpby, dim3(gN), dim3(256), 0, s, 1.0 / mu, v, 0.0, v, out, N);
      return ARPC_OK;
    }
    KBCHK(rocblas_dgemv(h, rocblas_operation_transpose, (rocblas_int)N, (rocblas_int)k, &one, Fd, (rocblas_int)N, v,
                        1, &zero, t, 1));
    KBCHK(rocblas_dtrsv(h, rocblas_fill_lower, rocblas_operation_none, rocblas_diagonal_non_unit, (rocblas_int)k, M,
                        (rocblas_int)k, t, 1));
    KBCHK(rocblas_dtrsv(h, rocblas_fill_lower, rocblas_operation_transpose, rocblas_diagonal_non_unit,
                        (rocblas_int)k, M, (rocblas_int)k, t, 1));
    KBCHK(rocblas_dgemv(h, rocblas_operation_none, (rocblas_int)N, (rocblas_int)k, &one, Fd, (rocblas_int)N, t, 1,
                        &zero, out, 1));
    hipLaunchKernelGGL(k_krr_axpby, dim3(gN), dim3(256), 0, s, 1.0 / mu, v, -1.0 / mu, out, out, N);
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
  auto dot = [&](const double* a, const double* b, double* res) -> arpc_status {
    KBCHK(rocblas_ddot(h, (rocblas_int)N, a, 1, b, 1, res));   // host result: waits for the stream
    return ARPC_OK;
  };
  double tm = 0.0, tp = 0.0;
  arpc_status e;
  // beta = 0, r = y, z = P^{-1} r, p = z
  KCHK(hipMemsetAsync(beta, 0, sizeof(double) * N, s));
  KCHK(hipMemcpyAsync(r, y, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  double yy = 0.0, rz = 0.0, rr = 0.0;
  if ((e = dot(y, y, &yy)) != ARPC_OK) return e;
  const double setup_ms = ms_since(t0);
  auto tq = clk::now();
  if ((e = precond(r, z)) != ARPC_OK) return e;
  KCHK(hipMemcpyAsync(p, z, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  if ((e = dot(r, z, &rz)) != ARPC_OK) return e;
  tp += ms_since(tq);
  const double ny = std::sqrt(yy);
  double rel = ny > 0 ? 1.0 : 0.0;
  int64_t it = 0;
  while (it < max_iter && rel > tol) {
    tq = clk::now();
    matvec(p, q);
    double pq = 0.0;
    if ((e = dot(p, q, &pq)) != ARPC_OK) return e;
    tm += ms_since(tq);
    const double alpha = rz / pq;
    hipLaunchKernelGGL(k_krr_axpby, dim3(gN), dim3(256), 0, s, 1.0, beta, alpha, p, beta, N);
    hipLaunchKernelGGL(k_krr_axpby, dim3(gN), dim3(256), 0, s, 1.0, r, -alpha, q, r, N);
    if ((e = dot(r, r, &rr)) != ARPC_OK) return e;
    ++it;
    rel = std::sqrt(rr) / ny;
    if (rel <= tol) break;
    tq = clk::now();
    if ((e = precond(r, z)) != ARPC_OK) return e;
    double rz_new = 0.0;
    if ((e = dot(r, z, &rz_new)) != ARPC_OK) return e;
    tp += ms_since(tq);
    hipLaunchKernelGGL(k_krr_axpby, dim3(gN), dim3(256), 0, s, 1.0, z, rz_new / rz, p, p, N);
    rz = rz_new;
  }
  KCHK(hipGetLastError());
  int hbad = 0;
  KCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  KCHK(hipStreamSynchronize(s));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->iterations = it;
    stats->rel_residual = rel;
    stats->ms_total = ms_since(t0);
    stats->ms_setup = setup_ms;
    stats->ms_matvec = tm;
    stats->ms_precond = tp;
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
