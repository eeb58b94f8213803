// Dense FP64 building blocks on the gfx950 matrix cores, used by accelerated
// randomly pivoted QR (Alg. 5) and by the low-rank preconditioner of kernel
// ridge regression (Section 3.2):
//   - dgemm: C = alpha op(A) op(B) + beta C for column-major operands, with
//     the contraction optionally split over workgroups (partial products
//     summed afterwards in a fixed order, so results do not depend on timing);
//   - the inverse of a lower-triangular matrix, one workgroup per column;
//   - a blocked Cholesky factorization built from the two;
//   - dot products reduced in a fixed order into device memory.
//
// dgemm tiles C by 64 x 64 per workgroup of four wavefronts (32 x 32 each,
// 2 x 2 products of v_mfma_f64_16x16x4f64) and steps through the contraction
// 16 at a time: each chunk of op(A) and op(B) is staged in LDS, and the next
// chunk is loaded into registers while the current one is multiplied.
// Operand roles in the product: lane (g, l16) supplies op(B)(k, j0 + l16) as
// the first operand and op(A)(i0 + l16, k) as the second, k = 4 ks + g, so
// entry e of its accumulator is C(i0 + l16, j0 + g + 4 e): for fixed e the
// sixteen lanes of a group write sixteen consecutive rows of one column.
#include <hip/hip_runtime.h>

#include "arpc_common.h"
#include "arpc_dense.h"

namespace arpc {
namespace {

typedef double dd4 __attribute__((ext_vector_type(4)));

constexpr int GBM = 64, GBN = 64, GBK = 16, GPAD = 4;

struct GemmArgs {
  int64_t m, n, K, kper;
  double alpha, beta;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  double* part;   // splits > 1: partial products, split z at part + z m n (ld m)
};

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_dgemm(GemmArgs a) {
  __shared__ double As[GBK][GBM + GPAD];   // As[k][i] = op(A)(i0 + i, k0 + k)
  __shared__ double Bs[GBK][GBN + GPAD];   // Bs[k][j] = op(B)(k0 + k, j0 + j)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, l16 = lane & 15;
  const int64_t i0 = (int64_t)blockIdx.x * GBM, j0 = (int64_t)blockIdx.y * GBN;
  const int64_t kb = (int64_t)blockIdx.z * a.kper;
  const int64_t ke = (kb + a.kper < a.K) ? kb + a.kper : a.K;
  // per-thread staging coordinates: a k-contiguous operand is read 16 k at a
  // time per row (coalesced along k), an index-contiguous one 64 rows at a
  // time per k
  double ra[4], rb[4];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if constexpr (TA) {   // op(A)(i, k) = A[k + i lda]
        const int kk = tid & 15, ii = (tid >> 4) + 16 * r;
        const int64_t i = i0 + ii, k = k0 + kk;
        ra[r] = (i < a.m && k < ke) ? a.A[k + i * a.lda] : 0.0;
      } else {              // op(A)(i, k) = A[i + k lda]
        const int ii = tid & 63, kk = (tid >> 6) + 4 * r;
        const int64_t i = i0 + ii, k = k0 + kk;
        ra[r] = (i < a.m && k < ke) ? a.A[i + k * a.lda] : 0.0;
      }
      if constexpr (TB) {   // op(B)(k, j) = B[j + k ldb]
        const int jj = tid & 63, kk = (tid >> 6) + 4 * r;
        const int64_t j = j0 + jj, k = k0 + kk;
        rb[r] = (j < a.n && k < ke) ? a.B[j + k * a.ldb] : 0.0;
      } else {              // op(B)(k, j) = B[k + j ldb]
        const int kk = tid & 15, jj = (tid >> 4) + 16 * r;
        const int64_t j = j0 + jj, k = k0 + kk;
        rb[r] = (j < a.n && k < ke) ? a.B[k + j * a.ldb] : 0.0;
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if constexpr (TA) As[tid & 15][(tid >> 4) + 16 * r] = ra[r];
      else As[(tid >> 6) + 4 * r][tid & 63] = ra[r];
      if constexpr (TB) Bs[(tid >> 6) + 4 * r][tid & 63] = rb[r];
      else Bs[tid & 15][(tid >> 4) + 16 * r] = rb[r];
    }
  };
  dd4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = dd4{0.0, 0.0, 0.0, 0.0};
  const int wi = 32 * (w & 1), wj = 32 * (w >> 1);
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += GBK) {
    __syncthreads();   // the previous chunk's products are done with the LDS tiles
    stash();
    __syncthreads();
    if (k0 + GBK < ke) load(k0 + GBK);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int k = 4 * ks + g;
      double av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = As[k][wi + 16 * x + l16];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = Bs[k][wj + 16 * y + l16];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[y], av[x], acc[x][y], 0, 0, 0);
    }
  }
  // entry e of acc[x][y]: C(i0 + wi + 16 x + l16, j0 + wj + 16 y + g + 4 e)
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    const int64_t i = i0 + wi + 16 * x + l16;
    if (i >= a.m) continue;
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t j = j0 + wj + 16 * y + g + 4 * e;
        if (j >= a.n) continue;
        if (a.part) {
          a.part[(int64_t)blockIdx.z * a.m * a.n + i + j * a.m] = acc[x][y][e];
        } else {
          double* c = a.C + i + j * a.ldc;
          *c = a.beta == 0.0 ? a.alpha * acc[x][y][e] : a.alpha * acc[x][y][e] + a.beta * *c;
        }
      }
  }
}

// C = alpha (sum over z of the partial products, in order z = 0, 1, ...) + beta C.
__global__ __launch_bounds__(256) void k_dgemm_reduce(const double* __restrict__ part, int splits, int64_t m,
                                                      int64_t n, double alpha, double beta, double* __restrict__ C,
                                                      int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e % m, j = e / m;
  double v = 0.0;
  for (int z = 0; z < splits; ++z) v += part[(int64_t)z * m * n + e];
  double* c = C + i + j * ldc;
  *c = beta == 0.0 ? alpha * v : alpha * v + beta * *c;
}

// Column c of the inverse of the n x n lower-triangular L (n <= 4096): the
// solution of L x = e_c by column-oriented forward substitution, x in LDS;
// step t divides x_t by L(t, t) and subtracts x_t L(t+1:n, t) from the rest.
// Entries above the diagonal of the inverse are written as zeros.
__global__ __launch_bounds__(256) void k_trinv_lower(const double* __restrict__ L, int n, int64_t ldl,
                                                     double* __restrict__ Linv, int64_t ldi) {
  __shared__ double x[4096];
  const int c = blockIdx.x, tid = threadIdx.x;
  for (int i = tid; i < n; i += 256) x[i] = (i == c) ? 1.0 : 0.0;
  __syncthreads();
  for (int t = c; t < n; ++t) {
    const double xt = x[t] / L[t + (int64_t)t * ldl];
    for (int i = t + 1 + tid; i < n; i += 256) x[i] -= xt * L[i + (int64_t)t * ldl];
    __syncthreads();
    if (tid == 0) x[t] = xt;
    __syncthreads();
  }
  for (int i = tid; i < n; i += 256) Linv[i + (int64_t)c * ldi] = x[i];
}

// In-place lower Cholesky factor of the nb x nb diagonal block at G (ld ldg),
// right-looking, one workgroup; the strict upper triangle of the block is set
// to zero.  A non-positive pivot is replaced by 1 and reported in *bad.
__global__ __launch_bounds__(256) void k_chol_block(double* __restrict__ G, int nb, int64_t ldg, int* __restrict__ bad) {
  const int tid = threadIdx.x;
  for (int j = 0; j < nb; ++j) {
    __syncthreads();
    double dj = G[j + (int64_t)j * ldg];
    if (!(dj > 0.0)) {
      if (tid == 0) *bad = 1;
      dj = 1.0;
    }
    const double d = sqrt(dj);
    __syncthreads();
    for (int i = j + 1 + tid; i < nb; i += 256) G[i + (int64_t)j * ldg] /= d;
    if (tid == 0) G[j + (int64_t)j * ldg] = d;
    __syncthreads();
    const int m = nb - j - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int c = j + 1 + e / m, i = j + 1 + e % m;
      if (i >= c) G[i + (int64_t)c * ldg] -= G[i + (int64_t)j * ldg] * G[c + (int64_t)j * ldg];
    }
  }
  __syncthreads();
  for (int e = tid; e < nb * nb; e += 256) {
    const int c = e / nb, i = e % nb;
    if (i < c) G[i + (int64_t)c * ldg] = 0.0;
  }
}

// Dot products: partial sums of 2048-element blocks (a fixed tree inside the
// block), then their sum in block order.
constexpr int DOT_BLOCK = 2048;

__global__ __launch_bounds__(256) void k_dot_part(const double* __restrict__ x, const double* __restrict__ y,
                                                  int64_t n, double* __restrict__ part) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * DOT_BLOCK;
  double v = 0.0;
#pragma unroll
  for (int r = 0; r < DOT_BLOCK / 256; ++r) {
    const int64_t i = base + r * 256 + tid;
    if (i < n) v = fma(x[i], y[i], v);
  }
  red[tid] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ part, int64_t nb,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double v = 0.0;
  for (int64_t i = tid; i < nb; i += 256) v += part[i];
  red[tid] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) *out = red[0];
}

}  // namespace

int dgemm_splits(int64_t m, int64_t n, int64_t K, size_t part_elems) {
  const int64_t tiles = ((m + GBM - 1) / GBM) * ((n + GBN - 1) / GBN);
  int64_t s = (1024 + tiles - 1) / tiles;          // about four workgroups per compute unit
  const int64_t kmax = (K + 511) / 512;            // at least 512 of the contraction per split
  if (s > kmax) s = kmax;
  if (s > 64) s = 64;
  while (s > 1 && (size_t)(s * m * n) > part_elems) --s;
  return (int)(s < 1 ? 1 : s);
}

size_t dgemm_part_elems(int64_t m, int64_t n, int64_t K) { return (size_t)dgemm_splits(m, n, K, SIZE_MAX) * m * n; }

hipError_t dgemm(hipStream_t s, bool ta, bool tb, int64_t m, int64_t n, int64_t K, double alpha, const double* A,
                 int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* part,
                 size_t part_elems) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int splits = (K > 0 && part) ? dgemm_splits(m, n, K, part_elems) : 1;
  int64_t kper = K > 0 ? (K + splits - 1) / splits : 0;
  kper = (kper + GBK - 1) / GBK * GBK;
  GemmArgs a{m, n, K, kper, alpha, beta, A, lda, B, ldb, C, ldc, splits > 1 ? part : nullptr};
  const dim3 grid((unsigned)((m + GBM - 1) / GBM), (unsigned)((n + GBN - 1) / GBN), (unsigned)splits);
  if (ta && tb) hipLaunchKernelGGL((k_dgemm<true, true>), grid, dim3(256), 0, s, a);
  else if (ta) hipLaunchKernelGGL((k_dgemm<true, false>), grid, dim3(256), 0, s, a);
  else if (tb) hipLaunchKernelGGL((k_dgemm<false, true>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_dgemm<false, false>), grid, dim3(256), 0, s, a);
  if (splits > 1)
    hipLaunchKernelGGL(k_dgemm_reduce, dim3((unsigned)((m * n + 255) / 256)), dim3(256), 0, s, part, splits, m, n,
                       alpha, beta, C, ldc);
  return hipGetLastError();
}

void launch_trinv_lower(hipStream_t s, const double* L, int n, int64_t ldl, double* Linv, int64_t ldi) {
  hipLaunchKernelGGL(k_trinv_lower, dim3((unsigned)n), dim3(256), 0, s, L, n, ldl, Linv, ldi);
}

hipError_t chol_lower(hipStream_t s, double* M, int n, int64_t ldm, double* work, int* bad) {
  constexpr int NB = 64;
  double* Dinv = work;             // NB x NB inverse of the diagonal block
  double* T = work + NB * NB;      // (n - NB) x NB panel
  for (int j = 0; j < n; j += NB) {
    const int nb = n - j < NB ? n - j : NB;
    double* Ajj = M + j + (int64_t)j * ldm;
    hipLaunchKernelGGL(k_chol_block, dim3(1), dim3(256), 0, s, Ajj, nb, ldm, bad);
    const int rest = n - j - nb;
    if (rest > 0) {
      // panel A21 <- A21 L11^{-T}, then the trailing matrix A22 <- A22 - A21 A21^T
      launch_trinv_lower(s, Ajj, nb, ldm, Dinv, NB);
      double* A21 = M + (j + nb) + (int64_t)j * ldm;
      hipError_t e = dgemm(s, false, true, rest, nb, nb, 1.0, A21, ldm, Dinv, NB, 0.0, T, rest, nullptr, 0);
      if (e != hipSuccess) return e;
      e = hipMemcpy2DAsync(A21, sizeof(double) * ldm, T, sizeof(double) * rest, sizeof(double) * rest, nb,
                           hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
      e = dgemm(s, false, true, rest, rest, nb, -1.0, A21, ldm, A21, ldm, 1.0, M + (j + nb) + (int64_t)(j + nb) * ldm,
                ldm, nullptr, 0);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

size_t chol_work_elems(int n) { return (size_t)64 * 64 + (size_t)(n > 64 ? n - 64 : 0) * 64; }

void launch_chol_block(hipStream_t s, double* G, int nb, int64_t ldg, int* bad) {
  hipLaunchKernelGGL(k_chol_block, dim3(1), dim3(256), 0, s, G, nb, ldg, bad);
}

void launch_dot(hipStream_t s, const double* x, const double* y, int64_t n, double* part, double* out) {
  const int64_t nb = (n + DOT_BLOCK - 1) / DOT_BLOCK;
  hipLaunchKernelGGL(k_dot_part, dim3((unsigned)nb), dim3(256), 0, s, x, y, n, part);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, part, nb, out);
}

int64_t dot_part_elems(int64_t n) { return (n + DOT_BLOCK - 1) / DOT_BLOCK; }

}  // namespace arpc
