// The two N-sized products of each round of accelerated RPCholesky (Alg. 2,
// step 3):
//   colgemm:  C = A(:, S_r) - F F(S_r,:)^T      (N x s_r, K = k_r)
//   trsm:     G = C L^{-T} = C Linv^T           (N x s_r, K = s_r), G -> F columns
// Shapes k_r and s_r are read from the device-resident round state, so the
// grid is sized for the block size b and idle tiles exit at once.
#include "arpc_common.h"
#include "arpc_launch.h"

namespace arpc {

constexpr int TM = 64, TN = 64, TK = 16;

// Register-tiled product: each of 256 threads accumulates a 4 x 4 tile; rows
// tr + 16 i and columns tc + 16 j so that stores are coalesced along rows.
// A is column-major (ld lda), B row-major (ld ldb).
template <typename T>
__device__ inline void tile_product(const T* __restrict__ A, int64_t lda, int64_t M, int64_t row0,
                                    const T* __restrict__ B, int64_t ldb, int ncols, int col0, int64_t K,
                                    T (&acc)[4][4], T (*As)[TM + 1], T (*Bs)[TN + 1]) {
  const int tid = threadIdx.x, tr = tid & 15, tc = tid >> 4;
  for (int64_t k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = (tid >> 6) + 4 * q, r = tid & 63;
      const int64_t kg = k0 + kk, row = row0 + r;
      As[kk][r] = (row < M && kg < K) ? A[kg * lda + row] : (T)0;
      const int cc = col0 + r;
      Bs[kk][r] = (kg < K && cc < ncols) ? B[kg * ldb + cc] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      T a[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tr + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tc + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_colgemm(const T* __restrict__ F, int64_t N, const T* __restrict__ Bt,
                                                 int ldb, const double* __restrict__ X, int d,
                                                 const double* __restrict__ Xp, KParams kp, T* __restrict__ C,
                                                 const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  const int col0 = blockIdx.y * TN;
  if (col0 >= s) return;
  const int64_t K = st->k_r;
  const int64_t row0 = (int64_t)blockIdx.x * TM;
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (T)0;
  tile_product<T>(F, N, N, row0, Bt, ldb, s, col0, K, acc, As, Bs);
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = row0 + tr + 16 * i;
    if (row >= N) continue;
    const double* xr = X + row * d;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = col0 + tc + 16 * j;
      if (col >= s) continue;
      const double kap = kappa_r2(sqdist(xr, Xp + (int64_t)col * d, d), kp);
      C[(int64_t)col * N + row] = (T)(kap - (double)acc[i][j]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_trsm(const T* __restrict__ C, int64_t N, const T* __restrict__ Bt2,
                                              int b, T* __restrict__ F, double* __restrict__ P,
                                              const RoundState* st) {
  if (st->status != ST_RUNNING) return;
  const int s = st->s_r;
  const int col0 = blockIdx.y * TN;
  if (col0 >= s) return;
  const int64_t kr = st->k_r;
  const int64_t row0 = (int64_t)blockIdx.x * TM;
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  __shared__ double red[16][TM + 1];
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (T)0;
  // Linv^T is upper triangular: columns col0.. need t < min(s, col0 + TN)
  const int64_t K = (col0 + TN < s) ? col0 + TN : s;
  tile_product<T>(C, N, N, row0, Bt2, b, s, col0, K, acc, As, Bs);
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = row0 + tr + 16 * i;
    double g2 = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = col0 + tc + 16 * j;
      if (row < N && col < s) {
        const T g = acc[i][j];
        F[(kr + col) * N + row] = g;
        g2 += (double)g * (double)g;
      }
    }
    red[tc][tr + 16 * i] = g2;
  }
  __syncthreads();
  if (threadIdx.x < TM) {
    const int64_t row = row0 + threadIdx.x;
    double g2 = 0.0;
    for (int q = 0; q < 16; ++q) g2 += red[q][threadIdx.x];
    if (row < N) P[(int64_t)blockIdx.y * N + row] = g2;
  }
}

template <typename T>
void launch_colgemm(hipStream_t s, const T* F, int64_t N, const T* Bt, int ldb, const double* X, int d,
                    const double* Xp, KParams kp, T* C, int b, const RoundState* st) {
  dim3 grid((unsigned)((N + TM - 1) / TM), (unsigned)((b + TN - 1) / TN));
  hipLaunchKernelGGL(k_colgemm<T>, grid, dim3(256), 0, s, F, N, Bt, ldb, X, d, Xp, kp, C, st);
}

template <typename T>
void launch_trsm(hipStream_t s, const T* C, int64_t N, const T* Bt2, int b, T* F, double* P,
                 const RoundState* st) {
  dim3 grid((unsigned)((N + TM - 1) / TM), (unsigned)((b + TN - 1) / TN));
  hipLaunchKernelGGL(k_trsm<T>, grid, dim3(256), 0, s, C, N, Bt2, b, F, P, st);
}

template void launch_colgemm<double>(hipStream_t, const double*, int64_t, const double*, int, const double*, int,
                                     const double*, KParams, double*, int, const RoundState*);
template void launch_colgemm<float>(hipStream_t, const float*, int64_t, const float*, int, const double*, int,
                                    const double*, KParams, float*, int, const RoundState*);
template void launch_trsm<double>(hipStream_t, const double*, int64_t, const double*, int, double*, double*,
                                  const RoundState*);
template void launch_trsm<float>(hipStream_t, const float*, int64_t, const float*, int, float*, double*,
                                 const RoundState*);

}  // namespace arpc
