// Host-side launchers of the library's kernels (internal).
#pragma once

#include "arpc_common.h"

namespace arpc {

void launch_init(hipStream_t s, double* u, double* csum, const double* X, int64_t N, int d, KParams kp,
                 RoundState* st, int64_t nchunks);
// Round state and chunk sums from a residual diagonal u already in place
// (the state must have been zeroed; a set nonfinite flag stops the run).
void launch_init_from_diag(hipStream_t s, const double* u, int64_t N, double* csum, RoundState* st,
                           int64_t nchunks);
// Xq = X with every coordinate rounded to FP8 e4m3 (the FP8 mode's points), n values.
void launch_round_e4m3(hipStream_t s, const double* X, double* Xq, int64_t n);
// The same rounding with the e4m3 codes and FP32 norms of the rows (d % 4 == 0)
// and the non-finite flag in st, in one pass.
void launch_round_pack_e4m3(hipStream_t s, const double* X, int64_t N, int d, double* Xq, unsigned* X8, float* xn,
                            RoundState* st);
void launch_propose(hipStream_t s, const double* u, const double* csum, double* cpre, int64_t nchunks,
                    int64_t N, int b, Unif un, RoundState* st, int64_t* props);
// Partitions of the contraction index in the product F(S',:) F(S',:)^T of
// H (its partial products are summed in partition order); Hp holds
// gather_splits(kmax) * b * b doubles.
int gather_splits(int64_t kmax);
// Contraction columns per partition of Hp at this kmax.
int64_t gather_width(int64_t kmax);
// H = kappa(X(props), X(props)) (b x b, column-major), direct differences in FP64.
void launch_kernel_block(hipStream_t s, const double* X, int d, KParams kp, const int64_t* props, int b, double* H,
                         const RoundState* st);
// RejectionSampleSubmatrix (keep_all: block RPCholesky, every distinct proposal
// with a positive residual); L(T,T) is left in H (see LFactor).
void launch_reject(hipStream_t s, double* H, int b, const int64_t* props, Unif un, RoundState* st,
                   int32_t* acc, int64_t* pivots, double* u, int64_t kmax, bool keep_all);
template <typename T>
void launch_prep(hipStream_t s, const double* Fs, int64_t ldf, const int32_t* acc, const int64_t* props,
                 const double* X, int d, T* Bt, int ldb, double* Xp, const double* H, int b, T* Bt2,
                 int64_t kmax, const RoundState* st);
void launch_diag(hipStream_t s, double* u, double* csum, const double* P, int part_cols, int64_t N,
                 int64_t nchunks, const RoundState* st);
void launch_finish(hipStream_t s, RoundState* st, int b, int64_t kmax, int64_t max_rounds, int32_t* hist);
void launch_trace(hipStream_t s, const double* csum, int64_t nchunks, double* out);

// The same round steps over a device table of n jobs (RoundJob rows; one
// launch per step serves them all, row blockIdx.y per workgroup).  The grid
// of each step is the largest any row needs; rows that need fewer workgroups
// leave the rest idle.
struct RoundGrid {
  unsigned propose, gather_rows, gather_hp, gather_hs, diag;
};
RoundGrid round_grid_of(const RoundJob& j);
void round_grid_max(RoundGrid& g, const RoundGrid& other);
void launch_propose_tab(hipStream_t s, const RoundJob* tab, int n, const RoundGrid& g);
// fdouble: F is FP64; tiled: the residual submatrix form for d > 32
void launch_gather_tab(hipStream_t s, const RoundJob* tab, int n, const RoundGrid& g, bool fdouble, bool tiled);
void launch_reject_tab(hipStream_t s, const RoundJob* tab, int n, int bmax);
void launch_prep_xp_tab(hipStream_t s, const RoundJob* tab, int n, int64_t bd);   // bd: the largest b d
unsigned prep_xp_blocks(int64_t bd);   // its workgroups: one element per thread
void launch_diag_tab(hipStream_t s, const RoundJob* tab, int n, const RoundGrid& g);
void launch_finish_tab(hipStream_t s, const RoundJob* tab, int n);
// *dst = j by a kernel (graph-capturable; j need not outlive the call).
void launch_store_job(hipStream_t s, const RoundJob& j, RoundJob* dst);
// Zero columns k_r .. k-1 of F (es-byte elements, N rows) and set pivots
// k_r .. k-1 to -1, k_r read from the round state on the device.
void launch_zero_tail(hipStream_t s, const RoundState* st, int64_t k, int64_t N, int es, void* F, int64_t* pivots);
// out[i] = *tab[i].st for i < n (out: pinned host memory).
void launch_collect_tab(hipStream_t s, const RoundJob* tab, int n, RoundState* out);

// Update GEMM (Alg. 2 step 3, first factor): C = A(:,S_r) - F F(S_r,:)^T,
// kernel columns evaluated from the points in the epilogue.
template <typename T>
void launch_colgemm(hipStream_t s, const T* F, int64_t N, const T* Bt, int ldb, const double* X, int d,
                    const double* Xp, KParams kp, T* C, int b, const RoundState* st);
// Triangular solve as a product with the explicit inverse: G = C Linv^T,
// written into F(:, k_r : k_r + s_r), with FP64 partial row norms of G as stored.
template <typename T>
void launch_trsm(hipStream_t s, const T* C, int64_t N, const T* Bt2, int b, T* F, double* P,
                 const RoundState* st);

}  // namespace arpc
