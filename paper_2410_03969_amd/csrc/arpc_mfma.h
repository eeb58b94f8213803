// Matrix-core round products (internal).
#pragma once

#include "arpc_common.h"

namespace arpc {

// Device pointers and sizes of one factorization used by the matrix-core
// update GEMM and triangular solve.
struct MfmaRound {
  void* F;                 // N x k column-major output factor (storage per mode)
  void* Fb;                // the same factor in the panel-blocked layout
  void* C;                 // panel-blocked scratch for A(:,S_r) - F F(S_r,:)^T (N x b)
  int64_t N;
  const double* X;         // N x d points
  int d;
  const double* Xp;        // s_r x d accepted points
  KParams kp;
  unsigned char* Bm1;      // F(S_r,:)^T in contraction chunks
  unsigned char* Bm2;      // Linv in contraction chunks
  int Ctot;                // b rounded up to a multiple of 16
  double* P;               // partial row norms, groups x N
  const double* Fs;        // F rows at the proposals, FP64, ld ldf
  int64_t ldf;
  const int32_t* acc;      // accepted local indices
  const double* L;         // Cholesky factor of H(T,T), column-major, ld b
  int b;
  int64_t kmax;
};

size_t mfma_operand_bytes(int prec, int64_t kmax, int b);
size_t mfma_blocked_bytes(int prec, int64_t N, int64_t cols);
int mfma_part_cols(int prec, int b);
void launch_mfma_prep(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st);
void launch_mfma_colgemm(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st);
void launch_mfma_trsm(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st);
void launch_prep_xp(hipStream_t s, const int32_t* acc, const int64_t* props, const double* X, int d,
                    double* Xp, const RoundState* st);

}  // namespace arpc
