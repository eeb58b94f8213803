// Matrix-core round products (internal).
#pragma once

#include "arpc_common.h"

namespace arpc {

// Rows per panel of the panel-blocked layout of the N-row operands.
constexpr int PH = 256;

// Device pointers and sizes of one factorization used by the matrix-core
// update GEMM and triangular solve.
struct MfmaRound {
  void* F;                 // N x k column-major output factor (storage per mode)
  void* Fb;                // the same factor in the panel-blocked layout (BF16 modes), or null
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
  const double* H;         // H as left by RejectionSampleSubmatrix (holds L(T,T), see LFactor)
  int b;
  int64_t kmax;
  void* C0;                // kernel columns for d > 16 (FP64 in the FP64 mode, else FP32; N x b
                           // column-major), or null
  const unsigned* X8;      // FP8 mode with d % 4 == 0: the rounded points as e4m3 codes (N x d
                           // bytes, row-major), or null
  const float* xn8;        // their squared norms (FP32), or null
  const unsigned char* Xp8;  // FP8 mode with the distances in the update GEMM's epilogue: the
                             // accepted points as e4m3 codes (b x d bytes), else null
  const float* ypn;        // their squared norms (FP32)
  const float* Fs32 = nullptr;   // F rows at the proposals in FP32 (F stored in FP32), ld fs32_ld(ldf)
};

// Device pointers and sizes of the one-kernel round product of the BF16
// modes (update GEMM, kernel columns, solve and stores in one launch).
struct FusedRound {
  void* F;                 // N x k column-major FP32 output factor
  void* Fb;                // panel-blocked BF16 planes of F (read and written)
  int64_t nkc;             // 32-column chunks per panel of Fb
  int64_t N;
  const double* X;         // N x d points
  int d;
  const double* Xp;        // s_r x d accepted points
  KParams kp;
  unsigned char* Bm1;      // F(S_r,:)^T in chunks
  unsigned char* Bm2;      // permuted inverse factor in chunks
  double* P;               // FP64 row norms of G (one group)
  int b;
  int ncbt;                // compiled column-block count (>= ceil(b/16))
  int grid;                // persistent workgroups
};

// Column-block count of the fused path for (prec, b), or -1 when the fused
// path does not apply (FP64/FP32 modes, b > 256).
int fused_ncbt(int prec, int b);
size_t fused_operand_bytes(int prec, int64_t kmax, int b);
// Arguments of the round product for one job (the round state at st), and
// its persistent grid given two workgroups per compute unit (grid2).
FusedArgs fused_args_of(int prec, const FusedRound& r, const RoundState* st);
int fused_grid_of(int prec, const FusedArgs& a, int grid2);
// F(S_r,:)^T chunks, the permuted inverse factor and the accepted points (one
// launch; bd: the largest b d of the table), then the round product, over a
// device table of n jobs with the same mode and column-block count (and, for
// the product, the same coordinate class d <= 8 or <= 16 and the same kernel
// form as `any`); grid: workgroups per job.
void launch_fused_prep_tab(hipStream_t s, int prec, const RoundJob* tab, int n, int ncbt, int64_t bd);
void launch_fused_round_tab(hipStream_t s, int prec, int ncbt, int d, const FusedArgs& any, const RoundJob* tab,
                            int n, int grid);

size_t mfma_operand_bytes(int prec, int64_t kmax, int b);
size_t mfma_blocked_bytes(int prec, int64_t N, int64_t cols);
int mfma_part_cols(int prec, int b);
void launch_mfma_prep(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st);
void launch_mfma_colgemm(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st);
// Kernel columns on the matrix cores for d > 16 (into r.C0, read by the
// update GEMM's epilogue).
bool mfma_dist_contraction(int d);
// FP8 mode: the kernel columns formed in the update GEMM's epilogue (no C0).
bool mfma_dist_in_epilogue(int d);
// X8 = e4m3 codes of the (already rounded) points Xq, xn = their squared
// norms in FP32; d % 4 == 0.
void launch_pack_e4m3(hipStream_t s, const double* Xq, int64_t N, int d, unsigned* X8, float* xn);
void launch_dist(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st);
void launch_mfma_trsm(hipStream_t s, int prec, const MfmaRound& r, const RoundState* st);

}  // namespace arpc
