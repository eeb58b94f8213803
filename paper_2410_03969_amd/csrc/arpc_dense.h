// Dense FP64 building blocks on the matrix cores (internal): general matrix
// product, lower-triangular inverse, Cholesky factorization, dot product.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace arpc {

// C (m x n) = alpha op(A) op(B) + beta C, every matrix column-major; op(A) is
// m x K (A itself K x m when ta), op(B) is K x n (B itself n x K when tb).
// With beta == 0, C is not read.  part (part_elems doubles, may be null)
// lets the contraction be split over workgroups; the partial products are
// then summed in a fixed order by a second kernel.  C must not overlap A or B.
hipError_t dgemm(hipStream_t s, bool ta, bool tb, int64_t m, int64_t n, int64_t K, double alpha, const double* A,
                 int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, double* part,
                 size_t part_elems);
// Contraction splits dgemm uses for these sizes, and the partial-product
// space that lets it use all of them.
int dgemm_splits(int64_t m, int64_t n, int64_t K, size_t part_elems);
size_t dgemm_part_elems(int64_t m, int64_t n, int64_t K);

// Linv (n x n, ld ldi) = inverse of the lower-triangular n x n L (ld ldl),
// n <= 4096; zeros above the diagonal.  Linv must not overlap L.
void launch_trinv_lower(hipStream_t s, const double* L, int n, int64_t ldl, double* Linv, int64_t ldi);

// In-place lower Cholesky factor of the n x n symmetric positive definite M
// (lower triangle read; the strict upper triangle is overwritten with
// partial products and must be ignored), blocked by 64 columns.  work:
// chol_work_elems(n) doubles.  A non-positive pivot sets *bad.
hipError_t chol_lower(hipStream_t s, double* M, int n, int64_t ldm, double* work, int* bad);
size_t chol_work_elems(int n);
// The same for one block of at most a few hundred columns, in one workgroup;
// the strict upper triangle becomes zero.
void launch_chol_block(hipStream_t s, double* G, int nb, int64_t ldg, int* bad);

// *out = sum_i x_i y_i, reduced in a fixed order; part: dot_part_elems(n) doubles.
void launch_dot(hipStream_t s, const double* x, const double* y, int64_t n, double* part, double* out);
int64_t dot_part_elems(int64_t n);

}  // namespace arpc
