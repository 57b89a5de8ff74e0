// Internal FP64 dense linear algebra on gfx950 (MFMA f64 16x16x4).
#pragma once
#include "common.h"

namespace krr {

// C[M x N] = alpha * A[M x K] * op(B) + beta * C, row-major with leading
// dimensions.  b_trans = true: B is N x K (C = A B^T); false: B is K x N.
// beta == 0 never reads C.
// With `scratch`, a GEMM whose output has few tiles and a long K is split
// over K into fixed slots that are then added in a fixed order
// (deterministic); gemm_scratch_bytes() is the scratch it may take.
int gemm_f64(bool b_trans, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
             int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
             hipStream_t s, Arena* scratch = nullptr);
size_t gemm_scratch_bytes(int64_t M, int64_t N, int64_t K, bool lower_only = false);
// As gemm_f64; a_trans = true reads A as K x M (C = A^T op(B)).
int gemm_f64_ex(bool a_trans, bool b_trans, int64_t M, int64_t N, int64_t K, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                int64_t ldc, hipStream_t s, Arena* scratch = nullptr, bool lower_only = false);

// C[M x N] = alpha A[M x K] B[K x N] + beta Cin (C and Cin may differ or
// coincide), for M <= 8 rows: the kernels gemm_f64 uses for such products
// (the matrix-core one from N = 65536 columns, else the column-sum one),
// with the beta term read from Cin.
int gemm_colsum_into(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                     const double* B, int64_t ldb, double beta, const double* Cin, double* C,
                     int64_t ldc, hipStream_t s);

// In-place lower Cholesky of the n x n SPD matrix A (row-major, lda):
// A = L L^T, L in the lower triangle (the strict upper triangle is left
// holding values of no meaning).  `info` (device int) receives 0 or the
// 1-based column of the first non-positive pivot.
int potrf_lower(int64_t n, double* A, int64_t lda, int* info, hipStream_t s);

// X <- L^{-1} for lower-triangular L (n x n, lda); X (n x n, ldx) must hold
// the identity on entry.
int tri_inv_lower(int64_t n, const double* L, int64_t lda, double* X, int64_t ldx,
                  hipStream_t s);

// potrf_lower and tri_inv_lower together: A = L L^T in place and X <- L^{-1}
// (X holds the identity on entry).  Block row k of the inverse is formed on
// a second stream as soon as block column k of L is final, overlapping the
// rest of the factorisation; returns once both are complete (it
// synchronises the second stream; s is joined behind it).
int potrf_inverse_lower(int64_t n, double* A, int64_t lda, int* info, double* X, int64_t ldx,
                        hipStream_t s);

// Solves L X = B in place for lower-triangular L (n x n, lda) and B
// (n x ncols, ldb): B <- L^{-1} B.
int trsm_lower_left(int64_t n, int64_t ncols, const double* L, int64_t lda, double* B,
                    int64_t ldb, hipStream_t s);

}  // namespace krr
