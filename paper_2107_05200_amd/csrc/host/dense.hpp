// Host FP64 dense kernels used by the one-time factorisation of the global
// matrix.  Column-major storage throughout.
#pragma once
#include <cstdint>

namespace ffd {
namespace dense {

// C(m x n) = beta*C + alpha * A(m x k) * B(n x k)^T
void gemm_nt(int m, int n, int k, double alpha, const double* A, int64_t lda,
             const double* B, int64_t ldb, double beta, double* C, int64_t ldc);

// C(m x n) = beta*C + alpha * A(m x k) * B(k x n)
void gemm_nn(int m, int n, int k, double alpha, const double* A, int64_t lda,
             const double* B, int64_t ldb, double beta, double* C, int64_t ldc);

// lower triangle of C(n x n) -= A(n x k) A^T; the strict upper part may be
// overwritten with garbage
void syrk_sub(int n, int k, const double* A, int64_t lda, double* C, int64_t ldc);

// in-place lower Cholesky A = L L^T; returns 0, or j+1 if pivot j is not
// positive (then A is partially overwritten)
int potrf(int n, double* A, int64_t lda);

// B(m x n) <- B * L^{-T}, L (n x n) lower triangular
void trsm_rlt(int m, int n, const double* L, int64_t ldl, double* B, int64_t ldb);

// X(n x n) = L^{-1} (lower triangular, strict upper part of X set to 0)
void trtri(int n, const double* L, int64_t ldl, double* X, int64_t ldx);

}  // namespace dense
}  // namespace ffd
