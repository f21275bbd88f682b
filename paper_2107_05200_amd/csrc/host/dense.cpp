// Host FP64 dense kernels for the one-time factorisation: a packed 8x6
// register-tiled GEMM (AVX2/FMA through GCC vector extensions), with
// Cholesky, triangular solve, triangular inverse and rank-k update built on
// it.  OpenMP parallelism inside GEMM when the call is large and not already
// inside a parallel region.
#include "dense.hpp"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace ffd {
namespace dense {

namespace {

typedef double v4d __attribute__((vector_size(32)));

constexpr int MR = 8;
constexpr int NR = 6;
constexpr int KC = 256;
constexpr int MC = 128;

inline v4d load4(const double* p) {
  v4d v;
  std::memcpy(&v, p, sizeof(v));
  return v;
}

// C(mr x nr) += alpha * Ap(8 x kc) * Bp(kc x 6), packed panels
inline void ukernel(int kc, const double* __restrict Ap, const double* __restrict Bp,
                    double* __restrict C, int64_t ldc, double alpha, int mr, int nr) {
  v4d c00 = {0, 0, 0, 0}, c01 = c00, c10 = c00, c11 = c00, c20 = c00, c21 = c00;
  v4d c30 = c00, c31 = c00, c40 = c00, c41 = c00, c50 = c00, c51 = c00;
  for (int p = 0; p < kc; ++p) {
    const v4d a0 = load4(Ap + 8 * p);
    const v4d a1 = load4(Ap + 8 * p + 4);
    const double* b = Bp + 6 * p;
    v4d bb;
    bb = (v4d){b[0], b[0], b[0], b[0]}; c00 += a0 * bb; c01 += a1 * bb;
    bb = (v4d){b[1], b[1], b[1], b[1]}; c10 += a0 * bb; c11 += a1 * bb;
    bb = (v4d){b[2], b[2], b[2], b[2]}; c20 += a0 * bb; c21 += a1 * bb;
    bb = (v4d){b[3], b[3], b[3], b[3]}; c30 += a0 * bb; c31 += a1 * bb;
    bb = (v4d){b[4], b[4], b[4], b[4]}; c40 += a0 * bb; c41 += a1 * bb;
    bb = (v4d){b[5], b[5], b[5], b[5]}; c50 += a0 * bb; c51 += a1 * bb;
  }
  double acc[6][8];
  std::memcpy(&acc[0][0], &c00, 32); std::memcpy(&acc[0][4], &c01, 32);
  std::memcpy(&acc[1][0], &c10, 32); std::memcpy(&acc[1][4], &c11, 32);
  std::memcpy(&acc[2][0], &c20, 32); std::memcpy(&acc[2][4], &c21, 32);
  std::memcpy(&acc[3][0], &c30, 32); std::memcpy(&acc[3][4], &c31, 32);
  std::memcpy(&acc[4][0], &c40, 32); std::memcpy(&acc[4][4], &c41, 32);
  std::memcpy(&acc[5][0], &c50, 32); std::memcpy(&acc[5][4], &c51, 32);
  for (int j = 0; j < nr; ++j)
    for (int i = 0; i < mr; ++i) C[i + j * ldc] += alpha * acc[j][i];
}

struct Aligned {
  double* p = nullptr;
  explicit Aligned(size_t n) { p = static_cast<double*>(std::aligned_alloc(64, ((n * 8 + 63) / 64) * 64)); }
  ~Aligned() { std::free(p); }
};

// generic packed GEMM: C += alpha * A * op(B), op(B)(p, j) = TB ? B[j + p*ldb] : B[p + j*ldb]
template <bool TB>
void gemm_core(int m, int n, int k, double alpha, const double* A, int64_t lda,
               const double* B, int64_t ldb, double* C, int64_t ldc) {
  if (m <= 0 || n <= 0 || k <= 0) return;
  const int npan = (n + NR - 1) / NR;
  const int nmb = (m + MC - 1) / MC;
  const double flops = 2.0 * m * n * k;
  const bool par = flops > 4e6 && !omp_in_parallel() && omp_get_max_threads() > 1;
  Aligned bpack(static_cast<size_t>(npan) * NR * KC);
  for (int p0 = 0; p0 < k; p0 += KC) {
    const int kc = std::min(KC, k - p0);
    // pack B: panel jp holds columns jp*NR .. +NR, row-major over p (6 per p)
#pragma omp parallel for schedule(static) if (par)
    for (int jp = 0; jp < npan; ++jp) {
      double* dst = bpack.p + static_cast<size_t>(jp) * NR * KC;
      for (int p = 0; p < kc; ++p)
        for (int jj = 0; jj < NR; ++jj) {
          const int j = jp * NR + jj;
          double v = 0.0;
          if (j < n) v = TB ? B[j + static_cast<int64_t>(p0 + p) * ldb] : B[(p0 + p) + static_cast<int64_t>(j) * ldb];
          dst[p * NR + jj] = v;
        }
    }
#pragma omp parallel if (par)
    {
      Aligned apack(static_cast<size_t>(MC) * KC);
#pragma omp for schedule(dynamic, 1)
      for (int mb = 0; mb < nmb; ++mb) {
        const int i0 = mb * MC;
        const int mc = std::min(MC, m - i0);
        const int nmp = (mc + MR - 1) / MR;
        for (int ip = 0; ip < nmp; ++ip) {
          double* dst = apack.p + static_cast<size_t>(ip) * MR * KC;
          for (int p = 0; p < kc; ++p) {
            const double* src = A + (i0 + ip * MR) + static_cast<int64_t>(p0 + p) * lda;
            const int rows = std::min(MR, mc - ip * MR);
            for (int ii = 0; ii < MR; ++ii) dst[p * MR + ii] = ii < rows ? src[ii] : 0.0;
          }
        }
        for (int jp = 0; jp < npan; ++jp) {
          const int nr = std::min(NR, n - jp * NR);
          const double* bp = bpack.p + static_cast<size_t>(jp) * NR * KC;
          for (int ip = 0; ip < nmp; ++ip) {
            const int mr = std::min(MR, mc - ip * MR);
            ukernel(kc, apack.p + static_cast<size_t>(ip) * MR * KC, bp,
                    C + (i0 + ip * MR) + static_cast<int64_t>(jp * NR) * ldc, ldc, alpha, mr, nr);
          }
        }
      }
    }
  }
}

void scale(int m, int n, double beta, double* C, int64_t ldc) {
  if (beta == 1.0) return;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) C[i + j * ldc] = beta == 0.0 ? 0.0 : beta * C[i + j * ldc];
}

int potrf_unblocked(int n, double* A, int64_t lda) {
  for (int j = 0; j < n; ++j) {
    double d = A[j + j * lda];
    for (int l = 0; l < j; ++l) d -= A[j + l * lda] * A[j + l * lda];
    if (!(d > 0.0) || !std::isfinite(d)) return j + 1;
    d = std::sqrt(d);
    A[j + j * lda] = d;
    const double inv = 1.0 / d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i + j * lda];
      for (int l = 0; l < j; ++l) s -= A[i + l * lda] * A[j + l * lda];
      A[i + j * lda] = s * inv;
    }
  }
  return 0;
}

// rows of B(m x jb) <- rows * L(jb x jb)^{-T}
void trsm_rlt_unblocked(int m, int jb, const double* L, int64_t ldl, double* B, int64_t ldb) {
  const bool par = static_cast<double>(m) * jb * jb > 2e5 && !omp_in_parallel();
#pragma omp parallel for schedule(static) if (par)
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < jb; ++j) {
      double x = B[i + j * ldb];
      for (int l = 0; l < j; ++l) x -= B[i + l * ldb] * L[j + l * ldl];
      B[i + j * ldb] = x / L[j + j * ldl];
    }
  }
}

}  // namespace

void gemm_nt(int m, int n, int k, double alpha, const double* A, int64_t lda,
             const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
  scale(m, n, beta, C, ldc);
  gemm_core<true>(m, n, k, alpha, A, lda, B, ldb, C, ldc);
}

void gemm_nn(int m, int n, int k, double alpha, const double* A, int64_t lda,
             const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
  scale(m, n, beta, C, ldc);
  gemm_core<false>(m, n, k, alpha, A, lda, B, ldb, C, ldc);
}

void syrk_sub(int n, int k, const double* A, int64_t lda, double* C, int64_t ldc) {
  constexpr int W = 384;
  for (int j0 = 0; j0 < n; j0 += W) {
    const int w = std::min(W, n - j0);
    gemm_core<true>(n - j0, w, k, -1.0, A + j0, lda, A + j0, lda, C + j0 + j0 * ldc, ldc);
  }
}

int potrf(int n, double* A, int64_t lda) {
  constexpr int NB = 96;
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = std::min(NB, n - j0);
    double* Ajj = A + j0 + j0 * lda;
    const int info = potrf_unblocked(jb, Ajj, lda);
    if (info) return j0 + info;
    const int rest = n - j0 - jb;
    if (rest > 0) {
      double* Aij = A + (j0 + jb) + j0 * lda;
      trsm_rlt_unblocked(rest, jb, Ajj, lda, Aij, lda);
      syrk_sub(rest, jb, Aij, lda, A + (j0 + jb) + (j0 + jb) * lda, lda);
    }
  }
  return 0;
}

void trsm_rlt(int m, int n, const double* L, int64_t ldl, double* B, int64_t ldb) {
  constexpr int NB = 96;
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = std::min(NB, n - j0);
    trsm_rlt_unblocked(m, jb, L + j0 + j0 * ldl, ldl, B + j0 * ldb, ldb);
    const int rest = n - j0 - jb;
    if (rest > 0)
      gemm_core<true>(m, rest, jb, -1.0, B + j0 * ldb, ldb, L + (j0 + jb) + j0 * ldl, ldl,
                      B + (j0 + jb) * ldb, ldb);
  }
}

void trtri(int n, const double* L, int64_t ldl, double* X, int64_t ldx) {
  if (n <= 64) {
    for (int j = 0; j < n; ++j) {
      for (int i = 0; i < j; ++i) X[i + j * ldx] = 0.0;
      X[j + j * ldx] = 1.0 / L[j + j * ldl];
      for (int i = j + 1; i < n; ++i) {
        double s = 0.0;
        for (int l = j; l < i; ++l) s += L[i + l * ldl] * X[l + j * ldx];
        X[i + j * ldx] = -s / L[i + i * ldl];
      }
    }
    return;
  }
  const int n1 = ((n / 2) + 7) / 8 * 8;
  const int n2 = n - n1;
  trtri(n1, L, ldl, X, ldx);
  trtri(n2, L + n1 + n1 * ldl, ldl, X + n1 + n1 * ldx, ldx);
  for (int j = n1; j < n; ++j)
    for (int i = 0; i < n1; ++i) X[i + j * ldx] = 0.0;
  // X21 = -X22 * (L21 * X11)
  std::vector<double> Tm(static_cast<size_t>(n2) * n1, 0.0);
  gemm_core<false>(n2, n1, n1, 1.0, L + n1, ldl, X, ldx, Tm.data(), n2);
  scale(n2, n1, 0.0, X + n1, ldx);
  gemm_core<false>(n2, n1, n2, -1.0, X + n1 + n1 * ldx, ldx, Tm.data(), n2, X + n1, ldx);
}

}  // namespace dense
}  // namespace ffd
