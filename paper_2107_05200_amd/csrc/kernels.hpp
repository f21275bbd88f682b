// gfx950 kernels of the flip-free ADMM iteration.  One wave64 lane per
// element for the local steps; one lane per vertex row for the W-step
// right-hand side; per-level dense panel products for the triangular solves.
// No atomics: every reduction has a fixed order, so runs are bitwise
// reproducible.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_math.hpp"
#include "host/setup.hpp"  // the device panel layout (kPanelTile)

namespace ffd {

constexpr int kBlock = 256;      // threads per block for element / vertex kernels
constexpr int kNumSums = 9;       // per-block partial sums of the local step (fields 0 .. 8)
constexpr int kNumPartials = 11;  // ... followed by two per-block maxima (fields 9, 10)

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// fixed-order block reduction: fields below NSUM are summed, the others take
// the maximum (fmax: NaN entries are neutral)
template <int NF, int BS = kBlock, int NSUM = NF>
__device__ __forceinline__ void block_reduce_store(double (&v)[NF], double* __restrict out) {
  __shared__ double red[BS / 64][NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    double x = v[f];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double y = __shfl_down(x, off, 64);
      x = f < NSUM ? x + y : fmax(x, y);
    }
    v[f] = x;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int f = 0; f < NF; ++f) red[wave][f] = v[f];
  }
  __syncthreads();
  if (threadIdx.x < NF) {
    const bool sum = static_cast<int>(threadIdx.x) < NSUM;
    double s = sum ? 0.0 : red[0][threadIdx.x];
#pragma unroll
    for (int wv = sum ? 0 : 1; wv < BS / 64; ++wv) s = sum ? s + red[wv][threadIdx.x] : fmax(s, red[wv][threadIdx.x]);
    out[threadIdx.x] = s;
  }
}

// the local step's partials: sums, then maxima; a NaN is the neutral value of a maximum
__device__ __forceinline__ void partials_init(double (&v)[kNumPartials]) {
#pragma unroll
  for (int f = 0; f < kNumPartials; ++f) v[f] = f < kNumSums ? 0.0 : __longlong_as_double(0x7ff8000000000000LL);
}
// nf = kNumSums (an iteration without diagnostics: the maxima are not read) or kNumPartials
__device__ __forceinline__ void partials_add(double (&v)[kNumPartials], const double* __restrict p, int nf) {
#pragma unroll
  for (int f = 0; f < kNumPartials; ++f)
    if (f < nf) v[f] = f < kNumSums ? v[f] + p[f] : fmax(v[f], p[f]);
}

// element state sizes: U (2D: cos, sin; 3D: 9), P (sym: 3 / 6), Lambda d*d
template <int D> struct Sz;
template <> struct Sz<2> { static constexpr int U = 2, P = 3, L = 4, G = 6; };
template <> struct Sz<3> { static constexpr int U = 9, P = 6, L = 9, G = 12; };

template <int D, typename R>
__device__ __forceinline__ void load_P(const R* __restrict P, int64_t m, int64_t e, R out[D][D]) {
  if constexpr (D == 2) {
    out[0][0] = P[e];
    out[0][1] = out[1][0] = P[m + e];
    out[1][1] = P[2 * m + e];
  } else {
    out[0][0] = P[e];
    out[0][1] = out[1][0] = P[m + e];
    out[0][2] = out[2][0] = P[2 * m + e];
    out[1][1] = P[3 * m + e];
    out[1][2] = out[2][1] = P[4 * m + e];
    out[2][2] = P[5 * m + e];
  }
}

template <int D, typename R>
__device__ __forceinline__ void store_P(R* __restrict P, int64_t m, int64_t e, const R in[D][D]) {
  if constexpr (D == 2) {
    P[e] = in[0][0];
    P[m + e] = in[0][1];
    P[2 * m + e] = in[1][1];
  } else {
    P[e] = in[0][0];
    P[m + e] = in[0][1];
    P[2 * m + e] = in[0][2];
    P[3 * m + e] = in[1][1];
    P[4 * m + e] = in[1][2];
    P[5 * m + e] = in[2][2];
  }
}

template <int D, typename R>
__device__ __forceinline__ void load_U(const R* __restrict U, int64_t m, int64_t e, R out[D][D]) {
  if constexpr (D == 2) {
    const R c = U[e], s = U[m + e];
    out[0][0] = c;
    out[0][1] = -s;
    out[1][0] = s;
    out[1][1] = c;
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i / 3][i % 3] = U[i * m + e];
  }
}

template <int D, typename R>
__device__ __forceinline__ void store_U(R* __restrict U, int64_t m, int64_t e, const R in[D][D]) {
  if constexpr (D == 2) {
    U[e] = in[0][0];
    U[m + e] = in[1][0];
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) U[i * m + e] = in[i / 3][i % 3];
  }
}

template <int D, typename R>
__device__ __forceinline__ void matmul(const R A[D][D], const R B[D][D], R C[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < D; ++k) s += A[i][k] * B[k][j];
      C[i][j] = s;
    }
}

// P = V diag(p) V^T
template <int D, typename R>
__device__ __forceinline__ void spectral(const R V[D][D], const R p[D], R P[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i; j < D; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < D; ++k) s += V[i][k] * p[k] * V[j][k];
      P[i][j] = s;
      P[j][i] = s;
    }
}

template <int D, typename R>
__device__ __forceinline__ R det(const R J[D][D]) {
  if constexpr (D == 2) return J[0][0] * J[1][1] - J[0][1] * J[1][0];
  else
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// |adj(J)|^2 = |J^{-1}|^2 det(J)^2
template <int D, typename R>
__device__ __forceinline__ R adj_norm2(const R J[D][D]) {
  if constexpr (D == 2) return J[0][0] * J[0][0] + J[0][1] * J[0][1] + J[1][0] * J[1][0] + J[1][1] * J[1][1];
  else {
    R s = R(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        const R cf = J[i1][j1] * J[i2][j2] - J[i1][j2] * J[i2][j1];
        s += cf * cf;
      }
    return s;
  }
}

// closest rotation to Q; for a tie (Q == 0) the previous rotation is kept
template <int D, typename R>
__device__ __forceinline__ void rotation(const R Q[D][D], R U[D][D]) {
  if constexpr (D == 2) {
    const R zr = Q[0][0] + Q[1][1];
    const R zi = Q[1][0] - Q[0][1];
    const R nz2 = zr * zr + zi * zi;
    if (nz2 > R(0)) {
      const R inv = dm::rsqrt_(nz2);
      const R c = zr * inv, s = zi * inv;
      U[0][0] = c;
      U[0][1] = -s;
      U[1][0] = s;
      U[1][1] = c;
    }
  } else {
    R n2 = R(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) n2 += Q[i][j] * Q[i][j];
    if (!(n2 > R(0))) return;
    R W[3][3], sg[3], V[3][3];
    dm::svd3(Q, W, sg, V);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) U[i][j] = W[i][0] * V[j][0] + W[i][1] * V[j][1] + W[i][2] * V[j][2];
  }
}

// symmetric eigen-decomposition of a D x D symmetric matrix
template <int D, typename R>
__device__ __forceinline__ void sym_eig(R S[D][D], R q[D], R V[D][D]) {
  if constexpr (D == 2) dm::eig2(S[0][0], S[0][1], S[1][1], q, V);
  else dm::eig3(S, q, V);
}

// The Lambda-ratio proxy of the figure with the UV-mapping bounds for one
// element: |L1 - L0| / |1/2 (L1 - L0 + U1 L1^T U1 - U0 L0^T U0)|, with
// |L1 - L0|^2 = num2 (the element's primal residual); +inf for a zero
// denominator with a positive numerator, 0 when both vanish.
template <int D, typename R>
__device__ __forceinline__ double lambda_ratio(const R (&U0)[D][D], const R (&L0)[D][D], const R (&U1)[D][D],
                                               const R (&L1)[D][D], double num2) {
  double den2 = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      // (U L^T U)[a][b] = sum_ij U[a][i] L[j][i] U[j][b]
      double t1 = 0.0, t0 = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
          t1 += static_cast<double>(U1[a][i]) * static_cast<double>(L1[j][i]) * static_cast<double>(U1[j][b]);
          t0 += static_cast<double>(U0[a][i]) * static_cast<double>(L0[j][i]) * static_cast<double>(U0[j][b]);
        }
      const double q = 0.5 * ((static_cast<double>(L1[a][b]) - static_cast<double>(L0[a][b])) + t1 - t0);
      den2 += q * q;
    }
  if (den2 > 0.0) return sqrt(num2 / den2);
  return num2 > 0.0 ? __longlong_as_double(0x7ff0000000000000LL) : 0.0;
}

// corner vectors of G^T r: g[c][k] = sum_a C[a][c] r[a][k], C[:,0] = -sum_j B[:,j]
template <int D, typename R>
__device__ __forceinline__ void store_g(R* __restrict g, int64_t e, const R Bm[D][D], const R r[D][D]) {
  R out[(D + 1) * D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    R s0 = R(0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      R s = R(0);
#pragma unroll
      for (int a = 0; a < D; ++a) s += Bm[a][j] * r[a][k];
      out[(j + 1) * D + k] = s;
      s0 += s;
    }
    out[k] = -s0;
  }
  R* dst = g + e * (D + 1) * D;
#pragma unroll
  for (int i = 0; i < (D + 1) * D; ++i) dst[i] = out[i];
}

template <int D, typename R>
__device__ __forceinline__ void load_B(const R* __restrict B, int64_t m, int64_t e, R Bm[D][D]) {
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int j = 0; j < D; ++j) Bm[a][j] = B[(a * D + j) * m + e];
}

// ---------------------------------------------------------------------------
// K1: initialisation (Section "Implementation", "Initializing U, P, Lambda")
// ---------------------------------------------------------------------------
template <int D, typename R, int ENERGY>
__global__ __launch_bounds__(kBlock) void k_init(int64_t m, int64_t e0, int64_t e1, const int32_t* __restrict T,
                                                 const double* __restrict B64,
                                                 const R* __restrict Bm_, const R* __restrict w, R rho,
                                                 const double* __restrict x, R* __restrict U, R* __restrict P,
                                                 R* __restrict Lam, R* __restrict gnorm2, R* __restrict g) {
  const int64_t e = e0 + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= e1) return;
  double x0[D], E[D][D];
  const int32_t v0 = T[e];
#pragma unroll
  for (int k = 0; k < D; ++k) x0[k] = x[static_cast<int64_t>(v0) * D + k];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int32_t vj = T[(j + 1) * m + e];
#pragma unroll
    for (int k = 0; k < D; ++k) E[j][k] = x[static_cast<int64_t>(vj) * D + k] - x0[k];
  }
  double Jd[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) s += B64[(a * D + j) * m + e] * E[j][k];
      Jd[a][k] = s;
    }
  // flip decision in float64: det J0 <= 0
  const bool flipped = !(det<D, double>(Jd) > 0.0);
  R J[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int k = 0; k < D; ++k) J[a][k] = static_cast<R>(Jd[a][k]);
  const R eps = static_cast<R>(ENERGY == 1 ? dm::kInitEpsSG : dm::kInitEpsSD);
  R Ur[D][D], Pm[D][D], sv[D];
  if constexpr (D == 2) {
    // SVD J = [u0 u1] diag(s0, s1) V2^T: V2 from the eigenvectors of J^T J
    // (sorted descending, kept a rotation), u0 = J v0 / |J v0|, u1 = u0 turned
    // by 90 degrees, s1 = u1 . J v1 signed (negative when det J < 0)
    const R a = J[0][0], b = J[0][1], c = J[1][0], d = J[1][1];
    R q[2], V2[2][2];
    dm::eig2(a * a + c * c, a * b + c * d, b * b + d * d, q, V2);
    if (q[0] < q[1]) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const R t = V2[i][0];
        V2[i][0] = -V2[i][1];
        V2[i][1] = t;
      }
    }
    const R c0[2] = {a * V2[0][0] + b * V2[1][0], c * V2[0][0] + d * V2[1][0]};
    const R c1[2] = {a * V2[0][1] + b * V2[1][1], c * V2[0][1] + d * V2[1][1]};
    const R n0 = dm::sqrt_(c0[0] * c0[0] + c0[1] * c0[1]);
    R u0[2];
    if (n0 > R(0)) {
      u0[0] = c0[0] / n0;
      u0[1] = c0[1] / n0;
    } else {
      u0[0] = V2[0][0];
      u0[1] = V2[1][0];
    }
    const R u1[2] = {-u0[1], u0[0]};
    sv[0] = n0;
    sv[1] = u1[0] * c1[0] + u1[1] * c1[1];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) Ur[i][j] = u0[i] * V2[j][0] + u1[i] * V2[j][1];
#pragma unroll
    for (int j = 0; j < 2; ++j) sv[j] = flipped ? eps : (sv[j] > eps ? sv[j] : eps);
    spectral<2, R>(V2, sv, Pm);
  } else {
    R W[3][3], V3[3][3];
    dm::svd3(J, W, sv, V3);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Ur[i][j] = W[i][0] * V3[j][0] + W[i][1] * V3[j][1] + W[i][2] * V3[j][2];
#pragma unroll
    for (int j = 0; j < 3; ++j) sv[j] = flipped ? eps : (sv[j] > eps ? sv[j] : eps);
    spectral<3, R>(V3, sv, Pm);
  }
  store_U<D, R>(U, m, e, Ur);
  store_P<D, R>(P, m, e, Pm);
#pragma unroll
  for (int i = 0; i < D * D; ++i) Lam[i * m + e] = R(0);
  R gn = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const R p = sv[j];
    const R gj = ENERGY == 1 ? p - R(1) / p : p - R(1) / (p * p * p);
    gn += gj * gj;
  }
  gnorm2[e] = gn;
  // r0 = mu (U0 P0 - 0)
  R Bm[D][D], UP[D][D], r[D][D];
  load_B<D, R>(Bm_, m, e, Bm);
  matmul<D, R>(Ur, Pm, UP);
  const R mu = rho * w[e];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int k = 0; k < D; ++k) r[a][k] = mu * UP[a][k];
  store_g<D, R>(g, e, Bm, r);
}

// r = mu (U P - Lambda) -> corner vectors (after the state is set from outside)
template <int D, typename R, int ENERGY>
__global__ __launch_bounds__(kBlock) void k_prepare(int64_t m, int64_t e0, int64_t e1, const R* __restrict Bm_,
                                                    const R* __restrict w, R rho_u, const R* __restrict rho_e,
                                                    const R* __restrict U, const R* __restrict P,
                                                    const R* __restrict Lam, R* __restrict gnorm2, R* __restrict g) {
  const int64_t e = e0 + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= e1) return;
  const R rho = rho_e ? rho_e[e] : rho_u;  // mu_e / w_e
  R Ur[D][D], Pm[D][D], UP[D][D], Bm[D][D], r[D][D];
  load_U<D, R>(U, m, e, Ur);
  load_P<D, R>(P, m, e, Pm);
  load_B<D, R>(Bm_, m, e, Bm);
  matmul<D, R>(Ur, Pm, UP);
  const R mu = rho * w[e];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int k = 0; k < D; ++k) r[a][k] = mu * (UP[a][k] - Lam[(a * D + k) * m + e]);
  store_g<D, R>(g, e, Bm, r);
  R q[D], V[D][D];
  sym_eig<D, R>(Pm, q, V);
  R gn = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const R p = q[j];
    const R gj = ENERGY == 1 ? p - R(1) / p : p - R(1) / (p * p * p);
    gn += gj * gj;
  }
  gnorm2[e] = gn;
}

// ---------------------------------------------------------------------------
// K2: W-step right-hand side b = (G^T r)_F - L_FC x_C (eq. solvinginw), float64
// accumulation; LPR lanes (2, 4 or 8, picked by the autotuner) per vertex row share its incidence list and are
// combined by a fixed shuffle tree.  Rows >= nF copy the pinned positions into
// the new map.
// ---------------------------------------------------------------------------
// Block index that gives each of the 8 XCDs (blocks are dispatched to them
// round-robin by index) a contiguous eighth of the blocks, so that rows
// sharing data share an L2; a bijection on [0, gridDim.x) (the blocks past
// the largest multiple of 8 keep their index).
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t per = gridDim.x / 8, b = blockIdx.x;
  return b < 8 * per ? (b % 8) * per + b / 8 : b;
}

template <int D, typename R, int LPR = 4>
__global__ __launch_bounds__(kBlock) void k_wrhs(int64_t nF, int64_t n, const int32_t* __restrict dt_ptr,
                                                 const int32_t* __restrict dt_idx, const R* __restrict g,
                                                 const int32_t* __restrict pin_ptr, const int32_t* __restrict pin_col,
                                                 const double* __restrict pin_val, const double* __restrict xC,
                                                 double* __restrict b, double* __restrict xnew) {
  const int64_t t = xcd_block() * kBlock + threadIdx.x;
  const int64_t j = t / LPR;
  const int sub = static_cast<int>(t % LPR);
  if (j >= n) return;
  if (j >= nF) {
    if (sub == 0)
#pragma unroll
      for (int k = 0; k < D; ++k) xnew[j * D + k] = xC[(j - nF) * D + k];
    return;
  }
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  const int32_t s = dt_ptr[j], e = dt_ptr[j + 1];
  for (int32_t q = s + sub; q < e; q += LPR) {
    const int64_t o = static_cast<int64_t>(dt_idx[q]) * D;
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += static_cast<double>(g[o + k]);
  }
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int off = 1; off < LPR; off <<= 1) acc[k] += __shfl_xor(acc[k], off, 64);
  if (sub != 0) return;
  for (int32_t q = pin_ptr[j]; q < pin_ptr[j + 1]; ++q) {
    const double v = pin_val[q];
    const int64_t c = pin_col[q];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] -= v * xC[c * D + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) b[j * D + k] = acc[k];
}

// ---------------------------------------------------------------------------
// K4 / K5: level-scheduled triangular solves with the node panels
// [Linv; -M] ((c + r) x c): forward y = Linv v, u = carried - M v (v = the
// node's right-hand side plus its children's update vectors, gathered by the
// extend-add pull lists; carried = the children's update rows that pass
// through this node); backward x_C = [Linv^T | -M^T] [y; x_R].
//
// The lanes of a wave sit on OPT consecutive OUTPUTS (OPT = 64, 32 or 16,
// chosen per level so that the level offers enough blocks) times 64 / OPT
// inner streams; the NW waves of a block (4, 8 or 16) add streams, so a block
// runs NS = NW * 64 / OPT interleaved streams over its inner range and every
// wave load reads 64 / OPT runs of OPT contiguous doubles (whole 128-byte
// lines).  The forward reads a copy of the panel tiled by 64 output rows,
// the backward a copy tiled by 64 output columns: a task's entries are one
// contiguous tile, its columns (rows) of height ld = the tile's height.  The first batch of panel loads is issued before the
// LDS staging of the inner vector so the gather latency overlaps the stream.
// Streams are added in a fixed order.  Levels that still offer too few blocks
// split the inner ranges into chunks whose partials are added in chunk order
// (no atomics; bitwise reproducible) by a reduction kernel, or by waves of a
// later launch (see fwd_y_reduce and bwd_entry).  Panel entries are read with
// non-temporal loads: each is used once per pass, and keeping them out of
// the caches leaves L2 to the gathered inner vectors.
// ---------------------------------------------------------------------------
constexpr int kSolveOutMax = 64;  // outputs per task at most (partial slot stride)
static_assert(kSolveOutMax == kPanelTile, "a task's outputs lie in one panel tile");

// entry (output, inner) of a tiled panel copy (the layout of panel_tile_index)
__device__ __forceinline__ int64_t panel_tile_index_dev(int64_t out, int64_t in, int64_t nout, int64_t nin) {
  const int64_t t = out / kPanelTile, base = t * kPanelTile;
  const int64_t h = nout - base < kPanelTile ? nout - base : kPanelTile;
  return base * nin + in * h + (out - base);
}
constexpr int kSolveKC = 512;     // inner entries staged in LDS at a time
constexpr int kSolveBatch = 8;    // panel loads in flight per lane

// One block of a solve level (or one wave of a reduction), self-contained so
// a block starts streaming after a single scalar load.
struct SolveTask {
  int64_t pf;                // node panel offset (both copies)
  int64_t poff, uoff, soff;  // node: pull-list base, update-vector base, struct-index base
  int32_t ld;                // leading dimension of the copy the pass reads
  int32_t first, c, nf;      // node: first internal row, pivots, c + r
  int32_t out0, lo, hi;      // outputs [out0, out0 + OPT) of the pass, inner range [lo, hi)
  int32_t slot, nk;          // slot < 0: final outputs; else partial slot (reduction: nk slots from slot)
  int32_t pad[3];
};
static_assert(sizeof(SolveTask) == 80, "SolveTask layout");

// Carried part of forward rows: the children's update rows that extend-add
// into row ra of a node's front (pull-list entry ra, when ea) are added to aa
// in pull order, and likewise for row rb into ab.  The two rows' chains run
// side by side and the first two pulls of each are fetched together (pull
// range, then both indices, then both update rows: three dependent loads,
// which covers every row of a binary dissection tree); further pulls follow
// one at a time.
template <int D>
__device__ __forceinline__ void fwd_carried2(const int32_t* __restrict pull_ptr, const int32_t* __restrict pull_idx,
                                             const double* __restrict ub, int64_t ra, bool ea, double (&aa)[D],
                                             int64_t rb, bool eb, double (&ab)[D]) {
  int32_t qa0 = 0, qa1 = 0, qb0 = 0, qb1 = 0;
  if (ea) {
    qa0 = pull_ptr[ra];
    qa1 = pull_ptr[ra + 1];
  }
  if (eb) {
    qb0 = pull_ptr[rb];
    qb1 = pull_ptr[rb + 1];
  }
  int32_t ia[2], ib[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    ia[u] = qa0 + u < qa1 ? pull_idx[qa0 + u] : -1;
    ib[u] = qb0 + u < qb1 ? pull_idx[qb0 + u] : -1;
  }
  double va[2][D], vb[2][D];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      va[u][k] = ia[u] >= 0 ? ub[static_cast<int64_t>(ia[u]) * D + k] : 0.0;
      vb[u][k] = ib[u] >= 0 ? ub[static_cast<int64_t>(ib[u]) * D + k] : 0.0;
    }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      if (ia[u] >= 0) aa[k] += va[u][k];
      if (ib[u] >= 0) ab[k] += vb[u][k];
    }
  for (int32_t q = qa0 + 2; q < qa1; ++q) {
    const int64_t o = static_cast<int64_t>(pull_idx[q]) * D;
#pragma unroll
    for (int k = 0; k < D; ++k) aa[k] += ub[o + k];
  }
  for (int32_t q = qb0 + 2; q < qb1; ++q) {
    const int64_t o = static_cast<int64_t>(pull_idx[q]) * D;
#pragma unroll
    for (int k = 0; k < D; ++k) ab[k] += ub[o + k];
  }
}

// carried part of forward output i (an update row) alone
template <int D>
__device__ __forceinline__ void fwd_carried(const SolveTask& tk, int i, const int32_t* __restrict pull_ptr,
                                            const int32_t* __restrict pull_idx, const double* __restrict ub,
                                            double (&cv)[D]) {
  double none[D];
#pragma unroll
  for (int k = 0; k < D; ++k) none[k] = 0.0;
  fwd_carried2<D>(pull_ptr, pull_idx, ub, tk.poff + i, true, cv, 0, false, none);
}

template <int D>
__device__ __forceinline__ void fwd_store(const SolveTask& tk, int i, const double (&acc)[D],
                                          double* __restrict y, double* __restrict ub) {
  if (i < tk.c) {
#pragma unroll
    for (int k = 0; k < D; ++k) y[static_cast<int64_t>(tk.first + i) * D + k] = acc[k];
  } else {
#pragma unroll
    for (int k = 0; k < D; ++k) ub[(tk.uoff + i - tk.c) * D + k] = acc[k];
  }
}

// Stream the panel entries of inner range [lo, hi) of one block: acc +=
// sum_j P(out, j) v_j with v staged chunk by chunk into LDS by `stage`.
// Lane stream st covers j = lo + st, lo + st + NS, ... in order.
template <int D, int NS, typename Stage>
__device__ __forceinline__ void solve_stream(const double* __restrict base, int64_t ld, bool live, int lo, int hi,
                                             int st, double (&vs)[kSolveKC][D], double (&acc)[D], Stage stage) {
  for (int j0 = lo; j0 < hi; j0 += kSolveKC) {
    const int jn = min(kSolveKC, hi - j0);
    const double* __restrict p0 = base + static_cast<int64_t>(j0) * ld;
    double pv[kSolveBatch];
#pragma unroll
    for (int u = 0; u < kSolveBatch; ++u) {
      const int jj = st + u * NS;
      pv[u] = (live && jj < jn) ? __builtin_nontemporal_load(p0 + static_cast<int64_t>(jj) * ld) : 0.0;
    }
    stage(j0, jn);
    __syncthreads();
    for (int jb = 0; jb < jn; jb += kSolveBatch * NS) {
      double pn[kSolveBatch];
#pragma unroll
      for (int u = 0; u < kSolveBatch; ++u) {
        const int jj = jb + kSolveBatch * NS + st + u * NS;
        pn[u] = (live && jj < jn) ? __builtin_nontemporal_load(p0 + static_cast<int64_t>(jj) * ld) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kSolveBatch; ++u) {
        const int jj = jb + st + u * NS;
        if (jj < jn) {
#pragma unroll
          for (int k = 0; k < D; ++k) acc[k] += pv[u] * vs[jj][k];
        }
      }
#pragma unroll
      for (int u = 0; u < kSolveBatch; ++u) pv[u] = pn[u];
    }
    __syncthreads();
  }
}

// sum of the NS streams of each output in stream order; valid for threads < OPT
template <int D, int OPT, int NW>
__device__ __forceinline__ void solve_streams_sum(double (&acc)[D], int o, int st) {
  constexpr int NS = NW * (64 / OPT);
  __shared__ double red[NS][OPT][D];
#pragma unroll
  for (int k = 0; k < D; ++k) red[st][o][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < OPT) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < NS; ++q) v += red[q][threadIdx.x][k];
      acc[k] = v;
    }
  }
}

template <int D, int OPT, int NW>
__global__ __launch_bounds__(NW * 64) void k_solve_fwd(const SolveTask* __restrict tasks,
                                                       const double* __restrict Pcol,
                                                       const int32_t* __restrict pull_ptr,
                                                       const int32_t* __restrict pull_idx, const double* __restrict b,
                                                       double* __restrict y, double* __restrict ub,
                                                       double* __restrict part) {
  constexpr int NS = NW * (64 / OPT);
  __shared__ double vs[kSolveKC][D];
  const SolveTask tk = tasks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int o = lane % OPT, st = wave * (64 / OPT) + lane / OPT;
  const int i = tk.out0 + o;
  const bool live = i < tk.nf;
  double cv[D], acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) cv[k] = acc[k] = 0.0;
  // the carried part of this thread's output row is gathered side by side
  // with the first chunk's staging (in a pass of its own for a thread that
  // stages no row)
  bool cv_todo = tk.slot < 0 && threadIdx.x < OPT && live && i >= tk.c;
  auto stage = [&](int j0, int jn) {
    for (int t = threadIdx.x; t < jn || cv_todo; t += NW * 64) {
      const bool sg = t < jn;
      double a[D];
#pragma unroll
      for (int k = 0; k < D; ++k) a[k] = sg ? b[static_cast<int64_t>(tk.first + j0 + t) * D + k] : 0.0;
      fwd_carried2<D>(pull_ptr, pull_idx, ub, tk.poff + j0 + t, sg, a, tk.poff + i, cv_todo, cv);
      cv_todo = false;
      if (sg) {
#pragma unroll
        for (int k = 0; k < D; ++k) vs[t][k] = a[k];
      }
    }
  };
  solve_stream<D, NS>(Pcol + tk.pf + i, tk.ld, live, tk.lo, tk.hi, st, vs, acc, stage);
  if (cv_todo) fwd_carried<D>(tk, i, pull_ptr, pull_idx, ub, cv);
  solve_streams_sum<D, OPT, NW>(acc, o, st);
  if (threadIdx.x >= OPT || !live) return;
  if (tk.slot >= 0) {
#pragma unroll
    for (int k = 0; k < D; ++k) part[(static_cast<int64_t>(tk.slot) * kSolveOutMax + o) * D + k] = acc[k];
  } else {
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += cv[k];
    fwd_store<D>(tk, i, acc, y, ub);
  }
}

// one wave per split output block: add its nk chunk partials in order
template <int D>
__global__ __launch_bounds__(kBlock) void k_solve_fwd_reduce(const SolveTask* __restrict tasks, int ntasks,
                                                             const int32_t* __restrict pull_ptr,
                                                             const int32_t* __restrict pull_idx,
                                                             double* __restrict y, double* __restrict ub,
                                                             const double* __restrict part) {
  const int t = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (t >= ntasks) return;
  const SolveTask tk = tasks[t];
  const int lane = threadIdx.x & 63;
  const int i = tk.out0 + lane;
  if (lane >= tk.hi || i >= tk.nf) return;  // hi: outputs of the block
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int q = 0; q < tk.nk; ++q)
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += part[(static_cast<int64_t>(tk.slot + q) * kSolveOutMax + lane) * D + k];
  if (i >= tk.c) fwd_carried<D>(tk, i, pull_ptr, pull_idx, ub, acc);
  fwd_store<D>(tk, i, acc, y, ub);
}

// A split forward task only ever covers y rows (outputs < c), so its chunk
// partials are added lazily: by one wave of a later backward launch that
// precedes the backward pass over the same node (extra blocks or waves at the
// end of that launch's grid).
template <int D>
__device__ __forceinline__ void fwd_y_reduce(const SolveTask& tk, int lane, const double* __restrict fpart,
                                             double* y) {
  const int i = tk.out0 + lane;
  if (lane >= tk.hi || i >= tk.c) return;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int q = 0; q < tk.nk; ++q)
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += fpart[(static_cast<int64_t>(tk.slot + q) * kSolveOutMax + lane) * D + k];
#pragma unroll
  for (int k = 0; k < D; ++k) y[static_cast<int64_t>(tk.first + i) * D + k] = acc[k];
}

// The backward counterpart: a split backward level may leave its chunk
// partials to the next backward launch.  Its tasks read the pending rows
// straight from the partials (an entry of the structure list coded
// -(1 + (slot << 12 | lane << 6 | (nk - 1))) instead of a row index), and
// waves appended to its grid write those rows of x for the launches after it.
constexpr int kDeferNkMax = 64, kDeferSlotLimit = 1 << 19;

template <int D>
__device__ __forceinline__ void bwd_x_reduce(const SolveTask& tk, int lane, const double* __restrict part,
                                             double* x) {
  const int j = tk.out0 + lane;
  if (lane >= tk.hi || j >= tk.c) return;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int q = 0; q < tk.nk; ++q)
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += part[(static_cast<int64_t>(tk.slot + q) * kSolveOutMax + lane) * D + k];
#pragma unroll
  for (int k = 0; k < D; ++k) x[static_cast<int64_t>(tk.first + j) * D + k] = acc[k];
}

// inner-vector entry p of a backward task: its own y row, an ancestor's x
// row, or an ancestor's row still held as chunk partials (added in the
// reduction's order, so the value is the one bwd_x_reduce writes)
template <int D>
__device__ __forceinline__ void bwd_entry(const SolveTask& tk, int p, const int32_t* __restrict sidx, const double* y,
                                          const double* x, const double* __restrict part, double (&v)[D]) {
  if (p < tk.c) {
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = y[static_cast<int64_t>(tk.first + p) * D + k];
    return;
  }
  const int32_t e = sidx[tk.soff + p - tk.c];
  if (e >= 0) {
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = x[static_cast<int64_t>(e) * D + k];
    return;
  }
  const uint32_t code = static_cast<uint32_t>(-(e + 1));
  const int nk = static_cast<int>(code & 63u) + 1, lane = static_cast<int>((code >> 6) & 63u);
  const int64_t slot = static_cast<int64_t>(code >> 12);
#pragma unroll
  for (int k = 0; k < D; ++k) v[k] = 0.0;
  for (int q = 0; q < nk; ++q)
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] += part[((slot + q) * kSolveOutMax + lane) * D + k];
}

// waves appended to a backward launch: pending forward y-row reductions
// [0, nyred), then pending backward x-row reductions [nyred, nyred + nxred)
template <int D>
__device__ __forceinline__ void bwd_appended(int t, int lane, const SolveTask* __restrict yred, int nyred,
                                             const double* __restrict fpart, double* y,
                                             const SolveTask* __restrict xred, int nxred,
                                             const double* __restrict part, double* x) {
  if (t < nyred) fwd_y_reduce<D>(yred[t], lane, fpart, y);
  else if (t - nyred < nxred) bwd_x_reduce<D>(xred[t - nyred], lane, part, x);
}

template <int D, int OPT, int NW>
__global__ __launch_bounds__(NW * 64) void k_solve_bwd(const SolveTask* __restrict tasks, int nmain,
                                                       const double* __restrict Prow, const int32_t* __restrict sidx,
                                                       double* y, double* x, double* part,
                                                       const SolveTask* __restrict yred, int nyred,
                                                       const double* __restrict fpart,
                                                       const SolveTask* __restrict xred, int nxred,
                                                       const double* xpart) {
  constexpr int NS = NW * (64 / OPT);
  __shared__ double vs[kSolveKC][D];
  if (static_cast<int>(blockIdx.x) >= nmain) {  // the whole block: pending reductions
    const int t = (static_cast<int>(blockIdx.x) - nmain) * NW + static_cast<int>(threadIdx.x >> 6);
    bwd_appended<D>(t, threadIdx.x & 63, yred, nyred, fpart, y, xred, nxred, xpart, x);
    return;
  }
  const SolveTask tk = tasks[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int o = lane % OPT, st = wave * (64 / OPT) + lane / OPT;
  const int j = tk.out0 + o;
  const bool live = j < tk.c;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  auto stage = [&](int p0, int pn) {
    for (int t = threadIdx.x; t < pn; t += NW * 64) {
      double v[D];
      bwd_entry<D>(tk, p0 + t, sidx, y, x, xpart, v);
#pragma unroll
      for (int k = 0; k < D; ++k) vs[t][k] = v[k];
    }
  };
  solve_stream<D, NS>(Prow + tk.pf + j, tk.ld, live, tk.lo, tk.hi, st, vs, acc, stage);
  solve_streams_sum<D, OPT, NW>(acc, o, st);
  if (threadIdx.x >= OPT || !live) return;
  if (tk.slot >= 0) {
#pragma unroll
    for (int k = 0; k < D; ++k) part[(static_cast<int64_t>(tk.slot) * kSolveOutMax + o) * D + k] = acc[k];
  } else {
#pragma unroll
    for (int k = 0; k < D; ++k) x[static_cast<int64_t>(tk.first + j) * D + k] = acc[k];
  }
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_solve_bwd_reduce(const SolveTask* __restrict tasks, int ntasks,
                                                             double* __restrict x, const double* __restrict part) {
  const int t = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if (t >= ntasks) return;
  bwd_x_reduce<D>(tasks[t], threadIdx.x & 63, part, x);
}

// Wave-per-task form for levels of small nodes: each wave owns one task (OPT
// outputs x 64 / OPT streams), stages its inner vector 64 entries at a time in
// a wave-private LDS slice and adds its streams with a fixed xor tree.  There
// is no block barrier, so a CU keeps up to 32 independent tasks in flight.
constexpr int kWaveKC = 64;
constexpr int kWavePF = 16;   // panel entries per lane loaded before the gather (backward)
constexpr int kWavePFf = 8;   // forward: its two pull chains need the registers

// orders this wave's LDS writes before its later LDS reads (LDS operations of
// one wave complete in order; the fences keep the compiler from moving them)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int D, int OPT>
__device__ __forceinline__ void wave_streams_sum(double (&acc)[D]) {
#pragma unroll
  for (int off = OPT; off < 64; off <<= 1)
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += __shfl_xor(acc[k], off, 64);
}

// (at least 4 waves per SIMD, which the register budget allows without
// spilling at this prefetch depth)
template <int D, int OPT>
__global__ __launch_bounds__(kBlock, 4) void k_solve_fwd_wave(const SolveTask* __restrict tasks, int ntasks,
                                                           const double* __restrict Pcol,
                                                           const int32_t* __restrict pull_ptr,
                                                           const int32_t* __restrict pull_idx,
                                                           const double* __restrict b, double* __restrict y,
                                                           double* __restrict ub) {
  constexpr int IS = 64 / OPT;
  __shared__ double vs[kBlock / 64][kWaveKC][D];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = blockIdx.x * (kBlock / 64) + wave;
  if (t >= ntasks) return;  // the whole wave leaves; no block barrier follows
  const SolveTask tk = tasks[t];
  const int o = lane % OPT, st = lane / OPT;
  const int i = tk.out0 + o;
  const bool live = i < tk.nf;
  double cv[D], acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) cv[k] = acc[k] = 0.0;
  bool cv_todo = st == 0 && live && i >= tk.c;
  const double* __restrict col = Pcol + tk.pf + i;
  for (int j0 = tk.lo; j0 < tk.hi; j0 += kWaveKC) {
    const int jn = min(kWaveKC, tk.hi - j0);
    // the chunk's first panel entries are in flight while the inner vector
    // is gathered
    double pf[kWavePFf];
#pragma unroll
    for (int u = 0; u < kWavePFf; ++u) {
      const int jj = st + u * IS;
      pf[u] = (live && jj < jn) ? __builtin_nontemporal_load(col + static_cast<int64_t>(j0 + jj) * tk.ld) : 0.0;
    }
    {  // stage the chunk; the carried part of the output row rides along
      const bool sg = lane < jn;
      double a[D];
#pragma unroll
      for (int k = 0; k < D; ++k) a[k] = sg ? b[static_cast<int64_t>(tk.first + j0 + lane) * D + k] : 0.0;
      fwd_carried2<D>(pull_ptr, pull_idx, ub, tk.poff + j0 + lane, sg, a, tk.poff + i, cv_todo, cv);
      cv_todo = false;
      if (sg) {
#pragma unroll
        for (int k = 0; k < D; ++k) vs[wave][lane][k] = a[k];
      }
    }
    wave_lds_sync();
    if (live) {
#pragma unroll
      for (int u = 0; u < kWavePFf; ++u) {
        const int jj = st + u * IS;
        if (jj < jn) {
#pragma unroll
          for (int k = 0; k < D; ++k) acc[k] += pf[u] * vs[wave][jj][k];
        }
      }
#pragma unroll 8
      for (int jj = st + kWavePFf * IS; jj < jn; jj += IS) {
        const double pv = __builtin_nontemporal_load(col + static_cast<int64_t>(j0 + jj) * tk.ld);
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] += pv * vs[wave][jj][k];
      }
    }
    wave_lds_sync();
  }
  if (cv_todo) fwd_carried<D>(tk, i, pull_ptr, pull_idx, ub, cv);
  wave_streams_sum<D, OPT>(acc);
  if (st != 0 || !live) return;
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] += cv[k];
  fwd_store<D>(tk, i, acc, y, ub);
}

// (at least 5 waves per SIMD: the level is bound by load latency, and the
// kernel fits the register budget of 5 without spilling)
template <int D, int OPT>
__global__ __launch_bounds__(kBlock, 5) void k_solve_bwd_wave(const SolveTask* __restrict tasks, int ntasks,
                                                           const double* __restrict Prow,
                                                           const int32_t* __restrict sidx, double* y, double* x,
                                                           const SolveTask* __restrict yred, int nyred,
                                                           const double* __restrict fpart,
                                                           const SolveTask* __restrict xred, int nxred,
                                                           const double* xpart) {
  constexpr int IS = 64 / OPT;
  __shared__ double vs[kBlock / 64][kWaveKC][D];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = blockIdx.x * (kBlock / 64) + wave;
  if (t >= ntasks) {  // the whole wave: a pending reduction, if any
    bwd_appended<D>(t - ntasks, lane, yred, nyred, fpart, y, xred, nxred, xpart, x);
    return;
  }
  const SolveTask tk = tasks[t];
  const int o = lane % OPT, st = lane / OPT;
  const int j = tk.out0 + o;
  const bool live = j < tk.c;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  const double* __restrict rowp = Prow + tk.pf + j;
  for (int p0 = tk.lo; p0 < tk.hi; p0 += kWaveKC) {
    const int pn = min(kWaveKC, tk.hi - p0);
    double pf[kWavePF];
#pragma unroll
    for (int u = 0; u < kWavePF; ++u) {
      const int pp = st + u * IS;
      pf[u] = (live && pp < pn) ? __builtin_nontemporal_load(rowp + static_cast<int64_t>(p0 + pp) * tk.ld) : 0.0;
    }
    if (lane < pn) {
      double v[D];
      bwd_entry<D>(tk, p0 + lane, sidx, y, x, xpart, v);
#pragma unroll
      for (int k = 0; k < D; ++k) vs[wave][lane][k] = v[k];
    }
    wave_lds_sync();
    if (live) {
#pragma unroll
      for (int u = 0; u < kWavePF; ++u) {
        const int pp = st + u * IS;
        if (pp < pn) {
#pragma unroll
          for (int k = 0; k < D; ++k) acc[k] += pf[u] * vs[wave][pp][k];
        }
      }
#pragma unroll 8
      for (int pp = st + kWavePF * IS; pp < pn; pp += IS) {
        const double pv = __builtin_nontemporal_load(rowp + static_cast<int64_t>(p0 + pp) * tk.ld);
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] += pv * vs[wave][pp][k];
      }
    }
    wave_lds_sync();
  }
  wave_streams_sum<D, OPT>(acc);
  if (st != 0 || !live) return;
#pragma unroll
  for (int k = 0; k < D; ++k) x[static_cast<int64_t>(tk.first + j) * D + k] = acc[k];
}

// ---------------------------------------------------------------------------
// K3: the fused local step: J = G W^k; U-step; P-step; Lambda-step; emit the
// next W-step's corner vectors; per-block partial sums (Algorithm 1 and eq.
// primaldualerror).  Partials: 0 e_prim^2, 1 e_dual^2, 2 E_P, 3 E_map (over
// det J > 0), 4 Phi, 5 flips, 6 non-finite Lambda, 7 |GW|^2, 8 |P|^2.
// PROX: the proximal term of the U-step (h_mode 1); DIAG: a diagnostic
// iteration (corner vectors of Lambda into glam, the two bound proxies) --
// compile-time, so the common kernel keeps no registers for them.
// ---------------------------------------------------------------------------
template <int D, typename R, int ENERGY, int BS, bool PROX, bool DIAG>
__global__ __launch_bounds__(BS) void k_local(int64_t m, int64_t e0, int64_t e1, const int32_t* __restrict T,
                                                  const R* __restrict Bm_,
                                                  const R* __restrict w, R rho_u, const R* __restrict rho_e,
                                                  int store_u,
                                                  const double* __restrict x, const double* __restrict xprev,
                                                  R* __restrict U, R* __restrict P, R* __restrict Lam,
                                                  R* __restrict gnorm2, R* __restrict g,
                                                  double* __restrict partials, R* __restrict glam) {
  // each XCD takes a contiguous eighth of the element blocks, so the vertex
  // positions its elements gather are fetched into one L2
  const int64_t blk = xcd_block();
  const int64_t e = e0 + blk * BS + threadIdx.x;
  double part[kNumPartials];
  partials_init(part);
  if (e < e1) {
    const R we = w[e];
    const R rho = rho_e ? rho_e[e] : rho_u;  // mu_e / w_e (per element after a rescaling)
    const R mu = rho * we;
    const double wd = static_cast<double>(we), mud = static_cast<double>(mu);
    R J[D][D], Bm[D][D];  // B is kept for the corner vectors at the end
    {
      // edge differences in float64, then J = B E and the dual residual term
      double x0[D], d0[D];
      const int32_t v0 = T[e];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        x0[k] = x[static_cast<int64_t>(v0) * D + k];
        d0[k] = x0[k] - xprev[static_cast<int64_t>(v0) * D + k];
      }
      R E[D][D], dE[D][D];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const int64_t vj = T[(j + 1) * m + e];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const double xv = x[vj * D + k];
          E[j][k] = static_cast<R>(xv - x0[k]);
          dE[j][k] = static_cast<R>((xv - xprev[vj * D + k]) - d0[k]);
        }
      }
      R Jd[D][D];
      load_B<D, R>(Bm_, m, e, Bm);
      matmul<D, R>(Bm, E, J);
      matmul<D, R>(Bm, dE, Jd);
      double jd2 = 0.0, gw = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int k = 0; k < D; ++k) {
          jd2 += static_cast<double>(Jd[a][k]) * Jd[a][k];
          gw += static_cast<double>(J[a][k]) * J[a][k];
        }
      part[1] = mud * mud * jd2;
      part[7] = gw;
      const R dJ = det<D, R>(J);
      if (dJ > R(0)) {
        const double dd = static_cast<double>(dJ);
        double fJ;
        if constexpr (ENERGY == 1) fJ = 0.5 * gw - log(dd);
        else fJ = 0.5 * (gw + static_cast<double>(adj_norm2<D, R>(J)) / (dd * dd));
        part[3] = wd * fJ;
      } else {
        part[5] = 1.0;
      }
    }
    R Ur[D][D], Pm[D][D], L[D][D], A[D][D];
    // the previous rotation is an input only through the proximal term (h > 0)
    // and the 2D tie rule; otherwise the rotation is recomputed from Q alone
    if (D == 2 || PROX) {
      load_U<D, R>(U, m, e, Ur);
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) Ur[i][j] = i == j ? R(1) : R(0);
    }
    load_P<D, R>(P, m, e, Pm);
#pragma unroll
    for (int i = 0; i < D * D; ++i) L[i / D][i % D] = Lam[i * m + e];
    // diagnostic iterations keep U^k and Lambda^k for the Lambda-ratio proxy
    R Uo[D][D], Lo[D][D];
    if (DIAG) {
      if (D == 2 || PROX) {
#pragma unroll
        for (int i = 0; i < D * D; ++i) Uo[i / D][i % D] = Ur[i / D][i % D];
      } else {
        load_U<D, R>(U, m, e, Uo);
      }
#pragma unroll
      for (int i = 0; i < D * D; ++i) Lo[i / D][i % D] = L[i / D][i % D];
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int k = 0; k < D; ++k) A[a][k] = J[a][k] + L[a][k];
    {
      // U-step: Q = (J + Lambda) P + (h/mu) U_prev; h/mu = 20 (1 + |grad f(P_prev)|^2) / rho^2
      R Q[D][D];
      matmul<D, R>(A, Pm, Q);
      if (PROX) {
        const R hm = R(20) * (R(1) + gnorm2[e]) / (rho * rho);
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int k = 0; k < D; ++k) Q[a][k] += hm * Ur[a][k];
      }
      rotation<D, R>(Q, Ur);
    }
    // P-step: S = symm(U^T A), per-eigenvalue roots, floor
    R p[D];
    {
      R S[D][D];
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = i; j < D; ++j) {
          R s1 = R(0), s2 = R(0);
#pragma unroll
          for (int k = 0; k < D; ++k) {
            s1 += Ur[k][i] * A[k][j];
            s2 += Ur[k][j] * A[k][i];
          }
          S[i][j] = S[j][i] = R(0.5) * (s1 + s2);
        }
      R q[D], V[D][D];
      sym_eig<D, R>(S, q, V);
      R detp = R(1), trp = R(0);
#pragma unroll
      for (int j = 0; j < D; ++j) {
        p[j] = dm::root<ENERGY, R>(q[j], rho);
        detp *= p[j];
        trp += p[j];
      }
      const R fl = static_cast<R>(dm::kSqrtEps);
      if (detp < fl || trp < fl) {
#pragma unroll
        for (int j = 0; j < D; ++j) p[j] = p[j] > fl ? p[j] : fl;
      }
      spectral<D, R>(V, p, Pm);
    }
    // Lambda-step and the next right-hand side r = mu (U P - Lambda)
    R UP[D][D], r[D][D];
    matmul<D, R>(Ur, Pm, UP);
    double ep = 0.0, lam2 = 0.0, res2 = 0.0;
    bool finite = true;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const R dv = J[a][k] - UP[a][k];
        const R ln = L[a][k] + dv;
        L[a][k] = ln;
        r[a][k] = mu * (UP[a][k] - ln);
        ep += static_cast<double>(dv) * dv;
        lam2 += static_cast<double>(ln) * ln;
        res2 += static_cast<double>(dv + ln) * (dv + ln);
        finite = finite && (ln - ln == R(0));
      }
    if (D == 2 || PROX || store_u) store_U<D, R>(U, m, e, Ur);
    store_P<D, R>(P, m, e, Pm);
#pragma unroll
    for (int i = 0; i < D * D; ++i) Lam[i * m + e] = L[i / D][i % D];
    store_g<D, R>(g, e, Bm, r);
    if (DIAG) store_g<D, R>(glam, e, Bm, L);  // corner vectors of Lambda (|G^T Lambda|)
    double fP = 0.0, p2 = 0.0;
    R gn = R(0);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      fP += dm::f_eig<ENERGY, R>(p[j]);
      p2 += static_cast<double>(p[j]) * p[j];
      const R gj = ENERGY == 1 ? p[j] - R(1) / p[j] : p[j] - R(1) / (p[j] * p[j] * p[j]);
      gn += gj * gj;
    }
    if (PROX || store_u) gnorm2[e] = gn;
    if (DIAG) {  // the bound proxies (diagnostic iterations)
      part[9] = static_cast<double>(gn);  // max |grad f(P)|^2 (proxy for B_i of Condition "gradf")
      part[10] = lambda_ratio<D, R>(Uo, Lo, Ur, L, ep);
    }
    part[0] = ep;
    part[2] = wd * fP;
    part[4] = wd * fP + 0.5 * mud * (res2 - lam2);
    part[6] = finite ? 0.0 : 1.0;
    part[8] = p2;
  }
  // the maxima only on diagnostic iterations (their slots are not read
  // otherwise); partials in element-block order (the reduction's order)
  double* out = partials + blk * kNumPartials;
  if (DIAG) block_reduce_store<kNumPartials, BS, kNumSums>(part, out);
  else block_reduce_store<kNumSums, BS, kNumSums>(*reinterpret_cast<double(*)[kNumSums]>(part), out);
}

// first stage of the partial-sum reduction when the local step ran many small
// blocks: block j adds rows [j kFinalizeRows, (j + 1) kFinalizeRows) in a fixed
// order (strided per thread, then the shuffle tree)
constexpr int kFinalizeRows = 256;

__global__ __launch_bounds__(kBlock) void k_partials_reduce(const double* __restrict partials, int64_t nb,
                                                            double* __restrict out, int nf) {
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kFinalizeRows;
  const int64_t r1 = r0 + kFinalizeRows < nb ? r0 + kFinalizeRows : nb;
  double v[kNumPartials];
  partials_init(v);
  for (int64_t bi = r0 + threadIdx.x; bi < r1; bi += kBlock) partials_add(v, partials + bi * kNumPartials, nf);
  block_reduce_store<kNumPartials, kBlock, kNumSums>(v, out + static_cast<int64_t>(blockIdx.x) * kNumPartials);
}

// fixed-order reduction of the block partials into one history record: at
// hist, or (k_dev != nullptr) at record *k_dev of hist, after which *k_dev is
// advanced (an iteration counter kept on the device for replayed graphs)
__global__ __launch_bounds__(kBlock) void k_finalize(const double* __restrict partials, int64_t nb,
                                                     double* __restrict hist, int64_t* __restrict k_dev,
                                                     int fields, int nf) {
  double v[kNumPartials];
  partials_init(v);
  for (int64_t bi = threadIdx.x; bi < nb; bi += kBlock) partials_add(v, partials + bi * kNumPartials, nf);
  __shared__ double out[kNumPartials];
  block_reduce_store<kNumPartials, kBlock, kNumSums>(v, out);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (k_dev) hist += *k_dev * fields;
    const double flips = out[5];
    hist[0] = sqrt(out[0]);
    hist[1] = sqrt(out[1]);
    hist[2] = out[2];
    hist[3] = flips > 0.0 ? __longlong_as_double(0x7ff0000000000000LL) : out[3];
    hist[4] = out[4];
    hist[5] = flips;
    hist[6] = out[6];
    hist[7] = sqrt(out[7]);
    hist[8] = sqrt(out[8]);
    hist[9] = __longlong_as_double(0x7ff8000000000000LL);
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    hist[10] = nf > kNumSums ? sqrt(out[9]) : nan;  // the bound proxies: diagnostic iterations only
    hist[11] = nf > kNumSums ? out[10] : nan;
    if (k_dev) *k_dev += 1;
  }
}

// One rescaling event (Section "Implementation", "Rescaling mu_i and
// Lambda"), per element, from the state after an iteration: e_prim_e =
// |J_e - U_e P_e| and e_dual_e = mu_e |J_e - J_e^prev| (both maps are still
// in their buffers); mu_e is multiplied by rho_r / 2 if e_prim_e > rho_r
// e_dual_e and divided by it if e_dual_e > rho_r e_prim_e, never below half
// the bound of Prop. "Sufficient decrease" (gamma = 1, epsilon = 0) with the
// F_e of the Lipschitz lemma for B_e = sqrt(5 (1 + |grad f(P_e)|^2)) and F_e^2
// capped at eps_m^(-1/4); the scaled dual Lambda_e is divided by the factor
// and the next right-hand side's corner vectors are emitted again.  Decisions
// in float64.  mu_out: the new mu_e in float64 (for the new factor); glam (may
// be null): the corner vectors of the rescaled Lambda.
template <int D, typename R, int ENERGY>
__global__ __launch_bounds__(kBlock) void k_rescale(int64_t m, int64_t e0, int64_t e1, const int32_t* __restrict T,
                                                    const R* __restrict Bm_, const R* __restrict w,
                                                    R* __restrict rho_e, const double* __restrict x,
                                                    const double* __restrict xprev, const R* __restrict U,
                                                    const R* __restrict P, R* __restrict Lam,
                                                    const R* __restrict gnorm2, R* __restrict g, double rho_r,
                                                    double* __restrict mu_out, R* __restrict glam) {
  const int64_t e = e0 + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= e1) return;
  const double wd = static_cast<double>(w[e]);
  const double mu = static_cast<double>(rho_e[e]) * wd;
  R Bm[D][D];
  load_B<D, R>(Bm_, m, e, Bm);
  double E[D][D], dE[D][D], x0[D], p0[D];
  const int32_t v0 = T[e];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    x0[k] = x[static_cast<int64_t>(v0) * D + k];
    p0[k] = xprev[static_cast<int64_t>(v0) * D + k];
  }
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int64_t vj = T[(j + 1) * m + e];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      E[j][k] = x[vj * D + k] - x0[k];
      dE[j][k] = (x[vj * D + k] - xprev[vj * D + k]) - (x0[k] - p0[k]);
    }
  }
  R Ur[D][D], Pm[D][D];
  load_U<D, R>(U, m, e, Ur);
  load_P<D, R>(P, m, e, Pm);
  double ep2 = 0.0, ed2 = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double J = 0.0, Jd = 0.0, up = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        J += static_cast<double>(Bm[a][j]) * E[j][k];
        Jd += static_cast<double>(Bm[a][j]) * dE[j][k];
        up += static_cast<double>(Ur[a][j]) * static_cast<double>(Pm[j][k]);
      }
      ep2 += (J - up) * (J - up);
      ed2 += Jd * Jd;
    }
  const double e_prim = sqrt(ep2), e_dual = mu * sqrt(ed2);
  const double B = sqrt(5.0 * (1.0 + static_cast<double>(gnorm2[e])));
  double F;
  if (ENERGY == 1) {
    const double cl = 2.0 / (B + sqrt(4.0 + B * B));  // positive root of x^2 + B x - 1
    F = 1.0 + sqrt(static_cast<double>(D)) / (cl * cl);
  } else {
    double lo = 0.0, hi = 1.0;  // positive root of x^4 + B x^3 - 1 in [0, 1]
    for (int it = 0; it < 100; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid * mid * mid * mid + B * mid * mid * mid - 1.0 < 0.0) lo = mid;
      else hi = mid;
    }
    const double c = 0.5 * (lo + hi);
    F = 1.0 + 3.0 * sqrt(static_cast<double>(D)) / (c * c * c * c);
  }
  F = fmin(F, 90.50966799187809);  // F^2 <= eps_m^(-1/4) = 8192
  const double floor_mu = 0.25 * (-wd + sqrt(wd * wd + 16.0 * wd * wd * F * F));
  double nmu = e_prim > rho_r * e_dual ? mu * (0.5 * rho_r) : e_dual > rho_r * e_prim ? mu / (0.5 * rho_r) : mu;
  nmu = fmax(nmu, floor_mu);
  const double sc = nmu / mu;
  mu_out[e] = nmu;
  rho_e[e] = static_cast<R>(nmu / wd);
  R L[D][D], r[D][D];
  const R nmur = static_cast<R>(nmu);
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      L[a][k] = static_cast<R>(static_cast<double>(Lam[(a * D + k) * m + e]) / sc);
      Lam[(a * D + k) * m + e] = L[a][k];
      R up = R(0);
#pragma unroll
      for (int j = 0; j < D; ++j) up += Ur[a][j] * Pm[j][k];
      r[a][k] = nmur * (up - L[a][k]);
    }
  store_g<D, R>(g, e, Bm, r);
  if (glam) store_g<D, R>(glam, e, Bm, L);  // corner vectors of the rescaled Lambda (termination test)
}

// |G^T Lambda|^2 over all vertex rows (the dual threshold of eq.
// primaldualthresholds): row j adds the corner vectors of Lambda of its
// incident elements (four lanes per row, fixed shuffle tree); per-block sums.
template <int D, typename R>
__global__ __launch_bounds__(kBlock) void k_gtlam(int64_t n, const int32_t* __restrict av_ptr,
                                                  const int32_t* __restrict av_idx, const R* __restrict glam,
                                                  double* __restrict partials) {
  constexpr int LPR = 4;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t j = t / LPR;
  const int sub = static_cast<int>(t % LPR);
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  if (j < n)
    for (int32_t q = av_ptr[j] + sub; q < av_ptr[j + 1]; q += LPR) {
      const int64_t o = static_cast<int64_t>(av_idx[q]) * D;
#pragma unroll
      for (int k = 0; k < D; ++k) acc[k] += static_cast<double>(glam[o + k]);
    }
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int off = 1; off < LPR; off <<= 1) acc[k] += __shfl_xor(acc[k], off, 64);
  double v[1] = {0.0};
  if (sub == 0 && j < n)
#pragma unroll
    for (int k = 0; k < D; ++k) v[0] += acc[k] * acc[k];
  block_reduce_store<1>(v, partials + blockIdx.x);
}

// *out = sqrt of the fixed-order sum of the partials (history field 9)
__global__ __launch_bounds__(kBlock) void k_gtlam_finalize(const double* __restrict partials, int64_t nb,
                                                           double* __restrict out) {
  double v[1] = {0.0};
  for (int64_t bi = threadIdx.x; bi < nb; bi += kBlock) v[0] += partials[bi];
  __shared__ double red[1];
  block_reduce_store<1>(v, red);
  __syncthreads();
  if (threadIdx.x == 0) *out = sqrt(red[0]);
}

// ---------------------------------------------------------------------------
// Termination test of Algorithm 2 per problem (each mesh of a batch on its
// own; a plain handle is one problem), from the state as it stands after the
// iteration and any rescaling event of it: per problem, in float64, the sums
//   0 e_prim^2 = sum |J_e - U_e P_e|^2, 1 e_dual^2 = sum mu_e^2 |J_e - J_e^prev|^2
//   (eq. primaldualerror), 2 |G W|^2, 3 |P|^2, 4 flips (det J_e <= 0),
//   5 |G^T Lambda|^2 over the problem's vertex rows (eq. primaldualthresholds).
// A piece is a range of one problem's element list (kind 0) or vertex list
// (kind 1); a null list is the identity.  Fixed-order sums.
// ---------------------------------------------------------------------------
constexpr int kDiagFields = 6;
struct DiagPiece {
  int32_t kind, q0, q1, pad;
};

template <int D, typename R>
__global__ __launch_bounds__(kBlock) void k_diag_pieces(const DiagPiece* __restrict pieces,
                                                        const int32_t* __restrict elist,
                                                        const int32_t* __restrict vlist, int64_t m,
                                                        const int32_t* __restrict T, const double* __restrict B64,
                                                        const R* __restrict w, R rho_u, const R* __restrict rho_e,
                                                        const double* __restrict x, const double* __restrict xprev,
                                                        const R* __restrict U, const R* __restrict P,
                                                        const R* __restrict glam, const int32_t* __restrict av_ptr,
                                                        const int32_t* __restrict av_idx,
                                                        double* __restrict part) {
  const DiagPiece pc = pieces[blockIdx.x];
  double v[kDiagFields] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (pc.kind == 0) {
    for (int32_t q = pc.q0 + static_cast<int32_t>(threadIdx.x); q < pc.q1; q += kBlock) {
      const int64_t e = elist ? elist[q] : q;
      double E[D][D], dE[D][D];
      const int64_t v0 = T[e];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const int64_t vj = T[(j + 1) * m + e];
#pragma unroll
        for (int k = 0; k < D; ++k) {
          E[j][k] = x[vj * D + k] - x[v0 * D + k];
          dE[j][k] = (x[vj * D + k] - xprev[vj * D + k]) - (x[v0 * D + k] - xprev[v0 * D + k]);
        }
      }
      R Ur[D][D], Pm[D][D];
      load_U<D, R>(U, m, e, Ur);
      load_P<D, R>(P, m, e, Pm);
      double J[D][D], ep = 0.0, ed = 0.0, gw = 0.0, p2 = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int k = 0; k < D; ++k) {
          double jv = 0.0, jd = 0.0, up = 0.0;
#pragma unroll
          for (int j = 0; j < D; ++j) {
            const double b = B64[(a * D + j) * m + e];
            jv += b * E[j][k];
            jd += b * dE[j][k];
            up += static_cast<double>(Ur[a][j]) * static_cast<double>(Pm[j][k]);
          }
          J[a][k] = jv;
          ep += (jv - up) * (jv - up);
          ed += jd * jd;
          gw += jv * jv;
          p2 += static_cast<double>(Pm[a][k]) * static_cast<double>(Pm[a][k]);
        }
      const double mu = static_cast<double>(rho_e ? rho_e[e] : rho_u) * static_cast<double>(w[e]);
      v[0] += ep;
      v[1] += mu * mu * ed;
      v[2] += gw;
      v[3] += p2;
      v[4] += det<D, double>(J) <= 0.0 ? 1.0 : 0.0;
    }
  } else {
    for (int32_t q = pc.q0 + static_cast<int32_t>(threadIdx.x); q < pc.q1; q += kBlock) {
      const int64_t j = vlist ? vlist[q] : q;
      double acc[D];
#pragma unroll
      for (int k = 0; k < D; ++k) acc[k] = 0.0;
      for (int32_t r = av_ptr[j]; r < av_ptr[j + 1]; ++r) {
        const int64_t o = static_cast<int64_t>(av_idx[r]) * D;
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] += static_cast<double>(glam[o + k]);
      }
#pragma unroll
      for (int k = 0; k < D; ++k) v[5] += acc[k] * acc[k];
    }
  }
  block_reduce_store<kDiagFields>(v, part + static_cast<int64_t>(blockIdx.x) * kDiagFields);
}

// per problem, its pieces' sums in piece order: out[c][f]
__global__ __launch_bounds__(kBlock) void k_diag_problems(const int32_t* __restrict piece_ptr, int32_t nprob,
                                                          const double* __restrict part, double* __restrict out) {
  for (int32_t c = static_cast<int32_t>(blockIdx.x * kBlock + threadIdx.x); c < nprob;
       c += static_cast<int32_t>(gridDim.x * kBlock)) {
    double acc[kDiagFields] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t p = piece_ptr[c]; p < piece_ptr[c + 1]; ++p)
#pragma unroll
      for (int f = 0; f < kDiagFields; ++f) acc[f] += part[static_cast<int64_t>(p) * kDiagFields + f];
#pragma unroll
    for (int f = 0; f < kDiagFields; ++f) out[static_cast<int64_t>(c) * kDiagFields + f] = acc[f];
  }
}

// Several device-to-device copies in one launch (checkpoint slots of the
// adjoint: element state and map); 16-byte moves where both ends allow, 4-byte
// otherwise (every length is a multiple of 4).
constexpr int kMaxCopyJobs = 12;
struct CopyJobs {
  const char* src[kMaxCopyJobs];
  char* dst[kMaxCopyJobs];
  int64_t bytes[kMaxCopyJobs];
  int32_t n;
};

__global__ __launch_bounds__(kBlock) void k_copy_jobs(CopyJobs J) {
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int q = 0; q < J.n; ++q) {
    const char* __restrict src = J.src[q];
    char* __restrict dst = J.dst[q];
    const int64_t nb = J.bytes[q];
    int64_t done = 0;
    if (((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0) {
      const int64_t n16 = nb / 16;
      const uint4* __restrict s16 = reinterpret_cast<const uint4*>(src);
      uint4* __restrict d16 = reinterpret_cast<uint4*>(dst);
      for (int64_t i = tid; i < n16; i += stride) d16[i] = s16[i];
      done = n16 * 16;
    }
    const int64_t n4 = (nb - done) / 4;
    const uint32_t* __restrict s4 = reinterpret_cast<const uint32_t*>(src + done);
    uint32_t* __restrict d4 = reinterpret_cast<uint32_t*>(dst + done);
    for (int64_t i = tid; i < n4; i += stride) d4[i] = s4[i];
  }
}

__global__ void k_set_counter(int64_t* __restrict p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------------------
// layout conversions at the boundary
// ---------------------------------------------------------------------------
template <int D>
__global__ void k_map_in(int64_t n, const int32_t* __restrict new2old, const double* __restrict ext,
                         double* __restrict xint) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= n) return;
  const int64_t o = new2old[j];
#pragma unroll
  for (int k = 0; k < D; ++k) xint[j * D + k] = ext[o * D + k];
}

// ---------------------------------------------------------------------------
// General linear constraints A W = c in the W-step (eq. solvinginw).  The
// factor is of L~ = L_FF + gamma A_F^T A_F; with c' = c - A_C x_C the
// constrained minimiser is x = y - Z lambda with y = L~^{-1} (b + gamma A_F^T c'),
// Z = L~^{-1} A_F^T (precomputed, column-major ncon x nF) and lambda =
// S^{-1} (A_F y - c'), S = A_F Z (block elimination of the KKT system; the
// explicit S^{-1} is precomputed on the host).
// ---------------------------------------------------------------------------
constexpr int kMaxConstraints = 1024;

// c' = c - A_C x_C, one thread per constraint row
template <int D>
__global__ __launch_bounds__(kBlock) void k_con_shift(int64_t ncon, int64_t nF, const int64_t* __restrict con_ptr,
                                                      const int32_t* __restrict con_col,
                                                      const double* __restrict con_val, const double* __restrict c,
                                                      const double* __restrict xC, double* __restrict cp) {
  const int64_t a = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (a >= ncon) return;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = c[a * D + k];
  for (int64_t q = con_ptr[a]; q < con_ptr[a + 1]; ++q) {
    const int64_t j = con_col[q];
    if (j < nF) continue;
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] -= con_val[q] * xC[(j - nF) * D + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) cp[a * D + k] = acc[k];
}

// b_j += gamma (A_F^T c')_j on the free rows the constraints touch
template <int D>
__global__ __launch_bounds__(kBlock) void k_con_addq(int64_t nrows, const int32_t* __restrict rows,
                                                     const int32_t* __restrict cont_ptr,
                                                     const int32_t* __restrict cont_con,
                                                     const double* __restrict cont_val, double gamma,
                                                     const double* __restrict cp, double* __restrict b) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= nrows) return;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int32_t q = cont_ptr[i]; q < cont_ptr[i + 1]; ++q) {
    const int64_t a = cont_con[q];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += cont_val[q] * cp[a * D + k];
  }
  const int64_t j = rows[i];
#pragma unroll
  for (int k = 0; k < D; ++k) b[j * D + k] += gamma * acc[k];
}

// t = A x - c over all columns (the pinned rows of x hold x_C), i.e. A_F y - c'
template <int D>
__global__ __launch_bounds__(kBlock) void k_con_resid(int64_t ncon, const int64_t* __restrict con_ptr,
                                                      const int32_t* __restrict con_col,
                                                      const double* __restrict con_val, const double* __restrict c,
                                                      const double* __restrict x, double* __restrict t) {
  const int64_t a = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (a >= ncon) return;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = -c[a * D + k];
  for (int64_t q = con_ptr[a]; q < con_ptr[a + 1]; ++q) {
    const int64_t j = con_col[q];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += con_val[q] * x[j * D + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) t[a * D + k] = acc[k];
}

// lambda = S^{-1} t (S^{-1} symmetric, read by columns so lanes load
// consecutive entries)
template <int D>
__global__ __launch_bounds__(kBlock) void k_con_lambda(int64_t ncon, const double* __restrict Sinv,
                                                       const double* __restrict t, double* __restrict lam) {
  const int64_t a = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (a >= ncon) return;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int64_t b2 = 0; b2 < ncon; ++b2) {
    const double sv = Sinv[b2 * ncon + a];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += sv * t[b2 * D + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) lam[a * D + k] = acc[k];
}

// x_F -= Z lambda, one thread per free row; lambda staged in LDS
template <int D>
__global__ __launch_bounds__(kBlock) void k_con_correct(int64_t nF, int64_t ncon, const double* __restrict Z,
                                                        const double* __restrict lam, double* __restrict x) {
  __shared__ double sl[kMaxConstraints * D];
  for (int64_t i = threadIdx.x; i < ncon * D; i += kBlock) sl[i] = lam[i];
  __syncthreads();
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= nF) return;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int64_t a = 0; a < ncon; ++a) {
    const double z = Z[a * nF + j];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += z * sl[a * D + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) x[j * D + k] -= acc[k];
}

// set-up: the solution columns of one group of D constraint rows into Z
template <int D>
__global__ __launch_bounds__(kBlock) void k_con_zcols(int64_t nF, int64_t ncon, int64_t a0,
                                                      const double* __restrict xs, double* __restrict Z) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= nF) return;
#pragma unroll
  for (int k = 0; k < D; ++k)
    if (a0 + k < ncon) Z[(a0 + k) * nF + j] = xs[j * D + k];
}

// set-up: S = A_F Z, one thread per entry
__global__ __launch_bounds__(kBlock) void k_con_gram(int64_t nF, int64_t ncon, const int64_t* __restrict con_ptr,
                                                     const int32_t* __restrict con_col,
                                                     const double* __restrict con_val, const double* __restrict Z,
                                                     double* __restrict S) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= ncon * ncon) return;
  const int64_t a = t / ncon, b2 = t % ncon;
  double acc = 0.0;
  for (int64_t q = con_ptr[a]; q < con_ptr[a + 1]; ++q) {
    const int64_t j = con_col[q];
    if (j < nF) acc += con_val[q] * Z[b2 * nF + j];
  }
  S[t] = acc;
}

// ---------------------------------------------------------------------------
// Device factorisation of the top fronts (refactorisation after a rescaling
// event): assembly of a front from L and its children's update matrices, a
// lower-triangle copy, and the write of the node's panels [Linv; -M] into
// both device copies.  The dense steps between them are library calls.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_front_scatter(int64_t n, const int64_t* __restrict idx,
                                                          const double* __restrict val, double* __restrict F) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) F[idx[i]] += val[i];  // distinct entries
}

// F[rel[i] + rel[j] nf] += U[i + j ldu] for i >= j (lower triangle of one child)
__global__ __launch_bounds__(kBlock) void k_front_extend(int64_t rc, const int32_t* __restrict rel,
                                                         const double* __restrict U, int64_t ldu,
                                                         double* __restrict F, int64_t nf) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= rc * rc) return;
  const int64_t i = t % rc, j = t / rc;
  if (i < j) return;
  F[rel[i] + static_cast<int64_t>(rel[j]) * nf] += U[i + j * ldu];
}

// B = lower triangle of the n x n block A (zeros above the diagonal)
__global__ __launch_bounds__(kBlock) void k_lower_copy(int64_t n, const double* __restrict A, int64_t lda,
                                                       double* __restrict B, int64_t ldb) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= n * n) return;
  const int64_t i = t % n, j = t / n;
  B[i + j * ldb] = i >= j ? A[i + j * lda] : 0.0;
}

// panel entry (p, j) of [Linv; -M] into the column-major (ld ldc) and the
// row-major (ld ldr) copies at offset pf
__global__ __launch_bounds__(kBlock) void k_front_panels(int64_t c, int64_t r, const double* __restrict Linv,
                                                         const double* __restrict M, int64_t pf,
                                                         double* __restrict Pcol, double* __restrict Prow) {
  const int64_t nf = c + r;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= nf * c) return;
  const int64_t p = t % nf, j = t / nf;
  const double v = p < c ? (p >= j ? Linv[p + j * c] : 0.0) : -M[(p - c) + j * r];
  Pcol[pf + panel_tile_index_dev(p, j, nf, c)] = v;  // forward copy: output row p, inner column j
  Prow[pf + panel_tile_index_dev(j, p, c, nf)] = v;  // backward copy: output column j, inner row p
}

// right-hand side of a solve whose only data are the fixed rows: b_F = -L_FC x_C
// (the minimiser of a quadratic energy with fixed vertices); rows >= nF copy
// the fixed positions into x
template <int D>
__global__ __launch_bounds__(kBlock) void k_fixed_rhs(int64_t nF, int64_t n, const int32_t* __restrict pin_ptr,
                                                      const int32_t* __restrict pin_col,
                                                      const double* __restrict pin_val, const double* __restrict xC,
                                                      double* __restrict b, double* __restrict x) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= n) return;
  if (j >= nF) {
#pragma unroll
    for (int k = 0; k < D; ++k) x[j * D + k] = xC[(j - nF) * D + k];
    return;
  }
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int32_t q = pin_ptr[j]; q < pin_ptr[j + 1]; ++q) {
    const double v = pin_val[q];
    const int64_t c = pin_col[q];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] -= v * xC[c * D + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) b[j * D + k] = acc[k];
}

template <int D>
__global__ void k_map_out(int64_t n, const int32_t* __restrict new2old, const double* __restrict xint,
                          double* __restrict ext) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= n) return;
  const int64_t o = new2old[j];
#pragma unroll
  for (int k = 0; k < D; ++k) ext[o * D + k] = xint[j * D + k];
}

template <int D, typename R>
__global__ void k_state_in(int64_t m, const int32_t* __restrict e_new2old, const R* __restrict Uext,
                           const R* __restrict Pext, const R* __restrict Lext, R* __restrict U, R* __restrict P,
                           R* __restrict Lam) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= m) return;
  const int64_t o = static_cast<int64_t>(e_new2old[e]) * D * D;
  R Um[D][D], Pm[D][D];
#pragma unroll
  for (int i = 0; i < D * D; ++i) {
    Um[i / D][i % D] = Uext[o + i];
    Pm[i / D][i % D] = Pext[o + i];
    Lam[i * m + e] = Lext[o + i];
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = i + 1; j < D; ++j) Pm[i][j] = Pm[j][i] = R(0.5) * (Pm[i][j] + Pm[j][i]);
  store_U<D, R>(U, m, e, Um);
  store_P<D, R>(P, m, e, Pm);
}

template <int D, typename R>
__global__ void k_state_out(int64_t m, const int32_t* __restrict e_new2old, const R* __restrict U,
                            const R* __restrict P, const R* __restrict Lam, R* __restrict Uext, R* __restrict Pext,
                            R* __restrict Lext, R* __restrict Wext) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= m) return;
  const int64_t o = static_cast<int64_t>(e_new2old[e]) * D * D;
  R Um[D][D], Pm[D][D], W[D][D];
  load_U<D, R>(U, m, e, Um);
  load_P<D, R>(P, m, e, Pm);
  if (Uext)
#pragma unroll
    for (int i = 0; i < D * D; ++i) Uext[o + i] = Um[i / D][i % D];
  if (Pext)
#pragma unroll
    for (int i = 0; i < D * D; ++i) Pext[o + i] = Pm[i / D][i % D];
  if (Lext)
#pragma unroll
    for (int i = 0; i < D * D; ++i) Lext[o + i] = Lam[i * m + e];
  if (Wext) {
    matmul<D, R>(Um, Pm, W);
#pragma unroll
    for (int i = 0; i < D * D; ++i) Wext[o + i] = W[i / D][i % D];
  }
}

// pinned positions from the internal map (rows nF..n-1)
template <int D>
__global__ void k_pins_from_map(int64_t nF, int64_t nC, const double* __restrict x, double* __restrict xC) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= nC) return;
#pragma unroll
  for (int k = 0; k < D; ++k) xC[i * D + k] = x[(nF + i) * D + k];
}

}  // namespace ffd
