// Reverse-mode (adjoint) kernels of K unrolled ADMM iterations.
//
// Differentiated function: rest vertices V (element frames B_i, weights w_i,
// mu_i = rho w_i, W^0 = V) and pinned targets x_C  ->  the element state after
// K iterations; the seed is P-bar^K (e.g. w_i grad f(P_i^K) for the loss
// sum_i w_i f(P_i^K)).  With W^0 = V the initial Jacobians are the identity
// for every V, so the initial state carries no derivative.
//
// One reversed iteration k (state k-1 -> k), per element unless noted:
//   k_adj_local  : recompute J = G x^k, A = J + Lam, Q = A P, U' = rot(Q),
//                  S = symm(U'^T A), P' = F(S); reverse the Lambda-step, the
//                  spectral P-step (Daleckii-Krein divided differences with
//                  p'(q) = rho / (rho + f_s''(p)) from the scalar root), the
//                  polar U-step (dU = U [w]_x, (tr H - H) w = vee(U^T dQ - dQ^T U)),
//                  Q = A P and A = J + Lam; emit the corner vectors of G^T J-bar
//                  and accumulate B-bar += J-bar E_x^T.
//   k_adj_gather : x-bar = G^T J-bar per vertex (free rows -> right-hand side
//                  of the adjoint solve, pinned rows -> x_C-bar).
//   solve        : lambda = L_FF^{-1} x-bar_F with the same factor (L symmetric).
//   k_adj_wstep  : r-bar = G lambda, Y-bar = mu r-bar; U-bar += Y-bar P^T,
//                  P-bar += U^T Y-bar, Lam-bar -= Y-bar (Y = U P - Lam); the
//                  implicit-function terms of the W-step for B-bar and w-bar.
//   k_adj_pins   : x_C-bar -= L_CF lambda.
// Finally k_adj_vbar turns B-bar, w-bar into vertex gradients through
// Dm-bar = -B B-bar^T B + w-bar w B (B = Dm^{-T}, w = |det Dm| / d!).
// Adjoint arithmetic is float64 for every precision of the forward steps.
#pragma once
#include "kernels.hpp"

namespace ffd {

template <int D>
__device__ __forceinline__ void dmatmul(const double A[D][D], const double B[D][D], double C[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) s += A[i][k] * B[k][j];
      C[i][j] = s;
    }
}

// C = A^T B
template <int D>
__device__ __forceinline__ void dmatmul_tn(const double A[D][D], const double B[D][D], double C[D][D]) {
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) s += A[k][i] * B[k][j];
      C[i][j] = s;
    }
}

template <int D>
__device__ __forceinline__ void load_d(const double* __restrict a, int64_t m, int64_t e, double X[D][D]) {
#pragma unroll
  for (int i = 0; i < D * D; ++i) X[i / D][i % D] = a[i * m + e];
}

template <int D>
__device__ __forceinline__ void store_d(double* __restrict a, int64_t m, int64_t e, const double X[D][D]) {
#pragma unroll
  for (int i = 0; i < D * D; ++i) a[i * m + e] = X[i / D][i % D];
}

// E[j][k] = x[T_{j+1}][k] - x[T_0][k] in float64 (pinned rows of lam-type
// vectors are stored as zeros by the caller)
template <int D>
__device__ __forceinline__ void edges(const int32_t* __restrict T, int64_t m, int64_t e, const double* __restrict x,
                                      double E[D][D]) {
  const int64_t v0 = T[e];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int64_t vj = T[(j + 1) * m + e];
#pragma unroll
    for (int k = 0; k < D; ++k) E[j][k] = x[vj * D + k] - x[v0 * D + k];
  }
}

// corner vectors g[c][k] = sum_a C[a][c] X[a][k], C[:,0] = -sum_j B[:,j], float64
template <int D>
__device__ __forceinline__ void store_g64(double* __restrict g, int64_t e, const double Bm[D][D], const double X[D][D]) {
  double* dst = g + e * (D + 1) * D;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double s0 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) s += Bm[a][j] * X[a][k];
      dst[(j + 1) * D + k] = s;
      s0 += s;
    }
    dst[k] = -s0;
  }
}

// solve the symmetric 3x3 system K b = a by cofactors; zero if K is singular
__device__ __forceinline__ void solve3(const double K[3][3], const double a[3], double b[3]) {
  const double c00 = K[1][1] * K[2][2] - K[1][2] * K[2][1];
  const double c01 = K[1][2] * K[2][0] - K[1][0] * K[2][2];
  const double c02 = K[1][0] * K[2][1] - K[1][1] * K[2][0];
  const double det = K[0][0] * c00 + K[0][1] * c01 + K[0][2] * c02;
  const double sc = fabs(K[0][0]) + fabs(K[1][1]) + fabs(K[2][2]);
  if (!(fabs(det) > 1e-12 * sc * sc * sc)) {
    b[0] = b[1] = b[2] = 0.0;
    return;
  }
  const double inv[3][3] = {
      {c00, K[0][2] * K[2][1] - K[0][1] * K[2][2], K[0][1] * K[1][2] - K[0][2] * K[1][1]},
      {c01, K[0][0] * K[2][2] - K[0][2] * K[2][0], K[0][2] * K[1][0] - K[0][0] * K[1][2]},
      {c02, K[0][1] * K[2][0] - K[0][0] * K[2][1], K[0][0] * K[1][1] - K[0][1] * K[1][0]}};
#pragma unroll
  for (int i = 0; i < 3; ++i) b[i] = (inv[i][0] * a[0] + inv[i][1] * a[1] + inv[i][2] * a[2]) / det;
}

// adjoint of U = rot(Q): Q-bar from U-bar
template <int D>
__device__ __forceinline__ void rot_adjoint(const double U[D][D], const double Q[D][D], const double Ub[D][D],
                                            double Qb[D][D]) {
  double UtUb[D][D];
  dmatmul_tn<D>(U, Ub, UtUb);
  if constexpr (D == 2) {
    const double zr = Q[0][0] + Q[1][1], zi = Q[1][0] - Q[0][1];
    const double n2 = zr * zr + zi * zi;
    const double gphi = UtUb[1][0] - UtUb[0][1];
    const double s = n2 > 0.0 ? gphi / n2 : 0.0;
    Qb[0][0] = -zi * s;
    Qb[0][1] = -zr * s;
    Qb[1][0] = zr * s;
    Qb[1][1] = -zi * s;
  } else {
    double H[3][3];
    dmatmul_tn<3>(U, Q, H);
    const double tr = H[0][0] + H[1][1] + H[2][2];
    double K[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) K[i][j] = (i == j ? tr : 0.0) - 0.5 * (H[i][j] + H[j][i]);
    const double a[3] = {UtUb[2][1] - UtUb[1][2], UtUb[0][2] - UtUb[2][0], UtUb[1][0] - UtUb[0][1]};
    double bv[3];
    solve3(K, a, bv);
    const double Bx[3][3] = {{0.0, -bv[2], bv[1]}, {bv[2], 0.0, -bv[0]}, {-bv[1], bv[0], 0.0}};
    dmatmul<3>(U, Bx, Qb);
  }
}

template <int ENERGY>
__device__ __forceinline__ double fpp(double p) {
  if constexpr (ENERGY == 1) return 1.0 + 1.0 / (p * p);
  else return 1.0 + 3.0 / (p * p * p * p);
}

// recompute the forward local step of iteration k for element e (arithmetic R,
// exactly as k_local) and return its intermediates in float64
template <int D, typename R, int ENERGY>
struct LocalFwd {
  double J[D][D], A[D][D], Q[D][D], U1[D][D], P0[D][D], U0[D][D], L0[D][D], V[D][D], q[D], p[D], P1[D][D];
  bool clamped[D];
};

template <int D, typename R, int ENERGY>
__device__ __forceinline__ void local_forward(int64_t m, int64_t e, const int32_t* __restrict T,
                                              const R* __restrict Bm_, R rho, const double* __restrict x,
                                              const R* __restrict U, const R* __restrict P, const R* __restrict Lam,
                                              LocalFwd<D, R, ENERGY>& F) {
  double x0[D];
  const int32_t v0 = T[e];
#pragma unroll
  for (int k = 0; k < D; ++k) x0[k] = x[static_cast<int64_t>(v0) * D + k];
  R E[D][D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int64_t vj = T[(j + 1) * m + e];
#pragma unroll
    for (int k = 0; k < D; ++k) E[j][k] = static_cast<R>(x[vj * D + k] - x0[k]);
  }
  R Bm[D][D], J[D][D], Ur[D][D], Pm[D][D], L[D][D], A[D][D], Q[D][D];
  load_B<D, R>(Bm_, m, e, Bm);
  matmul<D, R>(Bm, E, J);
  load_U<D, R>(U, m, e, Ur);
  load_P<D, R>(P, m, e, Pm);
#pragma unroll
  for (int i = 0; i < D * D; ++i) L[i / D][i % D] = Lam[i * m + e];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int k = 0; k < D; ++k) A[a][k] = J[a][k] + L[a][k];
  matmul<D, R>(A, Pm, Q);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      F.U0[i][j] = Ur[i][j];
      F.P0[i][j] = Pm[i][j];
      F.L0[i][j] = L[i][j];
    }
  rotation<D, R>(Q, Ur);
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
  R qv[D], Vv[D][D], pv[D];
  sym_eig<D, R>(S, qv, Vv);
  R detp = R(1), trp = R(0);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    pv[j] = dm::root<ENERGY, R>(qv[j], rho);
    detp *= pv[j];
    trp += pv[j];
  }
  const R fl = static_cast<R>(dm::kSqrtEps);
  const bool small = detp < fl || trp < fl;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    F.clamped[j] = small && pv[j] < fl;
    if (small) pv[j] = pv[j] > fl ? pv[j] : fl;
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    F.q[i] = qv[i];
    F.p[i] = pv[i];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      F.J[i][j] = J[i][j];
      F.A[i][j] = A[i][j];
      F.Q[i][j] = Q[i][j];
      F.U1[i][j] = Ur[i][j];
      F.V[i][j] = Vv[i][j];
    }
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) s += F.V[i][k] * F.p[k] * F.V[j][k];
      F.P1[i][j] = s;
    }
}

// seed: P-bar = w grad f(P^K) (+ the caller's P-bar), U-bar = Lam-bar = 0,
// w-bar = f(P^K) (loss term), B-bar = 0
template <int D, typename R, int ENERGY>
__global__ __launch_bounds__(kBlock) void k_adj_seed(int64_t m, int64_t e0, int64_t e1, const R* __restrict P,
                                                     const R* __restrict w,
                                                     int energy_loss, const R* __restrict Pbar_ext,
                                                     const int32_t* __restrict e_new2old, double* __restrict Ub,
                                                     double* __restrict Pb, double* __restrict Lb,
                                                     double* __restrict Bb, double* __restrict wb) {
  const int64_t e = e0 + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= e1) return;
  R Pm[D][D], q[D], V[D][D];
  load_P<D, R>(P, m, e, Pm);
  sym_eig<D, R>(Pm, q, V);
  double G[D][D];
  double fP = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) G[i][j] = 0.0;
  if (energy_loss) {
    const double we = static_cast<double>(w[e]);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double p = static_cast<double>(q[k]);
      const double gk = ENERGY == 1 ? p - 1.0 / p : p - 1.0 / (p * p * p);
      fP += dm::f_eig<ENERGY, double>(p);
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) G[i][j] += we * static_cast<double>(V[i][k]) * gk * static_cast<double>(V[j][k]);
    }
  }
  if (Pbar_ext) {
    const int64_t o = static_cast<int64_t>(e_new2old[e]) * D * D;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) G[i][j] += static_cast<double>(Pbar_ext[o + i * D + j]);
  }
  double Z[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Z[i][j] = 0.0;
  store_d<D>(Pb, m, e, G);
  store_d<D>(Ub, m, e, Z);
  store_d<D>(Lb, m, e, Z);
  store_d<D>(Bb, m, e, Z);
  wb[e] = energy_loss ? fP : 0.0;
}

template <int D, typename R, int ENERGY>
__global__ __launch_bounds__(kBlock) void k_adj_local(int64_t m, int64_t e0, int64_t e1, const int32_t* __restrict T,
                                                      const R* __restrict Bm_,
                                                      const double* __restrict B64, R rho,
                                                      const double* __restrict x, const R* __restrict U,
                                                      const R* __restrict P, const R* __restrict Lam,
                                                      double* __restrict Ub, double* __restrict Pb,
                                                      double* __restrict Lb, double* __restrict Bb,
                                                      double* __restrict gJ) {
  const int64_t e = e0 + static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= e1) return;
  LocalFwd<D, R, ENERGY> F;
  local_forward<D, R, ENERGY>(m, e, T, Bm_, rho, x, U, P, Lam, F);
  double Ub1[D][D], Pb1[D][D], Lb1[D][D];
  load_d<D>(Ub, m, e, Ub1);
  load_d<D>(Pb, m, e, Pb1);
  load_d<D>(Lb, m, e, Lb1);
  // Lambda' = Lambda + J - U' P'
  double Jb[D][D], Lb0[D][D], T1[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      Jb[i][j] = Lb1[i][j];
      Lb0[i][j] = Lb1[i][j];
    }
  dmatmul<D>(Lb1, F.P1, T1);  // U'-bar -= Lam'-bar P'^T (P' symmetric)
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Ub1[i][j] -= T1[i][j];
  dmatmul_tn<D>(F.U1, Lb1, T1);  // P'-bar -= U'^T Lam'-bar
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Pb1[i][j] -= T1[i][j];
  // P' = F(S): S-bar = V (Gamma o (V^T sym(P'-bar) V)) V^T
  double Ps[D][D], W1[D][D], W2[D][D], Sb[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Ps[i][j] = 0.5 * (Pb1[i][j] + Pb1[j][i]);
  dmatmul_tn<D>(F.V, Ps, W1);
  dmatmul<D>(W1, F.V, W2);
  double dp[D];
  const double rd = static_cast<double>(rho);
#pragma unroll
  for (int a = 0; a < D; ++a) dp[a] = F.clamped[a] ? 0.0 : rd / (rd + fpp<ENERGY>(F.p[a]));
  const double tol = sizeof(R) == 4 ? 1e-5 : 1e-9;
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double g;
      if (a == b) g = dp[a];
      else {
        const double dq = F.q[a] - F.q[b];
        const double sc = fabs(F.q[a]) + fabs(F.q[b]);
        g = fabs(dq) <= tol * sc ? 0.5 * (dp[a] + dp[b]) : (F.p[a] - F.p[b]) / dq;
      }
      W2[a][b] *= g;
    }
  // Sb = V W2 V^T
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) s += F.V[i][a] * W2[a][b] * F.V[j][b];
      Sb[i][j] = s;
    }
  // S = sym(U'^T A): U'-bar += A S-bar, A-bar = U' S-bar
  double Ab[D][D];
  dmatmul<D>(F.A, Sb, T1);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Ub1[i][j] += T1[i][j];
  dmatmul<D>(F.U1, Sb, Ab);
  // U' = rot(Q)
  double Qb[D][D];
  rot_adjoint<D>(F.U1, F.Q, Ub1, Qb);
  // Q = A P0: A-bar += Q-bar P0^T, P0-bar = A^T Q-bar
  double Pb0[D][D];
  dmatmul<D>(Qb, F.P0, T1);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Ab[i][j] += T1[i][j];
  dmatmul_tn<D>(F.A, Qb, Pb0);
  // A = J + Lam0
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      Jb[i][j] += Ab[i][j];
      Lb0[i][j] += Ab[i][j];
    }
  // J = B E_x: B-bar += J-bar E_x^T; corner vectors of G^T J-bar
  double Ex[D][D], Bd[D][D], Bbar[D][D];
  edges<D>(T, m, e, x, Ex);
  load_d<D>(B64, m, e, Bd);
  load_d<D>(Bb, m, e, Bbar);
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) s += Jb[a][k] * Ex[j][k];
      Bbar[a][j] += s;
    }
  store_d<D>(Bb, m, e, Bbar);
  store_g64<D>(gJ, e, Bd, Jb);
  double Z[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Z[i][j] = 0.0;
  store_d<D>(Ub, m, e, Z);   // U^{k-1} enters only the W-step (k_adj_wstep adds it)
  store_d<D>(Pb, m, e, Pb0);
  store_d<D>(Lb, m, e, Lb0);
}

// x-bar = G^T J-bar gathered per vertex row (all rows): free rows -> b,
// pinned rows -> accumulated into the pinned-target gradient
template <int D>
__global__ __launch_bounds__(kBlock) void k_adj_gather(int64_t nF, int64_t n, const int32_t* __restrict av_ptr,
                                                       const int32_t* __restrict av_idx, const double* __restrict g,
                                                       double* __restrict b, double* __restrict pins_bar,
                                                       double scale) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (j >= n) return;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int32_t q = av_ptr[j]; q < av_ptr[j + 1]; ++q) {
    const int64_t o = static_cast<int64_t>(av_idx[q]) * D;
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += g[o + k];
  }
  if (j < nF) {
#pragma unroll
    for (int k = 0; k < D; ++k) b[j * D + k] = acc[k];
  } else if (pins_bar) {
#pragma unroll
    for (int k = 0; k < D; ++k) pins_bar[(j - nF) * D + k] += scale * acc[k];
  }
}

template <int D, typename R>
__global__ __launch_bounds__(kBlock) void k_adj_wstep(int64_t m, const int32_t* __restrict T,
                                                      const double* __restrict B64, const R* __restrict w, R rho,
                                                      const double* __restrict x, const double* __restrict lam,
                                                      const R* __restrict U, const R* __restrict P,
                                                      const R* __restrict Lam, double* __restrict Ub,
                                                      double* __restrict Pb, double* __restrict Lb,
                                                      double* __restrict Bb, double* __restrict wb) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= m) return;
  double Bd[D][D], El[D][D], Ex[D][D], rb[D][D], J[D][D];
  load_d<D>(B64, m, e, Bd);
  edges<D>(T, m, e, lam, El);
  edges<D>(T, m, e, x, Ex);
  dmatmul<D>(Bd, El, rb);
  dmatmul<D>(Bd, Ex, J);
  R Ur[D][D], Pr[D][D];
  load_U<D, R>(U, m, e, Ur);
  load_P<D, R>(P, m, e, Pr);
  double U0[D][D], P0[D][D], Y[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      U0[i][j] = Ur[i][j];
      P0[i][j] = Pr[i][j];
    }
  dmatmul<D>(U0, P0, Y);
#pragma unroll
  for (int i = 0; i < D * D; ++i) Y[i / D][i % D] -= static_cast<double>(Lam[i * m + e]);
  const double we = static_cast<double>(w[e]), rd = static_cast<double>(rho), mu = rd * we;
  double Yb[D][D], T1[D][D], A1[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Yb[i][j] = mu * rb[i][j];
  load_d<D>(Ub, m, e, A1);
  dmatmul<D>(Yb, P0, T1);  // U-bar += Y-bar P^T
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) A1[i][j] += T1[i][j];
  store_d<D>(Ub, m, e, A1);
  load_d<D>(Pb, m, e, A1);
  dmatmul_tn<D>(U0, Yb, T1);  // P-bar += U^T Y-bar
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) A1[i][j] += T1[i][j];
  store_d<D>(Pb, m, e, A1);
  load_d<D>(Lb, m, e, A1);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) A1[i][j] -= Yb[i][j];
  store_d<D>(Lb, m, e, A1);
  // W-step implicit terms: -d/dtheta [ mu <G lam, G x - Y> ] at fixed x, lam, Y
  double Bbar[D][D], dot = 0.0;
  load_d<D>(Bb, m, e, Bbar);
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) s += (J[a][k] - Y[a][k]) * El[j][k] + rb[a][k] * Ex[j][k];
      Bbar[a][j] -= mu * s;
    }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int k = 0; k < D; ++k) dot += rb[a][k] * (J[a][k] - Y[a][k]);
  store_d<D>(Bb, m, e, Bbar);
  wb[e] -= rd * dot;
}

// x_C-bar -= L_CF lambda
template <int D>
__global__ void k_adj_pins(int64_t nC, const int32_t* __restrict lcf_ptr, const int32_t* __restrict lcf_col,
                           const double* __restrict lcf_val, const double* __restrict lam,
                           double* __restrict pins_bar) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= nC) return;
  double acc[D];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = 0.0;
  for (int32_t q = lcf_ptr[i]; q < lcf_ptr[i + 1]; ++q) {
    const double v = lcf_val[q];
    const int64_t j = lcf_col[q];
#pragma unroll
    for (int k = 0; k < D; ++k) acc[k] += v * lam[j * D + k];
  }
#pragma unroll
  for (int k = 0; k < D; ++k) pins_bar[i * D + k] -= acc[k];
}

// vertex gradients: Dm-bar = -B B-bar^T B + w-bar w B; corner vectors
// (corner 0 gets minus the sum of the others)
template <int D, typename R>
__global__ __launch_bounds__(kBlock) void k_adj_vbar(int64_t m, const double* __restrict B64, const R* __restrict w,
                                                     const double* __restrict Bb, const double* __restrict wb,
                                                     double* __restrict gV) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (e >= m) return;
  double Bd[D][D], Bbar[D][D], T1[D][D], Dmb[D][D];
  load_d<D>(B64, m, e, Bd);
  load_d<D>(Bb, m, e, Bbar);
  // T1 = B B-bar^T
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) s += Bd[i][k] * Bbar[j][k];
      T1[i][j] = s;
    }
  dmatmul<D>(T1, Bd, Dmb);
  const double ww = wb[e] * static_cast<double>(w[e]);
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) Dmb[i][j] = -Dmb[i][j] + ww * Bd[i][j];
  double* dst = gV + e * (D + 1) * D;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double s0 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      dst[(j + 1) * D + a] = Dmb[a][j];
      s0 += Dmb[a][j];
    }
    dst[a] = -s0;
  }
}

}  // namespace ffd
