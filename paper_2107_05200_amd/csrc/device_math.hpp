// Per-element device math of the local steps, templated on the arithmetic
// type R (float or double).  Everything stays in registers; no branches that
// depend on more than one element.
//
//  - roots of the P-step per eigenvalue (supplement "Solving the Optimization
//    in P"): with mu = rho * w the scalar problems depend only on rho and q:
//      SG: (1+rho) p^2 - rho q p - 1 = 0   (quadratic formula, conjugate form for q < 0)
//      SD: (1+rho) p^4 - rho q p^3 - 1 = 0 (Newton from a left bracket)
//  - Procrustes rotations (supplement "Solving the Optimization in U"):
//      d = 2: U = z / |z| with z = (Q00 + Q11) + i (Q10 - Q01)
//      d = 3: U = R1 R2^T from an SVD with det-corrected last singular vector;
//             the SVD is a one-sided (Hestenes) Jacobi iteration on the columns.
//  - symmetric eigen-decomposition: 2x2 closed-form Jacobi rotation, 3x3 cyclic Jacobi.
#pragma once
#include <hip/hip_runtime.h>

namespace ffd {
namespace dm {

template <typename R> struct Tol;
template <> struct Tol<float> {
  static constexpr float rel = 1e-7f;
  static constexpr int sweeps = 6;
};
template <> struct Tol<double> {
  static constexpr double rel = 1e-15;
  static constexpr int sweeps = 10;
};

// machine epsilon of float64 (the clamps of the paper use the same values for
// every arithmetic type of the element steps)
constexpr double kEpsM = 2.220446049250313e-16;
constexpr double kSqrtEps = 1.4901161193847656e-08;   // eps_m^(1/2)
constexpr double kInitEpsSG = 1.220703125e-04;        // eps_m^(1/4)
constexpr double kInitEpsSD = 1.1048543456039805e-02; // eps_m^(1/8)

// reciprocal: one v_rcp_f32 (1 ulp) in float32, exact division in float64
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
__device__ __forceinline__ float cbrt_(float x) { return cbrtf(x); }
__device__ __forceinline__ double cbrt_(double x) { return cbrt(x); }
__device__ __forceinline__ float log_(float x) { return logf(x); }
__device__ __forceinline__ double log_(double x) { return log(x); }
__device__ __forceinline__ float abs_(float x) { return fabsf(x); }
__device__ __forceinline__ double abs_(double x) { return fabs(x); }

// ---------------------------------------------------------------------------
// scalar roots
// ---------------------------------------------------------------------------

// symmetric gradient: positive root of (1+rho) p^2 - rho q p - 1 = 0
template <typename R>
__device__ __forceinline__ R root_sg(R q, R rho) {
  const R a = R(1) + rho;
  const R disc = sqrt_(rho * rho * q * q + R(4) * a);
  return q >= R(0) ? (rho * q + disc) * rcp_(R(2) * a) : R(2) * rcp_(disc - rho * q);
}

// symmetric Dirichlet: unique positive root of h(p) = (1+rho) p - p^-3 - rho q.
// h is increasing and concave on (0, inf), so Newton started at a point with
// h <= 0 increases monotonically to the root; it stops when a step no longer
// increases p (converged to rounding).
template <typename R>
__device__ __forceinline__ R root_sd(R q, R rho) {
  const R a = R(1) + rho;
  R p;
  if (q >= R(0)) {
    const R lo1 = sqrt_(rsqrt_(a));  // a^(-1/4)
    const R lo2 = rho * q * rcp_(a);
    p = lo1 > lo2 ? lo1 : lo2;
  } else {
    const R lo1 = sqrt_(rsqrt_(R(2) * a));
    const R lo2 = cbrt_(rcp_(R(2) * rho * (-q)));
    p = lo1 < lo2 ? lo1 : lo2;
  }
#pragma unroll 1
  for (int it = 0; it < 40; ++it) {
    const R ip = rcp_(p);
    const R ip3 = ip * ip * ip;
    const R h = a * p - ip3 - rho * q;
    const R dh = a + R(3) * ip3 * ip;
    const R pn = p - h * rcp_(dh);
    if (!(pn > p)) break;
    p = pn;
  }
  return p;
}

template <int ENERGY, typename R>
__device__ __forceinline__ R root(R q, R rho) {
  if constexpr (ENERGY == 1) return root_sg(q, rho);
  else return root_sd(q, rho);
}

// per-eigenvalue energy density on S+: SD 1/2 (p^2 + p^-2), SG 1/2 p^2 - log p
template <int ENERGY, typename R>
__device__ __forceinline__ double f_eig(R p) {
  const double pd = static_cast<double>(p);
  if constexpr (ENERGY == 1) return 0.5 * pd * pd - log(pd);
  else return 0.5 * (pd * pd + 1.0 / (pd * pd));
}

// ---------------------------------------------------------------------------
// symmetric 2x2 Jacobi rotation (Golub & Van Loan, symmetric Schur 2x2):
// returns (c, s) and t such that [c s; -s c]^T A [c s; -s c] is diagonal with
// entries app - t apq, aqq + t apq
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void schur2(R app, R apq, R aqq, R& c, R& s, R& t) {
  if (apq == R(0)) {
    c = R(1);
    s = R(0);
    t = R(0);
    return;
  }
  const R tau = (aqq - app) * rcp_(R(2) * apq);
  const R at = abs_(tau);
  // for |tau| huge the rotation is negligible: t ~ 1/(2 tau)
  t = at > R(1e18) ? R(0.5) * rcp_(tau) : (tau >= R(0) ? R(1) : R(-1)) * rcp_(at + sqrt_(R(1) + tau * tau));
  c = rsqrt_(R(1) + t * t);
  s = t * c;
}

// 2x2 symmetric eigen: S = [a b; b d] = V diag(q) V^T, V = [c s; -s c]
template <typename R>
__device__ __forceinline__ void eig2(R a, R b, R d, R q[2], R V[2][2]) {
  R c, s, t;
  schur2(a, b, d, c, s, t);
  q[0] = a - t * b;
  q[1] = d + t * b;
  V[0][0] = c;
  V[0][1] = s;
  V[1][0] = -s;
  V[1][1] = c;
}

// 3x3 symmetric eigen by cyclic Jacobi: S (symmetric, destroyed) = V diag(q) V^T
template <typename R>
__device__ __forceinline__ void eig3(R S[3][3], R q[3], R V[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = i == j ? R(1) : R(0);
#pragma unroll 1
  for (int sweep = 0; sweep < Tol<R>::sweeps; ++sweep) {
    const R off = abs_(S[0][1]) + abs_(S[0][2]) + abs_(S[1][2]);
    const R dia = abs_(S[0][0]) + abs_(S[1][1]) + abs_(S[2][2]);
    if (off <= Tol<R>::rel * R(0.1) * dia || off == R(0)) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int qq = pq == 0 ? 1 : 2;
      const int r = 3 - p - qq;
      R c, s, t;
      schur2(S[p][p], S[p][qq], S[qq][qq], c, s, t);
      if (t == R(0)) continue;
      const R apq = S[p][qq];
      S[p][p] -= t * apq;
      S[qq][qq] += t * apq;
      S[p][qq] = S[qq][p] = R(0);
      const R srp = S[r][p], srq = S[r][qq];
      S[r][p] = S[p][r] = c * srp - s * srq;
      S[r][qq] = S[qq][r] = s * srp + c * srq;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const R vp = V[i][p], vq = V[i][qq];
        V[i][p] = c * vp - s * vq;
        V[i][qq] = s * vp + c * vq;
      }
    }
  }
  q[0] = S[0][0];
  q[1] = S[1][1];
  q[2] = S[2][2];
}

// ---------------------------------------------------------------------------
// 3x3 SVD: A = U diag(sig) V^T with U, V rotations, sig[0] >= sig[1] >= |sig[2]|,
// sig[2] carrying the sign of det A.  One-sided Jacobi on the columns of A.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void svd3(const R A[3][3], R U[3][3], R sig[3], R V[3][3]) {
  R Bm[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      Bm[i][j] = A[i][j];
      V[i][j] = i == j ? R(1) : R(0);
    }
#pragma unroll 1
  for (int sweep = 0; sweep < Tol<R>::sweeps; ++sweep) {
    bool rotated = false;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0;
      const int q = pq == 0 ? 1 : 2;
      const R al = Bm[0][p] * Bm[0][p] + Bm[1][p] * Bm[1][p] + Bm[2][p] * Bm[2][p];
      const R be = Bm[0][q] * Bm[0][q] + Bm[1][q] * Bm[1][q] + Bm[2][q] * Bm[2][q];
      const R ga = Bm[0][p] * Bm[0][q] + Bm[1][p] * Bm[1][q] + Bm[2][p] * Bm[2][q];
      if (!(abs_(ga) > Tol<R>::rel * sqrt_(al * be))) continue;
      rotated = true;
      const R zeta = (be - al) * rcp_(R(2) * ga);
      const R az = abs_(zeta);
      const R t = az > R(1e18) ? R(0.5) * rcp_(zeta) : (zeta >= R(0) ? R(1) : R(-1)) * rcp_(az + sqrt_(R(1) + zeta * zeta));
      const R c = rsqrt_(R(1) + t * t);
      const R s = c * t;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const R bp = Bm[i][p], bq = Bm[i][q];
        Bm[i][p] = c * bp - s * bq;
        Bm[i][q] = s * bp + c * bq;
        const R vp = V[i][p], vq = V[i][q];
        V[i][p] = c * vp - s * vq;
        V[i][q] = s * vp + c * vq;
      }
    }
    if (!rotated) break;
  }
  R n[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) n[j] = Bm[0][j] * Bm[0][j] + Bm[1][j] * Bm[1][j] + Bm[2][j] * Bm[2][j];
  // sort columns by descending norm; each swap negates one column so V stays a rotation
  auto swapcols = [&](int a, int b) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      R t = Bm[i][a];
      Bm[i][a] = -Bm[i][b];
      Bm[i][b] = t;
      t = V[i][a];
      V[i][a] = -V[i][b];
      V[i][b] = t;
    }
    const R t = n[a];
    n[a] = n[b];
    n[b] = t;
  };
  if (n[0] < n[1]) swapcols(0, 1);
  if (n[0] < n[2]) swapcols(0, 2);
  if (n[1] < n[2]) swapcols(1, 2);
  // U = [u1, u2, u1 x u2]
  R u1[3], u2[3];
  if (n[0] > R(0)) {
    const R inv = rsqrt_(n[0]);
#pragma unroll
    for (int i = 0; i < 3; ++i) u1[i] = Bm[i][0] * inv;
  } else {
    u1[0] = R(1);
    u1[1] = R(0);
    u1[2] = R(0);
  }
  const R d12 = u1[0] * Bm[0][1] + u1[1] * Bm[1][1] + u1[2] * Bm[2][1];
#pragma unroll
  for (int i = 0; i < 3; ++i) u2[i] = Bm[i][1] - d12 * u1[i];
  R l2 = u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2];
  if (!(l2 > R(1e-24) * (n[0] > R(0) ? n[0] : R(1)))) {
    // rank <= 1: any unit vector orthogonal to u1
    const int ax = (abs_(u1[0]) <= abs_(u1[1]) && abs_(u1[0]) <= abs_(u1[2])) ? 0 : (abs_(u1[1]) <= abs_(u1[2]) ? 1 : 2);
    R e[3] = {R(0), R(0), R(0)};
    e[ax] = R(1);
    u2[0] = u1[1] * e[2] - u1[2] * e[1];
    u2[1] = u1[2] * e[0] - u1[0] * e[2];
    u2[2] = u1[0] * e[1] - u1[1] * e[0];
    l2 = u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2];
  }
  const R inv2 = rsqrt_(l2);
#pragma unroll
  for (int i = 0; i < 3; ++i) u2[i] *= inv2;
  const R u3[3] = {u1[1] * u2[2] - u1[2] * u2[1], u1[2] * u2[0] - u1[0] * u2[2], u1[0] * u2[1] - u1[1] * u2[0]};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    U[i][0] = u1[i];
    U[i][1] = u2[i];
    U[i][2] = u3[i];
  }
  sig[0] = u1[0] * Bm[0][0] + u1[1] * Bm[1][0] + u1[2] * Bm[2][0];
  sig[1] = u2[0] * Bm[0][1] + u2[1] * Bm[1][1] + u2[2] * Bm[2][1];
  sig[2] = u3[0] * Bm[0][2] + u3[1] * Bm[1][2] + u3[2] * Bm[2][2];
}

}  // namespace dm
}  // namespace ffd
