// Host setup: geometry, global matrix, ordering and the FP64 factor.
//
// Paper passages: the Jacobian / gradient operator G (Def. "Piecewise
// constant Jacobian" and supplement "Computing the Jacobian Map"); the W-step
// system L W = G^T r with L = G^T M G, M = diag(mu) (eq. solvinginw), fixed
// vertices eliminated, and a factorisation computed once and reused by a
// back-substitution every iteration (Section "Efficient Evaluation &
// Parallelization").
//
// The factorisation is multifrontal over a geometric nested-dissection tree.
// For each tree node s (columns C, row structure R below) it stores
//   forward panel  [Linv; -M]   with Linv = L_CC^{-1}, M = L_RC * Linv,
//   backward panel [Linv^T | -M^T],
// so both triangular solves become dense matrix-vector products per node with
// no sequential dependency inside a node (the partitioned-inverse form of a
// supernodal triangular solve).
#include "setup.hpp"

#include <omp.h>
#include <tuple>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>

#include "dense.hpp"

namespace ffd {

namespace {

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ----------------------------------------------------------------------------
// nested dissection on source coordinates
// ----------------------------------------------------------------------------

struct NDBuilder {
  const std::vector<int64_t>& adj_ptr;
  const std::vector<int32_t>& adj;
  const double* V;
  int din;
  int leaf;
  const std::vector<uint8_t>& is_pinned;
  std::vector<int32_t> stamp;
  std::vector<int8_t> side;
  int32_t cur = 0;
  // tree (old vertex ids per node)
  std::vector<std::vector<int32_t>> cols;
  std::vector<std::vector<int32_t>> kids;

  NDBuilder(const std::vector<int64_t>& ap, const std::vector<int32_t>& a, const double* V_, int din_,
            int leaf_, const std::vector<uint8_t>& pinned, int64_t n)
      : adj_ptr(ap), adj(a), V(V_), din(din_), leaf(leaf_), is_pinned(pinned), stamp(n, -1), side(n, 0) {}

  int new_node(std::vector<int32_t>&& c, std::vector<int32_t>&& k) {
    cols.push_back(std::move(c));
    kids.push_back(std::move(k));
    return static_cast<int>(cols.size()) - 1;
  }

  // returns the roots of the forest built for S
  std::vector<int32_t> run(std::vector<int32_t>& S) {
    if (S.empty()) return {};
    if (static_cast<int>(S.size()) <= leaf) return {new_node(std::move(S), {})};
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t v : S)
      for (int a = 0; a < din; ++a) {
        lo[a] = std::min(lo[a], V[static_cast<int64_t>(v) * din + a]);
        hi[a] = std::max(hi[a], V[static_cast<int64_t>(v) * din + a]);
      }
    int ax = 0;
    for (int a = 1; a < din; ++a)
      if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
    std::vector<double> co(S.size());
    for (size_t i = 0; i < S.size(); ++i) co[i] = V[static_cast<int64_t>(S[i]) * din + ax];
    std::vector<double> tmp = co;
    const size_t k = S.size() / 2;
    std::nth_element(tmp.begin(), tmp.begin() + k, tmp.end());
    const double med = tmp[k];
    const int32_t st = cur++;
    size_t nleft = 0;
    for (size_t i = 0; i < S.size(); ++i) nleft += co[i] < med;
    bool le = false;
    if (nleft == 0) {  // ties at the minimum: split at <= med instead
      le = true;
      for (size_t i = 0; i < S.size(); ++i) nleft += co[i] <= med;
    }
    for (size_t i = 0; i < S.size(); ++i) {
      stamp[S[i]] = st;
      const bool isleft = le ? co[i] <= med : co[i] < med;
      side[S[i]] = isleft ? 1 : 2;
    }
    if (nleft == 0 || nleft == S.size()) {  // all coordinates equal: split by position
      for (size_t i = 0; i < S.size(); ++i) side[S[i]] = i < k ? 1 : 2;
    }
    std::vector<int32_t> sepL, sepR;
    for (int32_t v : S) {
      const int8_t sv = side[v];
      bool touches = false;
      for (int64_t e = adj_ptr[v]; e < adj_ptr[v + 1]; ++e) {
        const int32_t u = adj[e];
        if (stamp[u] == st && side[u] != sv) {
          touches = true;
          break;
        }
      }
      if (touches) (sv == 1 ? sepL : sepR).push_back(v);
    }
    const bool useL = sepL.size() <= sepR.size();
    std::vector<int32_t>& sep = useL ? sepL : sepR;
    for (int32_t v : sep) side[v] = 3;
    std::vector<int32_t> L, R;
    L.reserve(S.size() / 2 + 1);
    R.reserve(S.size() / 2 + 1);
    for (int32_t v : S) {
      if (side[v] == 1) L.push_back(v);
      else if (side[v] == 2) R.push_back(v);
    }
    std::vector<int32_t>().swap(S);
    std::vector<int32_t> sep_copy = sep;
    std::vector<int32_t> roots = run(L);
    std::vector<int32_t> rr = run(R);
    roots.insert(roots.end(), rr.begin(), rr.end());
    if (sep_copy.empty()) return roots;
    return {new_node(std::move(sep_copy), std::move(roots))};
  }
};

}  // namespace

int element_geometry(int d, int din, int64_t m, const double* V, int64_t n, const int32_t* T,
                     std::vector<double>& B, std::vector<double>& w, std::string& err) {
  B.assign(static_cast<size_t>(m) * d * d, 0.0);
  w.assign(static_cast<size_t>(m), 0.0);
  int bad = 0;
  int64_t bad_elem = -1;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    const int32_t* t = T + e * (d + 1);
    double E[3][3];  // E[j][k]: edge j, source coordinate k
    for (int j = 0; j < d; ++j)
      for (int k = 0; k < din; ++k)
        E[j][k] = V[static_cast<int64_t>(t[j + 1]) * din + k] - V[static_cast<int64_t>(t[0]) * din + k];
    double Dm[3][3] = {};  // columns are the edges in the element frame
    if (din == d) {
      for (int a = 0; a < d; ++a)
        for (int j = 0; j < d; ++j) Dm[a][j] = E[j][a];
    } else {  // triangle in 3D: intrinsic frame e1 = edge 1 direction, e2 = n x e1
      const double l1 = std::sqrt(E[0][0] * E[0][0] + E[0][1] * E[0][1] + E[0][2] * E[0][2]);
      double e1[3] = {E[0][0] / l1, E[0][1] / l1, E[0][2] / l1};
      double nn[3] = {E[0][1] * E[1][2] - E[0][2] * E[1][1], E[0][2] * E[1][0] - E[0][0] * E[1][2],
                      E[0][0] * E[1][1] - E[0][1] * E[1][0]};
      const double ln = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
      for (double& x : nn) x /= ln;
      double e2[3] = {nn[1] * e1[2] - nn[2] * e1[1], nn[2] * e1[0] - nn[0] * e1[2], nn[0] * e1[1] - nn[1] * e1[0]};
      for (int j = 0; j < 2; ++j) {
        Dm[0][j] = E[j][0] * e1[0] + E[j][1] * e1[1] + E[j][2] * e1[2];
        Dm[1][j] = E[j][0] * e2[0] + E[j][1] * e2[1] + E[j][2] * e2[2];
      }
    }
    double det, inv[3][3];
    if (d == 2) {
      det = Dm[0][0] * Dm[1][1] - Dm[0][1] * Dm[1][0];
      inv[0][0] = Dm[1][1] / det;
      inv[0][1] = -Dm[0][1] / det;
      inv[1][0] = -Dm[1][0] / det;
      inv[1][1] = Dm[0][0] / det;
    } else {
      const double c00 = Dm[1][1] * Dm[2][2] - Dm[1][2] * Dm[2][1];
      const double c01 = Dm[1][2] * Dm[2][0] - Dm[1][0] * Dm[2][2];
      const double c02 = Dm[1][0] * Dm[2][1] - Dm[1][1] * Dm[2][0];
      det = Dm[0][0] * c00 + Dm[0][1] * c01 + Dm[0][2] * c02;
      inv[0][0] = c00 / det;
      inv[1][0] = c01 / det;
      inv[2][0] = c02 / det;
      inv[0][1] = (Dm[0][2] * Dm[2][1] - Dm[0][1] * Dm[2][2]) / det;
      inv[1][1] = (Dm[0][0] * Dm[2][2] - Dm[0][2] * Dm[2][0]) / det;
      inv[2][1] = (Dm[0][1] * Dm[2][0] - Dm[0][0] * Dm[2][1]) / det;
      inv[0][2] = (Dm[0][1] * Dm[1][2] - Dm[0][2] * Dm[1][1]) / det;
      inv[1][2] = (Dm[0][2] * Dm[1][0] - Dm[0][0] * Dm[1][2]) / det;
      inv[2][2] = (Dm[0][0] * Dm[1][1] - Dm[0][1] * Dm[1][0]) / det;
    }
    const double area = std::fabs(det) / (d == 2 ? 2.0 : 6.0);
    bool ok = std::isfinite(area) && area > 1e-300;
    for (int a = 0; a < d; ++a)
      for (int j = 0; j < d; ++j) {
        const double v = inv[j][a];  // B = Dm^{-T}
        B[static_cast<size_t>(e) * d * d + a * d + j] = v;
        ok = ok && std::isfinite(v);
      }
    w[e] = area;
    if (!ok) {
#pragma omp critical
      {
        bad = 1;
        if (bad_elem < 0 || e < bad_elem) bad_elem = e;
      }
    }
  }
  (void)n;
  if (bad) {
    err = "degenerate element " + std::to_string(bad_elem) + " (zero or non-finite area/volume)";
    return ERR_DEGENERATE_ELEMENT;
  }
  return OK;
}

int build_setup(const SetupInput& in, Setup& S, std::string& err) {
  const int d = in.d, din = in.din;
  const int64_t n = in.n, m = in.m;
  const int nc = d + 1;
  if (!(d == 2 || d == 3) || !(din == d || (d == 2 && din == 3))) {
    err = "unsupported (simplex_dim, dim_in)";
    return ERR_INVALID_ARG;
  }
  if (n <= 0 || m <= 0 || !in.V || !in.T || n > INT32_MAX / 2 || m > INT32_MAX / 4) {
    err = "empty or oversized mesh";
    return ERR_INVALID_ARG;
  }
  if (!(in.rho > 0) || !std::isfinite(in.rho)) {
    err = "rho must be positive and finite";
    return ERR_INVALID_ARG;
  }
  if (in.mu_elem)
    for (int64_t e = 0; e < m; ++e)
      if (!(in.mu_elem[e] > 0) || !std::isfinite(in.mu_elem[e])) {
        err = "per-element penalties must be positive and finite";
        return ERR_INVALID_ARG;
      }
  for (int64_t i = 0; i < n * din; ++i)
    if (!std::isfinite(in.V[i])) {
      err = "non-finite source vertex";
      return ERR_NOT_FINITE;
    }
  for (int64_t i = 0; i < m * nc; ++i)
    if (in.T[i] < 0 || in.T[i] >= n) {
      err = "element index out of range";
      return ERR_INVALID_ARG;
    }
  for (int64_t e = 0; e < m; ++e)
    for (int a = 0; a < nc; ++a)
      for (int b = a + 1; b < nc; ++b)
        if (in.T[e * nc + a] == in.T[e * nc + b]) {
          err = "element " + std::to_string(e) + " repeats a vertex";
          return ERR_DEGENERATE_ELEMENT;
        }
  if (in.n_con < 0 || (in.n_con > 0 && (!in.con_ptr || !in.con_col || !in.con_val || in.tutte))) {
    err = "bad constraint arrays";
    return ERR_INVALID_ARG;
  }
  if (in.n_con > 0) {
    if (in.con_ptr[0] != 0) {
      err = "constraint row_ptr must start at 0";
      return ERR_INVALID_ARG;
    }
    for (int64_t a = 0; a < in.n_con; ++a) {
      if (in.con_ptr[a + 1] <= in.con_ptr[a]) {
        err = "constraint row " + std::to_string(a) + " is empty or row_ptr decreases";
        return ERR_INVALID_ARG;
      }
      for (int64_t q = in.con_ptr[a]; q < in.con_ptr[a + 1]; ++q) {
        if (in.con_col[q] < 0 || in.con_col[q] >= n) {
          err = "constraint column out of range";
          return ERR_INVALID_ARG;
        }
        if (!std::isfinite(in.con_val[q])) {
          err = "non-finite constraint coefficient";
          return ERR_NOT_FINITE;
        }
        for (int64_t q2 = in.con_ptr[a]; q2 < q; ++q2)
          if (in.con_col[q2] == in.con_col[q]) {
            err = "constraint row " + std::to_string(a) + " repeats a vertex";
            return ERR_INVALID_ARG;
          }
      }
    }
  }
  std::vector<uint8_t> pinned(n, 0);
  for (int64_t i = 0; i < in.n_pinned; ++i) {
    const int32_t v = in.pinned_idx[i];
    if (v < 0 || v >= n || pinned[v]) {
      err = "pinned index out of range or repeated";
      return ERR_INVALID_ARG;
    }
    pinned[v] = 1;
  }
  if (in.elem_energy)
    for (int64_t e = 0; e < m; ++e)
      if (in.elem_energy[e] != 0 && in.elem_energy[e] != 1) {
        err = "element energies must be 0 or 1";
        return ERR_INVALID_ARG;
      }
  S.d = d;
  S.din = din;
  S.n = n;
  S.m = m;
  S.rho = in.rho;
  S.nC = in.n_pinned;
  S.nF = n - in.n_pinned;

  double t0 = now();
  std::vector<double> B0, w0;
  int st = element_geometry(d, din, m, in.V, n, in.T, B0, w0, err);
  if (st) return st;

  // vertex -> element incidence
  std::vector<int64_t> inc_ptr(n + 1, 0);
  for (int64_t i = 0; i < m * nc; ++i) inc_ptr[in.T[i] + 1]++;
  for (int64_t v = 0; v < n; ++v) inc_ptr[v + 1] += inc_ptr[v];
  std::vector<int32_t> inc(m * nc);
  {
    std::vector<int64_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
    for (int64_t e = 0; e < m; ++e)
      for (int c = 0; c < nc; ++c) inc[fill[in.T[e * nc + c]]++] = static_cast<int32_t>(e * nc + c);
  }
  // L = sum_e mu_e C_e^T C_e in the input numbering (rows include self)
  std::vector<int64_t> Lptr(n + 1, 0);
  std::vector<std::vector<int32_t>> rowpat(n);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t v = 0; v < n; ++v) {
    std::vector<int32_t>& p = rowpat[v];
    for (int64_t k = inc_ptr[v]; k < inc_ptr[v + 1]; ++k) {
      const int64_t e = inc[k] / nc;
      for (int c = 0; c < nc; ++c) p.push_back(in.T[e * nc + c]);
    }
    std::sort(p.begin(), p.end());
    p.erase(std::unique(p.begin(), p.end()), p.end());
  }
  for (int64_t v = 0; v < n; ++v) Lptr[v + 1] = Lptr[v] + static_cast<int64_t>(rowpat[v].size());
  std::vector<int32_t> Lcol(Lptr[n]);
  std::vector<double> Lval(Lptr[n], 0.0);
  int64_t zero_edge = -1;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t v = 0; v < n; ++v) {
    std::copy(rowpat[v].begin(), rowpat[v].end(), Lcol.begin() + Lptr[v]);
    std::vector<int32_t>().swap(rowpat[v]);
    if (in.tutte) {
      // Tutte's energy (supplement "Tutte's Energy"): every edge (v, u) of an
      // element counted once with weight 1 / |V_v - V_u|; its Hessian is twice
      // this graph Laplacian, whose minimiser with the fixed rows is the map
      double diag = 0.0;
      int64_t self = -1;
      for (int64_t k = Lptr[v]; k < Lptr[v + 1]; ++k) {
        const int64_t u = Lcol[k];
        if (u == v) {
          self = k;
          continue;
        }
        double len2 = 0.0;
        for (int a = 0; a < din; ++a) {
          const double dv = in.V[v * din + a] - in.V[u * din + a];
          len2 += dv * dv;
        }
        if (!(len2 > 0.0)) {
#pragma omp critical
          zero_edge = v;
          continue;
        }
        const double wgt = 1.0 / std::sqrt(len2);
        Lval[k] = -wgt;
        diag += wgt;
      }
      Lval[self] = diag;
      continue;
    }
    const int32_t* cb = Lcol.data() + Lptr[v];
    const int64_t len = Lptr[v + 1] - Lptr[v];
    for (int64_t k = inc_ptr[v]; k < inc_ptr[v + 1]; ++k) {
      const int64_t e = inc[k] / nc;
      const int cv = inc[k] % nc;
      const double mu = in.mu_elem ? in.mu_elem[e] : in.rho * w0[e];
      const double* Be = B0.data() + e * d * d;
      // C[a][0] = -sum_j B[a][j], C[a][j+1] = B[a][j]
      double C[3][4];
      for (int a = 0; a < d; ++a) {
        double s = 0;
        for (int j = 0; j < d; ++j) {
          C[a][j + 1] = Be[a * d + j];
          s += Be[a * d + j];
        }
        C[a][0] = -s;
      }
      for (int c2 = 0; c2 < nc; ++c2) {
        double val = 0;
        for (int a = 0; a < d; ++a) val += C[a][cv] * C[a][c2];
        const int32_t u = in.T[e * nc + c2];
        const int64_t pos = std::lower_bound(cb, cb + len, u) - cb;
        Lval[Lptr[v] + pos] += mu * val;
      }
    }
  }
  std::vector<std::vector<int32_t>>().swap(rowpat);
  if (zero_edge >= 0) {
    err = "an edge at vertex " + std::to_string(zero_edge) + " has zero length (Tutte weight undefined)";
    return ERR_DEGENERATE_ELEMENT;
  }
  S.t_geometry = now() - t0;

  // every connected component needs a pinned vertex (G maps constants to 0),
  // or, with general constraints, the constraints must fix the translations
  // of the components without one: A times their indicator vectors has full
  // column rank
  {
    std::vector<int32_t> comp(n, -1), stack;
    std::vector<int64_t> unpinned;  // one vertex of each component without a pin
    int32_t nco = 0;
    for (int64_t s0 = 0; s0 < n; ++s0) {
      if (comp[s0] >= 0) continue;
      bool has_pin = false;
      stack.push_back(static_cast<int32_t>(s0));
      comp[s0] = nco;
      while (!stack.empty()) {
        const int32_t v = stack.back();
        stack.pop_back();
        has_pin |= pinned[v] != 0;
        for (int64_t k = Lptr[v]; k < Lptr[v + 1]; ++k)
          if (comp[Lcol[k]] < 0) {
            comp[Lcol[k]] = nco;
            stack.push_back(Lcol[k]);
          }
      }
      if (!has_pin) unpinned.push_back(s0);
      ++nco;
    }
    if (!unpinned.empty() && in.n_con == 0) {
      err = "a connected component (containing vertex " + std::to_string(unpinned[0]) +
            ") has no pinned vertex: the W-step system is singular";
      return ERR_SINGULAR_SYSTEM;
    }
    if (!unpinned.empty()) {
      const int64_t nu = static_cast<int64_t>(unpinned.size());
      if (nu > 4096) {
        err = "more than 4096 connected components without a pinned vertex";
        return ERR_INVALID_ARG;
      }
      std::vector<int32_t> slot(nco, -1);
      for (int64_t i = 0; i < nu; ++i) slot[comp[unpinned[i]]] = static_cast<int32_t>(i);
      // Gram matrix of the columns A 1_c, then a Cholesky with a relative pivot floor
      std::vector<double> Mrow(nu), Gm(nu * nu, 0.0);
      for (int64_t a = 0; a < in.n_con; ++a) {
        std::fill(Mrow.begin(), Mrow.end(), 0.0);
        for (int64_t q = in.con_ptr[a]; q < in.con_ptr[a + 1]; ++q) {
          const int32_t c = slot[comp[in.con_col[q]]];
          if (c >= 0 && !pinned[in.con_col[q]]) Mrow[c] += in.con_val[q];
        }
        for (int64_t i = 0; i < nu; ++i)
          if (Mrow[i] != 0.0)
            for (int64_t j = 0; j < nu; ++j) Gm[i * nu + j] += Mrow[i] * Mrow[j];
      }
      double dmax = 0.0;
      for (int64_t i = 0; i < nu; ++i) dmax = std::max(dmax, Gm[i * nu + i]);
      bool ok = dmax > 0.0;
      for (int64_t j = 0; ok && j < nu; ++j) {
        double dj = Gm[j * nu + j];
        for (int64_t l = 0; l < j; ++l) dj -= Gm[j * nu + l] * Gm[j * nu + l];
        if (!(dj > 1e-12 * dmax)) {
          ok = false;
          break;
        }
        dj = std::sqrt(dj);
        Gm[j * nu + j] = dj;
        for (int64_t i = j + 1; i < nu; ++i) {
          double t = Gm[i * nu + j];
          for (int64_t l = 0; l < j; ++l) t -= Gm[i * nu + l] * Gm[j * nu + l];
          Gm[i * nu + j] = t / dj;
        }
      }
      if (!ok) {
        err = "the constraints leave the translation of a component without pinned vertex free "
              "(containing vertex " + std::to_string(unpinned[0]) + "): the W-step system is singular";
        return ERR_SINGULAR_SYSTEM;
      }
    }
  }
  // constraint rows must involve a free vertex
  for (int64_t a = 0; a < in.n_con; ++a) {
    bool any_free = false;
    for (int64_t q = in.con_ptr[a]; q < in.con_ptr[a + 1]; ++q) any_free |= !pinned[in.con_col[q]];
    if (!any_free) {
      err = "constraint row " + std::to_string(a) + " involves pinned vertices only";
      return ERR_INVALID_ARG;
    }
  }
  // gamma A_F^T A_F: gamma scales the rows of A to the mean diagonal of L_FF
  // (any gamma > 0 gives the same constrained minimiser); its pattern joins L's
  if (in.n_con > 0) {
    double dsum = 0.0, asum = 0.0;
    for (int64_t v = 0; v < n; ++v) {
      if (pinned[v]) continue;
      const int64_t pos = std::lower_bound(Lcol.begin() + Lptr[v], Lcol.begin() + Lptr[v + 1], static_cast<int32_t>(v)) -
                          Lcol.begin();
      dsum += Lval[pos];
    }
    for (int64_t a = 0; a < in.n_con; ++a)
      for (int64_t q = in.con_ptr[a]; q < in.con_ptr[a + 1]; ++q)
        if (!pinned[in.con_col[q]]) asum += in.con_val[q] * in.con_val[q];
    const double gamma = (dsum / static_cast<double>(n - in.n_pinned)) / (asum / static_cast<double>(in.n_con));
    S.con_gamma = gamma;
    // vertex -> constraint rows
    std::vector<int64_t> vc_ptr(n + 1, 0);
    for (int64_t q = 0; q < in.con_ptr[in.n_con]; ++q) vc_ptr[in.con_col[q] + 1]++;
    for (int64_t v = 0; v < n; ++v) vc_ptr[v + 1] += vc_ptr[v];
    std::vector<int64_t> vc_q(in.con_ptr[in.n_con]);
    {
      std::vector<int64_t> fill(vc_ptr.begin(), vc_ptr.end() - 1);
      for (int64_t a = 0; a < in.n_con; ++a)
        for (int64_t q = in.con_ptr[a]; q < in.con_ptr[a + 1]; ++q) vc_q[fill[in.con_col[q]]++] = q;
    }
    std::vector<int64_t> qrow(in.con_ptr[in.n_con]);
    for (int64_t a = 0; a < in.n_con; ++a)
      for (int64_t q = in.con_ptr[a]; q < in.con_ptr[a + 1]; ++q) qrow[q] = a;
    // merge the pattern and the values row by row
    std::vector<int64_t> Nptr(n + 1, 0);
    std::vector<std::vector<std::pair<int32_t, double>>> extra(n);
    for (int64_t v = 0; v < n; ++v) {
      if (pinned[v]) continue;
      for (int64_t k = vc_ptr[v]; k < vc_ptr[v + 1]; ++k) {
        const int64_t q = vc_q[k], a = qrow[q];
        for (int64_t q2 = in.con_ptr[a]; q2 < in.con_ptr[a + 1]; ++q2)
          if (!pinned[in.con_col[q2]]) extra[v].push_back({in.con_col[q2], gamma * in.con_val[q] * in.con_val[q2]});
      }
      std::sort(extra[v].begin(), extra[v].end(),
                [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) { return x.first < y.first; });
    }
    std::vector<int32_t> Ncol;
    std::vector<double> Nval;
    Ncol.reserve(Lcol.size());
    Nval.reserve(Lcol.size());
    for (int64_t v = 0; v < n; ++v) {
      int64_t k = Lptr[v];
      size_t e = 0;
      const auto& ex = extra[v];
      while (k < Lptr[v + 1] || e < ex.size()) {
        int32_t col;
        if (e >= ex.size() || (k < Lptr[v + 1] && Lcol[k] <= ex[e].first)) col = Lcol[k];
        else col = ex[e].first;
        double val = 0.0;
        while (k < Lptr[v + 1] && Lcol[k] == col) val += Lval[k++];
        while (e < ex.size() && ex[e].first == col) val += ex[e++].second;
        Ncol.push_back(col);
        Nval.push_back(val);
      }
      Nptr[v + 1] = static_cast<int64_t>(Ncol.size());
    }
    Lptr.swap(Nptr);
    Lcol.swap(Ncol);
    Lval.swap(Nval);
  }

  // ---- ordering -------------------------------------------------------------
  t0 = now();
  int nn = 0;                                 // tree nodes
  std::vector<std::vector<int32_t>> strct;    // row structure below each node's diagonal block
  int64_t pf = 0;                             // panel entries
  if (in.structure) {
    // the structure of an earlier set-up (it depends on the pattern only)
    const Setup& P = *in.structure;
    S.vnew2old = P.vnew2old;
    S.vold2new = P.vold2new;
    S.nodes = P.nodes;
    S.children = P.children;
    S.struct_idx = P.struct_idx;
    S.panel_entries = P.panel_entries;
    nn = static_cast<int>(S.nodes.size());
    strct.resize(nn);
    for (int i = 0; i < nn; ++i)
      strct[i].assign(S.struct_idx.begin() + S.nodes[i].soff, S.struct_idx.begin() + S.nodes[i].soff + S.nodes[i].r);
    pf = S.panel_entries;
  } else {
  std::vector<int64_t> aptr(n + 1, 0);
  std::vector<int32_t> adjv;
  adjv.reserve(Lptr[n]);
  for (int64_t v = 0; v < n; ++v) {
    for (int64_t k = Lptr[v]; k < Lptr[v + 1]; ++k)
      if (Lcol[k] != v && !pinned[Lcol[k]]) adjv.push_back(Lcol[k]);
    aptr[v + 1] = static_cast<int64_t>(adjv.size());
  }
  // default leaf sizes: on the 64^3 tet cube 60 gives one level fewer than
  // 48 for 1% more factor bytes, and the shallower level chain solves faster
  int leaf = in.leaf_size > 0 ? in.leaf_size : (d == 3 ? 60 : 64);
  NDBuilder nd(aptr, adjv, in.V, din, leaf, pinned, n);
  std::vector<int32_t> freev;
  freev.reserve(S.nF);
  for (int64_t v = 0; v < n; ++v)
    if (!pinned[v]) freev.push_back(static_cast<int32_t>(v));
  // nested dissection per connected component of the free-vertex graph, so
  // that separate meshes (a batch of charts) never share a separator
  std::vector<int32_t> roots;
  {
    std::vector<int32_t> comp(n, -1), stack;
    int32_t ncomp = 0;
    std::vector<std::vector<int32_t>> members;
    for (int32_t s0 : freev) {
      if (comp[s0] >= 0) continue;
      members.emplace_back();
      comp[s0] = ncomp;
      stack.push_back(s0);
      while (!stack.empty()) {
        const int32_t v = stack.back();
        stack.pop_back();
        members.back().push_back(v);
        for (int64_t k = aptr[v]; k < aptr[v + 1]; ++k)
          if (comp[adjv[k]] < 0) {
            comp[adjv[k]] = ncomp;
            stack.push_back(adjv[k]);
          }
      }
      ++ncomp;
    }
    std::vector<int32_t>().swap(freev);
    // the level count is set by the tallest tree, the largest component's:
    // components of at most a quarter of its size take leaves of 32, which
    // cuts their factor bytes (leaf blocks are dense) without adding levels
    size_t nmax = 0;
    for (const auto& mem : members) nmax = std::max(nmax, mem.size());
    for (auto& mem : members) {
      std::sort(mem.begin(), mem.end());
      nd.leaf = in.leaf_size > 0 || 4 * mem.size() > nmax ? leaf : std::min(leaf, 32);
      std::vector<int32_t> r = nd.run(mem);
      roots.insert(roots.end(), r.begin(), r.end());
    }
  }
  nn = static_cast<int>(nd.cols.size());
  // postorder numbering
  S.vnew2old.assign(n, -1);
  S.vold2new.assign(n, -1);
  std::vector<int32_t> order;  // nodes in postorder
  order.reserve(nn);
  {
    std::vector<std::pair<int32_t, int>> stk;
    for (auto it = roots.rbegin(); it != roots.rend(); ++it) stk.push_back({*it, 0});
    while (!stk.empty()) {
      auto& top = stk.back();
      const int32_t s = top.first;
      if (top.second < static_cast<int>(nd.kids[s].size())) {
        const int32_t ch = nd.kids[s][top.second++];
        stk.push_back({ch, 0});
      } else {
        order.push_back(s);
        stk.pop_back();
      }
    }
  }
  std::vector<int32_t> node_id(nn);  // builder node -> postorder index
  for (int i = 0; i < nn; ++i) node_id[order[i]] = i;
  S.nodes.assign(nn, SolveNode());
  S.children.assign(nn, {});
  {
    int32_t next = 0;
    for (int i = 0; i < nn; ++i) {
      const int32_t s = order[i];
      SolveNode& N = S.nodes[i];
      N.first = next;
      N.c = static_cast<int32_t>(nd.cols[s].size());
      for (int32_t v : nd.cols[s]) {
        S.vnew2old[next] = v;
        S.vold2new[v] = next;
        ++next;
      }
      for (int32_t ch : nd.kids[s]) S.children[i].push_back(node_id[ch]);
    }
    for (int64_t i = 0; i < in.n_pinned; ++i) {
      S.vnew2old[S.nF + i] = in.pinned_idx[i];
      S.vold2new[in.pinned_idx[i]] = static_cast<int32_t>(S.nF + i);
    }
  }
  S.t_order = now() - t0;

  // ---- symbolic ---------------------------------------------------------------
  t0 = now();
  strct.assign(nn, {});
  for (int i = 0; i < nn; ++i) {
    SolveNode& N = S.nodes[i];
    const int32_t last = N.first + N.c - 1;
    std::vector<int32_t> acc;
    for (int32_t j = 0; j < N.c; ++j) {
      const int32_t v = S.vnew2old[N.first + j];
      for (int64_t k = aptr[v]; k < aptr[v + 1]; ++k) {
        const int32_t u = S.vold2new[adjv[k]];
        if (u > last) acc.push_back(u);
      }
    }
    for (int32_t ch : S.children[i])
      for (int32_t u : strct[ch])
        if (u > last) acc.push_back(u);
    std::sort(acc.begin(), acc.end());
    acc.erase(std::unique(acc.begin(), acc.end()), acc.end());
    strct[i] = std::move(acc);
    N.r = static_cast<int32_t>(strct[i].size());
    int lvl = 0;
    for (int32_t ch : S.children[i]) lvl = std::max(lvl, S.nodes[ch].level + 1);
    N.level = lvl;
  }
  int64_t uo = 0, so = 0, po = 0;
  pf = 0;
  double flops = 0;
  int64_t fnnz = 0;
  int nlev = 0;
  for (int i = 0; i < nn; ++i) {
    SolveNode& N = S.nodes[i];
    N.pf = pf;
    N.uoff = uo;
    N.soff = so;
    N.poff = po;
    const double c = N.c, r = N.r;
    pf += static_cast<int64_t>(N.c + N.r) * N.c;
    uo += N.r;
    so += N.r;
    po += N.c + N.r + 1;
    flops += c * c * c / 3 + r * c * c + r * r * c + c * c * c / 3 + r * c * c;
    fnnz += static_cast<int64_t>(N.c) * (N.c + 1) / 2 + static_cast<int64_t>(N.c) * N.r;
    nlev = std::max(nlev, N.level + 1);
  }
  S.panel_entries = pf;
  S.ubuf_rows = uo;
  S.factor_flops = flops;
  S.factor_nnz = fnnz;
  S.struct_idx.resize(so);
  for (int i = 0; i < nn; ++i)
    std::copy(strct[i].begin(), strct[i].end(), S.struct_idx.begin() + S.nodes[i].soff);
  // forward pull lists: front position p of node s receives update rows of its
  // children (child update row i -> global index strct[child][i])
  S.pull_ptr.assign(po, 0);
  {
    std::vector<int64_t> cnt(po, 0);
    for (int i = 0; i < nn; ++i) {
      const SolveNode& N = S.nodes[i];
      const int32_t* sb = strct[i].data();
      for (int32_t ch : S.children[i])
        for (int32_t g : strct[ch]) {
          const int64_t p = g < N.first + N.c ? g - N.first
                                              : N.c + (std::lower_bound(sb, sb + N.r, g) - sb);
          cnt[N.poff + p]++;
        }
    }
    // pull_ptr[N.poff + p] = start of position p's list; per node c + r + 1 entries
    int64_t tot = 0;
    for (int i = 0; i < nn; ++i) {
      const SolveNode& N = S.nodes[i];
      for (int64_t p = 0; p <= N.c + N.r; ++p) {
        const int64_t k = N.poff + p;
        const int64_t cc = p < N.c + N.r ? cnt[k] : 0;
        S.pull_ptr[k] = static_cast<int32_t>(tot);
        tot += cc;
      }
    }
    if (tot > INT32_MAX) {
      err = "pull list too large";
      return ERR_OUT_OF_MEMORY;
    }
    S.pull_idx.assign(tot, 0);
    std::vector<int64_t> fill(po);
    for (int64_t k = 0; k < po; ++k) fill[k] = S.pull_ptr[k];
    for (int i = 0; i < nn; ++i) {
      const SolveNode& N = S.nodes[i];
      const int32_t* sb = strct[i].data();
      for (int32_t ch : S.children[i]) {
        const SolveNode& C = S.nodes[ch];
        for (int32_t q = 0; q < C.r; ++q) {
          const int32_t g = strct[ch][q];
          const int64_t p = g < N.first + N.c ? g - N.first
                                              : N.c + (std::lower_bound(sb, sb + N.r, g) - sb);
          S.pull_idx[fill[N.poff + p]++] = static_cast<int32_t>(C.uoff + q);
        }
      }
    }
  }
  S.level_nodes.assign(nlev, {});
  for (int i = 0; i < nn; ++i) S.level_nodes[S.nodes[i].level].push_back(i);
  S.t_symbolic = now() - t0;
  }  // ordering and symbolic

  // ---- numeric multifrontal factorisation --------------------------------------
  t0 = now();
  S.panel_f.resize(pf);  // not zero-filled: each host node writes its whole region
  std::vector<std::vector<double>> upd(nn);
  std::vector<int> fail(nn, 0);
  auto factor_node = [&](int i) {
    for (int32_t ch : S.children[i])
      if (fail[ch]) {
        fail[i] = 1;
        return;
      }
    const SolveNode& N = S.nodes[i];
    const int c = N.c, r = N.r, nf = c + r;
    const int32_t* sb = strct[i].data();
    auto pos = [&](int32_t g) -> int64_t {
      return g < N.first + c ? g - N.first : c + (std::lower_bound(sb, sb + r, g) - sb);
    };
    std::vector<double> F(static_cast<size_t>(nf) * nf, 0.0);
    for (int j = 0; j < c; ++j) {
      const int32_t gv = N.first + j;
      const int32_t v = S.vnew2old[gv];
      for (int64_t k = Lptr[v]; k < Lptr[v + 1]; ++k) {
        const int32_t gu = S.vold2new[Lcol[k]];
        if (gu >= S.nF || gu < gv) continue;
        F[pos(gu) + static_cast<int64_t>(j) * nf] += Lval[k];
      }
    }
    for (int32_t ch : S.children[i]) {
      const int rc = S.nodes[ch].r;
      std::vector<int64_t> rel(rc);
      for (int q = 0; q < rc; ++q) rel[q] = pos(strct[ch][q]);
      const std::vector<double>& U = upd[ch];
      for (int jj = 0; jj < rc; ++jj)
        for (int ii = jj; ii < rc; ++ii)
          F[rel[ii] + rel[jj] * nf] += U[ii + static_cast<size_t>(jj) * rc];
      std::vector<double>().swap(upd[ch]);
    }
    if (dense::potrf(c, F.data(), nf)) {
      fail[i] = 1;
      return;
    }
    if (r > 0) dense::trsm_rlt(r, c, F.data(), nf, F.data() + c, nf);
    std::vector<double> Linv(static_cast<size_t>(c) * c);
    dense::trtri(c, F.data(), nf, Linv.data(), c);
    std::vector<double> M(static_cast<size_t>(r) * c);
    if (r > 0) {
      dense::syrk_sub(r, c, F.data() + c, nf, F.data() + c + static_cast<int64_t>(c) * nf, nf);
      upd[i].assign(static_cast<size_t>(r) * r, 0.0);
      for (int jj = 0; jj < r; ++jj)
        for (int ii = jj; ii < r; ++ii)
          upd[i][ii + static_cast<size_t>(jj) * r] = F[(c + ii) + static_cast<int64_t>(c + jj) * nf];
      dense::gemm_nn(r, c, c, 1.0, F.data() + c, nf, Linv.data(), c, 0.0, M.data(), r);
    }
    double* Pf = S.panel_f.data() + N.pf;
    for (int j = 0; j < c; ++j) {
      for (int p = 0; p < c; ++p) Pf[p + static_cast<int64_t>(j) * nf] = p >= j ? Linv[p + static_cast<size_t>(j) * c] : 0.0;
      for (int q = 0; q < r; ++q) Pf[c + q + static_cast<int64_t>(j) * nf] = -M[q + static_cast<size_t>(j) * r];
    }
  };
  // subtree sizes (work) to split into parallel subtrees and a sequential top
  std::vector<double> work(nn, 0);
  for (int i = 0; i < nn; ++i) {
    const double c = S.nodes[i].c, r = S.nodes[i].r;
    work[i] = c * c * c + 2 * r * c * c + r * r * c;
    for (int32_t ch : S.children[i]) work[i] += work[ch];
  }
  double total = 0;
  std::vector<int32_t> parent(nn, -1);
  for (int i = 0; i < nn; ++i)
    for (int32_t ch : S.children[i]) parent[ch] = i;
  for (int i = 0; i < nn; ++i)
    if (parent[i] < 0) total += work[i];
  const int nth = std::max(1, omp_get_max_threads());
  // with the top fronts on the device a finer cut balances the host part better
  const bool dev_top = in.device_top && !in.selfcheck;
  const double cut = total / ((dev_top ? 64.0 : 8.0) * nth);
  // a node is in the parallel part if its subtree work is below the cut; the
  // parallel subtrees are the maximal such subtrees
  std::vector<uint8_t> small(nn, 0);
  for (int i = 0; i < nn; ++i) small[i] = work[i] <= cut;
  std::vector<int32_t> subroots, top;
  for (int i = 0; i < nn; ++i) {
    if (small[i] && (parent[i] < 0 || !small[parent[i]])) subroots.push_back(i);
    if (!small[i]) top.push_back(i);
  }
  std::sort(subroots.begin(), subroots.end(), [&](int a, int b) { return work[a] > work[b]; });
#pragma omp parallel for schedule(dynamic, 1)
  for (size_t k = 0; k < subroots.size(); ++k) {
    const int root = subroots[k];
    // postorder of a subtree is a contiguous index range ending at its root
    int lo = root;
    while (!S.children[lo].empty()) lo = *std::min_element(S.children[lo].begin(), S.children[lo].end());
    for (int i = lo; i <= root; ++i) factor_node(i);
  }
  if (dev_top) {
    // gather what the device needs to assemble each front; no numeric work
    for (int32_t i : top) {
      const SolveNode& N = S.nodes[i];
      const int c = N.c, nf = c + N.r;
      const int32_t* sb = strct[i].data();
      auto pos = [&](int32_t g) -> int64_t {
        return g < N.first + c ? g - N.first : c + (std::lower_bound(sb, sb + N.r, g) - sb);
      };
      TopNode T;
      T.node = i;
      for (int j = 0; j < c; ++j) {
        const int32_t gv = N.first + j;
        const int32_t v = S.vnew2old[gv];
        for (int64_t k = Lptr[v]; k < Lptr[v + 1]; ++k) {
          const int32_t gu = S.vold2new[Lcol[k]];
          if (gu >= S.nF || gu < gv) continue;
          T.lidx.push_back(pos(gu) + static_cast<int64_t>(j) * nf);
          T.lval.push_back(Lval[k]);
        }
      }
      for (int32_t ch : S.children[i]) {
        TopChild K;
        K.node = ch;
        K.host = small[ch] != 0;
        K.rel.resize(S.nodes[ch].r);
        for (int q = 0; q < S.nodes[ch].r; ++q) K.rel[q] = static_cast<int32_t>(pos(strct[ch][q]));
        if (K.host) K.upd = std::move(upd[ch]);
        T.kids.push_back(std::move(K));
      }
      S.top.push_back(std::move(T));
    }
  } else {
    for (int32_t i : top) factor_node(i);  // postorder: children before parents
  }
  for (int i = 0; i < nn; ++i)
    if (fail[i]) {
      err = "the W-step matrix is not positive definite (check the pins)";
      return ERR_SINGULAR_SYSTEM;
    }
  S.t_numeric = now() - t0;

  // ---- element order and device tables -------------------------------------------
  if (!in.structure) {
  std::vector<int32_t> key(m);
  for (int64_t e = 0; e < m; ++e) {
    int32_t k = INT32_MAX;
    for (int c = 0; c < nc; ++c) k = std::min(k, S.vold2new[in.T[e * nc + c]]);
    key[e] = k;
  }
  S.enew2old.resize(m);
  std::iota(S.enew2old.begin(), S.enew2old.end(), 0);
  if (in.elem_energy) {
    std::stable_sort(S.enew2old.begin(), S.enew2old.end(), [&](int32_t a, int32_t b) {
      return in.elem_energy[a] != in.elem_energy[b] ? in.elem_energy[a] < in.elem_energy[b] : key[a] < key[b];
    });
    S.m_energy0 = 0;
    for (int64_t e = 0; e < m; ++e) S.m_energy0 += in.elem_energy[e] == 0;
  } else {
    std::stable_sort(S.enew2old.begin(), S.enew2old.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    S.m_energy0 = m;
  }
  S.B.resize(static_cast<size_t>(m) * d * d);
  S.w.resize(m);
  S.T.resize(static_cast<size_t>(m) * nc);
  for (int64_t e = 0; e < m; ++e) {
    const int64_t o = S.enew2old[e];
    std::memcpy(S.B.data() + e * d * d, B0.data() + o * d * d, sizeof(double) * d * d);
    S.w[e] = w0[o];
    for (int c = 0; c < nc; ++c) S.T[e * nc + c] = S.vold2new[in.T[o * nc + c]];
  }
  S.dt_ptr.assign(S.nF + 1, 0);
  for (int64_t e = 0; e < m; ++e)
    for (int c = 0; c < nc; ++c)
      if (S.T[e * nc + c] < S.nF) S.dt_ptr[S.T[e * nc + c] + 1]++;
  for (int64_t v = 0; v < S.nF; ++v) S.dt_ptr[v + 1] += S.dt_ptr[v];
  S.dt_idx.assign(S.dt_ptr[S.nF], 0);
  {
    std::vector<int32_t> fill(S.dt_ptr.begin(), S.dt_ptr.end() - 1);
    for (int64_t e = 0; e < m; ++e)
      for (int c = 0; c < nc; ++c) {
        const int32_t v = S.T[e * nc + c];
        if (v < S.nF) S.dt_idx[fill[v]++] = static_cast<int32_t>(e * nc + c);
      }
  }
  // constraint rows in the device numbering, and their transpose over the
  // free rows they touch
  if (in.n_con > 0) {
    const int64_t nnz = in.con_ptr[in.n_con];
    S.con_ptr.assign(in.con_ptr, in.con_ptr + in.n_con + 1);
    S.con_val.assign(in.con_val, in.con_val + nnz);
    S.con_col.resize(nnz);
    std::vector<std::tuple<int32_t, int32_t, double>> ent;
    for (int64_t a = 0; a < in.n_con; ++a)
      for (int64_t q = in.con_ptr[a]; q < in.con_ptr[a + 1]; ++q) {
        const int32_t j = S.vold2new[in.con_col[q]];
        S.con_col[q] = j;
        if (j < S.nF) ent.emplace_back(j, static_cast<int32_t>(a), in.con_val[q]);
      }
    std::sort(ent.begin(), ent.end());
    S.cont_ptr.push_back(0);
    for (size_t i = 0; i < ent.size(); ++i) {
      if (i == 0 || std::get<0>(ent[i]) != std::get<0>(ent[i - 1])) {
        if (i > 0) S.cont_ptr.push_back(static_cast<int32_t>(i));
        S.cont_rows.push_back(std::get<0>(ent[i]));
      }
      S.cont_con.push_back(std::get<1>(ent[i]));
      S.cont_val.push_back(std::get<2>(ent[i]));
    }
    S.cont_ptr.push_back(static_cast<int32_t>(ent.size()));
  }
  if (in.selfcheck && S.nF > 0) {
    // solve L_FF x = b with the panels exactly as the device does (forward
    // pass bottom-up with extend-add pulls, backward pass top-down) and report
    // the relative residual
    const int64_t nF = S.nF;
    std::vector<double> b(nF), y(nF), x(nF), ub(S.ubuf_rows, 0.0);
    for (int64_t j = 0; j < nF; ++j) b[j] = std::sin(0.37 * j + 1.0) + 0.5 * std::cos(1.3 * j);
    for (int i = 0; i < nn; ++i) {
      const SolveNode& N = S.nodes[i];
      const int c = N.c, r = N.r, nf = c + r;
      std::vector<double> v(nf, 0.0);
      for (int p = 0; p < nf; ++p) {
        double a = p < c ? b[N.first + p] : 0.0;
        for (int32_t k = S.pull_ptr[N.poff + p]; k < S.pull_ptr[N.poff + p + 1]; ++k) a += ub[S.pull_idx[k]];
        v[p] = a;
      }
      const double* Pf = S.panel_f.data() + N.pf;
      for (int row = 0; row < nf; ++row) {
        double a = row < c ? 0.0 : v[row];
        for (int j = 0; j < c; ++j) a += Pf[row + static_cast<int64_t>(j) * nf] * v[j];
        if (row < c) y[N.first + row] = a;
        else ub[N.uoff + row - c] = a;
      }
    }
    for (int i = nn - 1; i >= 0; --i) {
      const SolveNode& N = S.nodes[i];
      const int c = N.c, r = N.r, nf = c + r;
      const double* Pf = S.panel_f.data() + N.pf;
      for (int j = 0; j < c; ++j) {
        double a = 0.0;
        for (int p = 0; p < nf; ++p)
          a += Pf[p + static_cast<int64_t>(j) * nf] * (p < c ? y[N.first + p] : x[S.struct_idx[N.soff + p - c]]);
        x[N.first + j] = a;
      }
    }
    double rn = 0, bn = 0;
    for (int64_t j = 0; j < nF; ++j) {
      const int32_t v = S.vnew2old[j];
      double a = -b[j];
      for (int64_t k = Lptr[v]; k < Lptr[v + 1]; ++k) {
        const int32_t u = S.vold2new[Lcol[k]];
        if (u < nF) a += Lval[k] * x[u];
      }
      rn += a * a;
      bn += b[j] * b[j];
    }
    S.selfcheck_residual = std::sqrt(rn / bn);
  }
  S.av_ptr.assign(n + 1, 0);
  for (int64_t e = 0; e < m; ++e)
    for (int c = 0; c < nc; ++c) S.av_ptr[S.T[e * nc + c] + 1]++;
  for (int64_t v = 0; v < n; ++v) S.av_ptr[v + 1] += S.av_ptr[v];
  S.av_idx.assign(S.av_ptr[n], 0);
  {
    std::vector<int32_t> fill(S.av_ptr.begin(), S.av_ptr.end() - 1);
    for (int64_t e = 0; e < m; ++e)
      for (int c = 0; c < nc; ++c) S.av_idx[fill[S.T[e * nc + c]]++] = static_cast<int32_t>(e * nc + c);
  }
  }  // element order and device tables
  S.lcf_ptr.assign(S.nC + 1, 0);
  for (int64_t i = 0; i < S.nC; ++i) {
    const int32_t v = S.vnew2old[S.nF + i];
    for (int64_t k = Lptr[v]; k < Lptr[v + 1]; ++k) {
      const int32_t u = S.vold2new[Lcol[k]];
      if (u < S.nF) {
        S.lcf_col.push_back(u);
        S.lcf_val.push_back(Lval[k]);
      }
    }
    S.lcf_ptr[i + 1] = static_cast<int32_t>(S.lcf_col.size());
  }
  S.pin_ptr.assign(S.nF + 1, 0);
  for (int64_t j = 0; j < S.nF; ++j) {
    const int32_t v = S.vnew2old[j];
    for (int64_t k = Lptr[v]; k < Lptr[v + 1]; ++k) {
      const int32_t u = S.vold2new[Lcol[k]];
      if (u >= S.nF) {
        S.pin_col.push_back(static_cast<int32_t>(u - S.nF));
        S.pin_val.push_back(Lval[k]);
      }
    }
    S.pin_ptr[j + 1] = static_cast<int32_t>(S.pin_col.size());
  }
  return OK;
}

int64_t device_panel_offsets(const Setup& S, std::vector<int64_t>& off) {
  const size_t nn = S.nodes.size();
  off.assign(nn, 0);
  int64_t tot = 0;
  for (size_t i = 0; i < nn; ++i) {
    const int64_t c = S.nodes[i].c, nf = S.nodes[i].c + S.nodes[i].r;
    off[i] = tot;
    tot += nf * c;
    tot = (tot + 1) & ~int64_t(1);
  }
  return tot;
}

int64_t build_host_panels(const Setup& S, const std::vector<int64_t>& off, int64_t tot, std::vector<int64_t>& coff,
                          std::unique_ptr<double[]>& prow, std::unique_ptr<double[]>& pcol) {
  const size_t nn = S.nodes.size();
  std::vector<uint8_t> skip(nn, 0);
  for (const TopNode& T : S.top) skip[T.node] = 1;
  coff.assign(nn, -1);
  int64_t len = 0;
  for (size_t i = 0; i < nn; ++i) {
    if (skip[i]) continue;
    coff[i] = len;
    len += (i + 1 < nn ? off[i + 1] : tot) - off[i];
  }
  prow.reset(new double[std::max<int64_t>(len, 1)]);
  pcol.reset(new double[std::max<int64_t>(len, 1)]);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < static_cast<int64_t>(nn); ++i) {
    if (skip[i]) continue;
    const int64_t c = S.nodes[i].c, nf = S.nodes[i].c + S.nodes[i].r;
    const int64_t seg = (i + 1 < static_cast<int64_t>(nn) ? off[i + 1] : tot) - off[i];
    double* R = prow.get() + coff[i];
    double* Cc = pcol.get() + coff[i];
    std::fill(R, R + seg, 0.0);
    std::fill(Cc, Cc + seg, 0.0);
    const double* src = S.panel_f.data() + S.nodes[i].pf;  // column-major, ld = nf
    for (int64_t j = 0; j < c; ++j)
      for (int64_t p = 0; p < nf; ++p) {
        const double v = src[p + j * nf];
        R[panel_tile_index(j, p, c, nf)] = v;
        Cc[panel_tile_index(p, j, nf, c)] = v;
      }
  }
  return len;
}

}  // namespace ffd
