// Device factorisation of the top fronts for a refactorisation after a
// rescaling event.  The host factorises the subtrees below the top as at set-up
// and hands over, per top node, the entries of L in its columns and its
// children's update matrices (Setup::top).  The device assembles each front
// and runs the dense steps: Cholesky of the pivot block, the triangular solve
// for the off-diagonal block, the Schur update passed to the parent, and the
// inverse of the pivot factor.  These are rocSOLVER / rocBLAS calls, loaded
// with dlopen on first use.  It then writes the node's panels [Linv; -M] into
// both device copies.  Part of the single translation unit capi.hip.
#pragma once

#include <dlfcn.h>

#include "schedule.hpp"

namespace {

struct DenseLib {
  bool ok = false;
  rocblas_status (*create_handle)(rocblas_handle*) = nullptr;
  rocblas_status (*destroy_handle)(rocblas_handle) = nullptr;
  rocblas_status (*set_stream)(rocblas_handle, hipStream_t) = nullptr;
  rocblas_status (*dtrsm)(rocblas_handle, rocblas_side, rocblas_fill, rocblas_operation, rocblas_diagonal, rocblas_int,
                          rocblas_int, const double*, const double*, rocblas_int, double*, rocblas_int) = nullptr;
  rocblas_status (*dsyrk)(rocblas_handle, rocblas_fill, rocblas_operation, rocblas_int, rocblas_int, const double*,
                          const double*, rocblas_int, const double*, double*, rocblas_int) = nullptr;
  rocblas_status (*dtrmm)(rocblas_handle, rocblas_side, rocblas_fill, rocblas_operation, rocblas_diagonal, rocblas_int,
                          rocblas_int, const double*, const double*, rocblas_int, const double*, rocblas_int, double*,
                          rocblas_int) = nullptr;
  rocblas_status (*dpotrf)(rocblas_handle, rocblas_fill, rocblas_int, double*, rocblas_int, rocblas_int*) = nullptr;
  rocblas_status (*dtrtri)(rocblas_handle, rocblas_fill, rocblas_diagonal, rocblas_int, double*, rocblas_int,
                           rocblas_int*) = nullptr;
};

// the libraries the process already has (PyTorch loads them) or the system's
const DenseLib& dense_lib() {
  static const DenseLib lib = [] {
    DenseLib L;
    void* b = dlopen("librocblas.so.5", RTLD_NOW | RTLD_GLOBAL);
    void* v = b ? dlopen("librocsolver.so.0", RTLD_NOW | RTLD_GLOBAL) : nullptr;
    if (!b || !v) return L;
    L.create_handle = reinterpret_cast<decltype(L.create_handle)>(dlsym(b, "rocblas_create_handle"));
    L.destroy_handle = reinterpret_cast<decltype(L.destroy_handle)>(dlsym(b, "rocblas_destroy_handle"));
    L.set_stream = reinterpret_cast<decltype(L.set_stream)>(dlsym(b, "rocblas_set_stream"));
    L.dtrsm = reinterpret_cast<decltype(L.dtrsm)>(dlsym(b, "rocblas_dtrsm"));
    L.dsyrk = reinterpret_cast<decltype(L.dsyrk)>(dlsym(b, "rocblas_dsyrk"));
    L.dtrmm = reinterpret_cast<decltype(L.dtrmm)>(dlsym(b, "rocblas_dtrmm"));
    L.dpotrf = reinterpret_cast<decltype(L.dpotrf)>(dlsym(v, "rocsolver_dpotrf"));
    L.dtrtri = reinterpret_cast<decltype(L.dtrtri)>(dlsym(v, "rocsolver_dtrtri"));
    L.ok = L.create_handle && L.destroy_handle && L.set_stream && L.dtrsm && L.dsyrk && L.dtrmm && L.dpotrf &&
           L.dtrtri;
    return L;
  }();
  return lib;
}

// device buffers of one refactorisation, freed when it ends
struct DevScratch {
  std::vector<void*> p;
  template <typename T_>
  hipError_t get(T_** out, size_t count) {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(out), std::max<size_t>(count, 1) * sizeof(T_));
    if (e == hipSuccess) p.push_back(*out);
    return e;
  }
  ~DevScratch() {
    for (void* q : p) (void)hipFree(q);
  }
};

// The host-built panels (every node but the top fronts) into both device
// copies, one copy per run of consecutive nodes.  Synchronous.
ffd_status upload_host_panels(ffd_ctx* h, const Setup& S, const std::vector<int64_t>& off, int64_t tot,
                              hipStream_t s) {
  std::vector<int64_t> coff;
  std::unique_ptr<double[]> prow, pcol;
  build_host_panels(S, off, tot, coff, prow, pcol);
  const size_t nn = S.nodes.size();
  for (size_t i = 0; i < nn;) {
    if (coff[i] < 0) {
      ++i;
      continue;
    }
    size_t j = i;
    while (j + 1 < nn && coff[j + 1] >= 0) ++j;
    const int64_t end = j + 1 < nn ? off[j + 1] : tot;
    const size_t bytes = static_cast<size_t>(end - off[i]) * sizeof(double);
    HIP_TRY(hipMemcpyAsync(h->Prow + off[i], prow.get() + coff[i], bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(h->Pcol + off[i], pcol.get() + coff[i], bytes, hipMemcpyHostToDevice, s));
    i = j + 1;
  }
  HIP_TRY(hipStreamSynchronize(s));  // the host copies are freed on return
  return FFD_OK;
}

#define BLAS_TRY(expr)                                                                   \
  do {                                                                                   \
    if ((expr) != rocblas_status_success) return fail(FFD_ERR_DEVICE, "dense library call failed: " #expr); \
  } while (0)

// Factorises the fronts of S.top on the device in postorder and writes their
// panels (the host wrote every other node's panels).  Synchronous.
ffd_status device_factor_top(ffd_ctx* h, const Setup& S, hipStream_t s) {
  if (S.top.empty()) return FFD_OK;
  const DenseLib& L = dense_lib();
  if (!L.ok) return fail(FFD_ERR_STATE, "rocBLAS / rocSOLVER not available");
  if (!h->blas) {
    BLAS_TRY(L.create_handle(&h->blas));
    h->blas_destroy = L.destroy_handle;
  }
  BLAS_TRY(L.set_stream(h->blas, s));
  const size_t nn = S.nodes.size();
  std::vector<int64_t> uoff(nn, -1);
  int64_t maxF = 1, maxC2 = 1, maxRC = 1, maxL = 1, maxRel = 1, maxUh = 1, totU = 1;
  for (const TopNode& T : S.top) {
    const int64_t c = S.nodes[T.node].c, r = S.nodes[T.node].r, nf = c + r;
    maxF = std::max(maxF, nf * nf);
    maxC2 = std::max(maxC2, c * c);
    maxRC = std::max(maxRC, r * c);
    maxL = std::max<int64_t>(maxL, static_cast<int64_t>(T.lidx.size()));
    if (r > 0) {
      uoff[T.node] = totU;
      totU += r * r;
    }
    for (const TopChild& K : T.kids) {
      const int64_t rc = static_cast<int64_t>(K.rel.size());
      maxRel = std::max(maxRel, rc);
      if (K.host) maxUh = std::max(maxUh, rc * rc);
    }
  }
  DevScratch w;
  double *F = nullptr, *Li = nullptr, *M = nullptr, *Uh = nullptr, *val = nullptr, *U = nullptr;
  int64_t* idx = nullptr;
  int32_t *rel = nullptr, *info = nullptr;
  const size_t ntop = S.top.size();
  HIP_TRY(w.get(&F, static_cast<size_t>(maxF)));
  HIP_TRY(w.get(&Li, static_cast<size_t>(maxC2)));
  HIP_TRY(w.get(&M, static_cast<size_t>(maxRC)));
  HIP_TRY(w.get(&Uh, static_cast<size_t>(maxUh)));
  HIP_TRY(w.get(&val, static_cast<size_t>(maxL)));
  HIP_TRY(w.get(&idx, static_cast<size_t>(maxL)));
  HIP_TRY(w.get(&rel, static_cast<size_t>(maxRel)));
  HIP_TRY(w.get(&U, static_cast<size_t>(totU)));
  HIP_TRY(w.get(&info, 2 * ntop));
  HIP_TRY(hipMemsetAsync(info, 0, 2 * ntop * sizeof(int32_t), s));
  const double one = 1.0, minus_one = -1.0;
  auto blocks = [](int64_t n) { return dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)); };
  for (size_t t = 0; t < ntop; ++t) {
    const TopNode& T = S.top[t];
    const SolveNode& N = S.nodes[T.node];
    const int64_t c = N.c, r = N.r, nf = c + r;
    HIP_TRY(hipMemsetAsync(F, 0, static_cast<size_t>(nf * nf) * sizeof(double), s));
    const int64_t nl = static_cast<int64_t>(T.lidx.size());
    if (nl > 0) {
      HIP_TRY(hipMemcpyAsync(idx, T.lidx.data(), nl * sizeof(int64_t), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(val, T.lval.data(), nl * sizeof(double), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_front_scatter, blocks(nl), dim3(kBlock), 0, s, nl, idx, val, F);
    }
    for (const TopChild& K : T.kids) {
      const int64_t rc = static_cast<int64_t>(K.rel.size());
      if (rc == 0) continue;
      HIP_TRY(hipMemcpyAsync(rel, K.rel.data(), rc * sizeof(int32_t), hipMemcpyHostToDevice, s));
      const double* src = U + uoff[K.node];
      if (K.host) {
        HIP_TRY(hipMemcpyAsync(Uh, K.upd.data(), static_cast<size_t>(rc * rc) * sizeof(double), hipMemcpyHostToDevice,
                               s));
        src = Uh;
      }
      hipLaunchKernelGGL(k_front_extend, blocks(rc * rc), dim3(kBlock), 0, s, rc, rel, src, rc, F, nf);
    }
    HIP_TRY(hipGetLastError());
    BLAS_TRY(L.dpotrf(h->blas, rocblas_fill_lower, static_cast<rocblas_int>(c), F, static_cast<rocblas_int>(nf),
                      info + 2 * t));
    if (r > 0)
      BLAS_TRY(L.dtrsm(h->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                       rocblas_diagonal_non_unit, static_cast<rocblas_int>(r), static_cast<rocblas_int>(c), &one, F,
                       static_cast<rocblas_int>(nf), F + c, static_cast<rocblas_int>(nf)));
    hipLaunchKernelGGL(k_lower_copy, blocks(c * c), dim3(kBlock), 0, s, c, F, nf, Li, c);
    BLAS_TRY(L.dtrtri(h->blas, rocblas_fill_lower, rocblas_diagonal_non_unit, static_cast<rocblas_int>(c), Li,
                      static_cast<rocblas_int>(c), info + 2 * t + 1));
    if (r > 0) {
      double* Frr = F + c + c * nf;
      BLAS_TRY(L.dsyrk(h->blas, rocblas_fill_lower, rocblas_operation_none, static_cast<rocblas_int>(r),
                       static_cast<rocblas_int>(c), &minus_one, F + c, static_cast<rocblas_int>(nf), &one, Frr,
                       static_cast<rocblas_int>(nf)));
      hipLaunchKernelGGL(k_lower_copy, blocks(r * r), dim3(kBlock), 0, s, r, Frr, nf, U + uoff[T.node], r);
      BLAS_TRY(L.dtrmm(h->blas, rocblas_side_right, rocblas_fill_lower, rocblas_operation_none,
                       rocblas_diagonal_non_unit, static_cast<rocblas_int>(r), static_cast<rocblas_int>(c), &one, Li,
                       static_cast<rocblas_int>(c), F + c, static_cast<rocblas_int>(nf), M,
                       static_cast<rocblas_int>(r)));
    }
    hipLaunchKernelGGL(k_front_panels, blocks(nf * c), dim3(kBlock), 0, s, c, r, Li, M, h->hpoff[T.node], h->Pcol,
                       h->Prow);
    HIP_TRY(hipGetLastError());
  }
  std::vector<int32_t> hinfo(2 * ntop);
  HIP_TRY(hipMemcpyAsync(hinfo.data(), info, hinfo.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int32_t v : hinfo)
    if (v != 0) return fail(FFD_ERR_SINGULAR_SYSTEM, "the W-step matrix is not positive definite (device refactorisation)");
  return FFD_OK;
}

#undef BLAS_TRY

}  // namespace
