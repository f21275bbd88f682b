// C ABI of the flip-free ADMM solver (include/ffd.h): handle, device memory,
// and the launch sequence of one iteration of Algorithm 1:
//   K2 W-step right-hand side -> K4 forward solve levels -> K5 backward solve
//   levels -> K3 fused U/P/Lambda step -> finalize (history record).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ffd.h"
#include "host/setup.hpp"
#include "kernels.hpp"

using namespace ffd;

namespace {

thread_local std::string g_last_error;

ffd_status fail(ffd_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? FFD_ERR_OUT_OF_MEMORY : FFD_ERR_DEVICE,     \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                     \
  } while (0)

constexpr int kRT = 64;  // output rows per solve task
constexpr int64_t kHistCap0 = 1 << 14;

inline unsigned nblk(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

}  // namespace

struct ffd_ctx {
  int d = 0, din = 0, prec = 32, energy = 0, h_mode = 0;
  double rho = 0;
  int64_t n = 0, m = 0, nF = 0, nC = 0;
  bool pins_given = false, auto_pinned = false, initialized = false;
  int64_t k = 0;          // completed iterations
  int cur = 0;            // index of the buffer holding W^k
  int dev = 0;
  hipStream_t last_stream = nullptr;
  ffd_info info{};
  // host copies
  std::vector<int32_t> vnew2old;
  std::vector<int32_t> level_fwd_off, level_bwd_off;  // task offsets per level (size nlev + 1)
  // device buffers
  int32_t *T = nullptr, *vnew2old_d = nullptr, *enew2old_d = nullptr;
  double* B64 = nullptr;
  void *B = nullptr, *w = nullptr;
  double *x[2] = {nullptr, nullptr}, *xC = nullptr;
  void *U = nullptr, *P = nullptr, *L = nullptr, *gn = nullptr, *g = nullptr;
  double *b = nullptr, *y = nullptr, *ub = nullptr, *partials = nullptr, *hist = nullptr;
  int64_t hist_cap = 0;
  int32_t *dt_ptr = nullptr, *dt_idx = nullptr, *pin_ptr = nullptr, *pin_col = nullptr;
  double* pin_val = nullptr;
  NodeDev* nodes = nullptr;
  double *Pf = nullptr, *Pb = nullptr;
  int32_t *sidx = nullptr, *pull_ptr = nullptr, *pull_idx = nullptr;
  int2 *tasks_fwd = nullptr, *tasks_bwd = nullptr;
  int64_t device_bytes = 0;
  std::vector<void*> allocs;
  std::vector<hipEvent_t> events;

  template <typename T_>
  hipError_t alloc(T_** p, size_t count) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T_);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
    if (e == hipSuccess) {
      allocs.push_back(*p);
      device_bytes += bytes;
    }
    return e;
  }
  size_t rsize() const { return prec == 32 ? 4 : 8; }
  ~ffd_ctx() {
    for (hipEvent_t ev : events) (void)hipEventDestroy(ev);
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

template <typename T_>
hipError_t upload(ffd_ctx* h, T_** dst, const std::vector<T_>& src) {
  hipError_t e = h->alloc(dst, src.size());
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T_), hipMemcpyHostToDevice);
  return e;
}

// element arrays as SoA [entry][m] in the arithmetic type
template <typename R>
std::vector<R> soa(const std::vector<double>& aos, int64_t m, int per) {
  std::vector<R> out(static_cast<size_t>(m) * per);
  for (int64_t e = 0; e < m; ++e)
    for (int i = 0; i < per; ++i) out[static_cast<size_t>(i) * m + e] = static_cast<R>(aos[e * per + i]);
  return out;
}

// --------------------------------------------------------------------------
// launch helpers (dispatch on d, precision, energy)
// --------------------------------------------------------------------------

template <int D, typename R, int E>
void launch_init(ffd_ctx* h, hipStream_t s) {
  hipLaunchKernelGGL((k_init<D, R, E>), dim3(nblk(h->m)), dim3(kBlock), 0, s, h->m, h->T, h->B64,
                     static_cast<const R*>(h->B), static_cast<const R*>(h->w), static_cast<R>(h->rho), h->x[h->cur],
                     static_cast<R*>(h->U), static_cast<R*>(h->P), static_cast<R*>(h->L), static_cast<R*>(h->gn),
                     static_cast<R*>(h->g));
}

template <int D, typename R, int E>
void launch_prepare(ffd_ctx* h, hipStream_t s) {
  hipLaunchKernelGGL((k_prepare<D, R, E>), dim3(nblk(h->m)), dim3(kBlock), 0, s, h->m, static_cast<const R*>(h->B),
                     static_cast<const R*>(h->w), static_cast<R>(h->rho), static_cast<const R*>(h->U),
                     static_cast<const R*>(h->P), static_cast<const R*>(h->L), static_cast<R*>(h->gn),
                     static_cast<R*>(h->g));
}

template <int D, typename R, int E>
void launch_local(ffd_ctx* h, const double* xnew, const double* xold, hipStream_t s) {
  hipLaunchKernelGGL((k_local<D, R, E>), dim3(nblk(h->m)), dim3(kBlock), 0, s, h->m, h->T,
                     static_cast<const R*>(h->B), static_cast<const R*>(h->w), static_cast<R>(h->rho), h->h_mode, xnew,
                     xold, static_cast<R*>(h->U), static_cast<R*>(h->P), static_cast<R*>(h->L), static_cast<R*>(h->gn),
                     static_cast<R*>(h->g), h->partials);
}

template <int D, typename R>
void launch_wrhs(ffd_ctx* h, double* xnew, hipStream_t s) {
  hipLaunchKernelGGL((k_wrhs<D, R>), dim3(nblk(h->n)), dim3(kBlock), 0, s, h->nF, h->n, h->dt_ptr, h->dt_idx,
                     static_cast<const R*>(h->g), h->pin_ptr, h->pin_col, h->pin_val, h->xC, h->b, xnew);
}

template <int D>
void launch_solve_fwd(ffd_ctx* h, const double* b, hipStream_t s) {
  const int nlev = static_cast<int>(h->level_fwd_off.size()) - 1;
  for (int l = 0; l < nlev; ++l) {
    const int nt = h->level_fwd_off[l + 1] - h->level_fwd_off[l];
    if (nt > 0)
      hipLaunchKernelGGL((k_solve_fwd<D, kRT>), dim3(nt), dim3(kBlock), 0, s, h->tasks_fwd + h->level_fwd_off[l],
                         h->nodes, h->Pf, h->pull_ptr, h->pull_idx, b, h->y, h->ub);
  }
}

template <int D>
void launch_solve_bwd(ffd_ctx* h, double* x, hipStream_t s) {
  const int nlev = static_cast<int>(h->level_fwd_off.size()) - 1;
  for (int l = nlev - 1; l >= 0; --l) {
    const int nt = h->level_bwd_off[l + 1] - h->level_bwd_off[l];
    if (nt > 0)
      hipLaunchKernelGGL((k_solve_bwd<D, kRT>), dim3(nt), dim3(kBlock), 0, s, h->tasks_bwd + h->level_bwd_off[l],
                         h->nodes, h->Pb, h->sidx, h->y, x);
  }
}

template <int D>
void launch_solve(ffd_ctx* h, const double* b, double* x, hipStream_t s) {
  launch_solve_fwd<D>(h, b, s);
  launch_solve_bwd<D>(h, x, s);
}

void do_init(ffd_ctx* h, hipStream_t s) {
  const int key = h->d * 100 + h->prec + h->energy;
#define CASE(D, P, E, R) \
  case D * 100 + P + E: launch_init<D, R, E>(h, s); break;
  switch (key) {
    CASE(2, 32, 0, float) CASE(2, 32, 1, float) CASE(2, 64, 0, double) CASE(2, 64, 1, double)
    CASE(3, 32, 0, float) CASE(3, 32, 1, float) CASE(3, 64, 0, double) CASE(3, 64, 1, double)
  }
#undef CASE
}

void do_prepare(ffd_ctx* h, hipStream_t s) {
  const int key = h->d * 100 + h->prec + h->energy;
#define CASE(D, P, E, R) \
  case D * 100 + P + E: launch_prepare<D, R, E>(h, s); break;
  switch (key) {
    CASE(2, 32, 0, float) CASE(2, 32, 1, float) CASE(2, 64, 0, double) CASE(2, 64, 1, double)
    CASE(3, 32, 0, float) CASE(3, 32, 1, float) CASE(3, 64, 0, double) CASE(3, 64, 1, double)
  }
#undef CASE
}

void do_local(ffd_ctx* h, const double* xnew, const double* xold, hipStream_t s) {
  const int key = h->d * 100 + h->prec + h->energy;
#define CASE(D, P, E, R) \
  case D * 100 + P + E: launch_local<D, R, E>(h, xnew, xold, s); break;
  switch (key) {
    CASE(2, 32, 0, float) CASE(2, 32, 1, float) CASE(2, 64, 0, double) CASE(2, 64, 1, double)
    CASE(3, 32, 0, float) CASE(3, 32, 1, float) CASE(3, 64, 0, double) CASE(3, 64, 1, double)
  }
#undef CASE
}

void do_wrhs(ffd_ctx* h, double* xnew, hipStream_t s) {
  if (h->d == 2) {
    if (h->prec == 32) launch_wrhs<2, float>(h, xnew, s);
    else launch_wrhs<2, double>(h, xnew, s);
  } else {
    if (h->prec == 32) launch_wrhs<3, float>(h, xnew, s);
    else launch_wrhs<3, double>(h, xnew, s);
  }
}

void do_solve(ffd_ctx* h, const double* b, double* x, hipStream_t s) {
  if (h->nF == 0) return;
  if (h->d == 2) launch_solve<2>(h, b, x, s);
  else launch_solve<3>(h, b, x, s);
}

// one iteration of Algorithm 1; with ev != nullptr an event is recorded after
// each of the five phases
void one_iteration(ffd_ctx* h, hipStream_t s, hipEvent_t* ev) {
  double* xold = h->x[h->cur];
  double* xnew = h->x[1 - h->cur];
  do_wrhs(h, xnew, s);
  if (ev) (void)hipEventRecord(ev[0], s);
  if (h->nF > 0) {
    if (h->d == 2) launch_solve_fwd<2>(h, h->b, s);
    else launch_solve_fwd<3>(h, h->b, s);
  }
  if (ev) (void)hipEventRecord(ev[1], s);
  if (h->nF > 0) {
    if (h->d == 2) launch_solve_bwd<2>(h, xnew, s);
    else launch_solve_bwd<3>(h, xnew, s);
  }
  if (ev) (void)hipEventRecord(ev[2], s);
  do_local(h, xnew, xold, s);
  if (ev) (void)hipEventRecord(ev[3], s);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, h->partials, static_cast<int64_t>(nblk(h->m)),
                     h->hist + h->k * FFD_HIST_FIELDS);
  if (ev) (void)hipEventRecord(ev[4], s);
  h->cur = 1 - h->cur;
  h->k += 1;
}

ffd_status ensure_hist(ffd_ctx* h, int64_t need, hipStream_t s) {
  if (need <= h->hist_cap) return FFD_OK;
  int64_t cap = std::max<int64_t>(kHistCap0, h->hist_cap);
  while (cap < need) cap *= 2;
  double* nh = nullptr;
  HIP_TRY(hipMalloc(&nh, cap * FFD_HIST_FIELDS * sizeof(double)));
  if (h->hist) {
    HIP_TRY(hipMemcpyAsync(nh, h->hist, h->hist_cap * FFD_HIST_FIELDS * sizeof(double), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (auto& p : h->allocs)
      if (p == h->hist) p = nh;
    (void)hipFree(h->hist);
    h->device_bytes += (cap - h->hist_cap) * FFD_HIST_FIELDS * sizeof(double);
  } else {
    h->allocs.push_back(nh);
    h->device_bytes += cap * FFD_HIST_FIELDS * sizeof(double);
  }
  h->hist = nh;
  h->hist_cap = cap;
  return FFD_OK;
}

}  // namespace

extern "C" {

const char* ffd_last_error(void) { return g_last_error.c_str(); }

ffd_status ffd_create(const ffd_mesh* mesh, const ffd_options* opt, ffd_handle* out) {
  if (!mesh || !opt || !out) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (!(opt->energy == 0 || opt->energy == 1)) return fail(FFD_ERR_INVALID_ARG, "energy must be 0 or 1");
  if (!(opt->precision == 32 || opt->precision == 64)) return fail(FFD_ERR_INVALID_ARG, "precision must be 32 or 64");
  if (!(opt->h_mode == 0 || opt->h_mode == 1)) return fail(FFD_ERR_INVALID_ARG, "h_mode must be 0 or 1");
  if (opt->n_pinned < 0 || (opt->n_pinned > 0 && !opt->pinned_idx))
    return fail(FFD_ERR_INVALID_ARG, "bad pinned vertex list");
  const int d = mesh->simplex_dim;
  std::vector<int32_t> pins;
  bool auto_pinned = false;
  if (opt->n_pinned > 0) {
    pins.assign(opt->pinned_idx, opt->pinned_idx + opt->n_pinned);
    if (opt->pinned_pos)
      for (int64_t i = 0; i < opt->n_pinned * d; ++i)
        if (!std::isfinite(opt->pinned_pos[i])) return fail(FFD_ERR_NOT_FINITE, "non-finite pinned position");
  } else if (opt->auto_pin) {
    pins.push_back(0);
    auto_pinned = true;
  }
  SetupInput in;
  in.d = d;
  in.din = mesh->dim_in;
  in.n = mesh->n_vertices;
  in.m = mesh->n_elements;
  in.V = mesh->V;
  in.T = mesh->T;
  in.rho = opt->rho;
  in.n_pinned = static_cast<int64_t>(pins.size());
  in.pinned_idx = pins.data();
  in.leaf_size = opt->leaf_size;
  Setup S;
  std::string err;
  int st = build_setup(in, S, err);
  if (st != OK) return fail(static_cast<ffd_status>(st), err);

  auto h = new ffd_ctx();
  auto cleanup = [&](ffd_status s2) {
    std::string msg = g_last_error;
    delete h;
    g_last_error = msg;
    return s2;
  };
  (void)hipGetDevice(&h->dev);
  const auto t0 = std::chrono::steady_clock::now();
  h->d = d;
  h->din = S.din;
  h->prec = opt->precision;
  h->energy = opt->energy;
  h->h_mode = opt->h_mode;
  h->rho = opt->rho;
  h->n = S.n;
  h->m = S.m;
  h->nF = S.nF;
  h->nC = S.nC;
  h->pins_given = opt->n_pinned > 0 && opt->pinned_pos != nullptr;
  h->auto_pinned = auto_pinned;
  h->vnew2old = S.vnew2old;
  const int64_t m = S.m, n = S.n, nc = d + 1;
  hipError_t e = hipSuccess;
#define UP(expr)                                                     \
  do {                                                               \
    e = (expr);                                                      \
    if (e != hipSuccess) {                                           \
      fail(e == hipErrorOutOfMemory ? FFD_ERR_OUT_OF_MEMORY : FFD_ERR_DEVICE, \
           std::string(#expr) + ": " + hipGetErrorString(e));        \
      return cleanup(e == hipErrorOutOfMemory ? FFD_ERR_OUT_OF_MEMORY : FFD_ERR_DEVICE); \
    }                                                                \
  } while (0)
  {
    std::vector<int32_t> Tsoa(static_cast<size_t>(m) * nc);
    for (int64_t el = 0; el < m; ++el)
      for (int c = 0; c < nc; ++c) Tsoa[static_cast<size_t>(c) * m + el] = S.T[el * nc + c];
    UP(upload(h, &h->T, Tsoa));
  }
  UP(upload(h, &h->vnew2old_d, S.vnew2old));
  UP(upload(h, &h->enew2old_d, S.enew2old));
  UP(upload(h, &h->B64, soa<double>(S.B, m, d * d)));
  if (h->prec == 32) {
    float *Bf = nullptr, *wf = nullptr;
    UP(upload(h, &Bf, soa<float>(S.B, m, d * d)));
    UP(upload(h, &wf, soa<float>(S.w, m, 1)));
    h->B = Bf;
    h->w = wf;
  } else {
    double *Bd = nullptr, *wd = nullptr;
    UP(upload(h, &Bd, soa<double>(S.B, m, d * d)));
    UP(upload(h, &wd, S.w));
    h->B = Bd;
    h->w = wd;
  }
  UP(h->alloc(&h->x[0], n * d));
  UP(h->alloc(&h->x[1], n * d));
  UP(h->alloc(&h->xC, std::max<int64_t>(h->nC, 1) * d));
  const size_t rs = h->rsize();
  const int nU = d == 2 ? 2 : 9, nP = d == 2 ? 3 : 6;
  char* tmp = nullptr;
  UP(h->alloc(&tmp, rs * m * nU));
  h->U = tmp;
  UP(h->alloc(&tmp, rs * m * nP));
  h->P = tmp;
  UP(h->alloc(&tmp, rs * m * d * d));
  h->L = tmp;
  UP(h->alloc(&tmp, rs * m));
  h->gn = tmp;
  UP(h->alloc(&tmp, rs * m * nc * d));
  h->g = tmp;
  UP(h->alloc(&h->b, std::max<int64_t>(h->nF, 1) * d));
  UP(h->alloc(&h->y, std::max<int64_t>(h->nF, 1) * d));
  UP(h->alloc(&h->ub, std::max<int64_t>(S.ubuf_rows, 1) * d));
  UP(h->alloc(&h->partials, static_cast<size_t>(nblk(m)) * kNumPartials));
  UP(upload(h, &h->dt_ptr, S.dt_ptr));
  UP(upload(h, &h->dt_idx, S.dt_idx));
  UP(upload(h, &h->pin_ptr, S.pin_ptr));
  UP(upload(h, &h->pin_col, S.pin_col));
  UP(upload(h, &h->pin_val, S.pin_val));
  {
    std::vector<NodeDev> nd(S.nodes.size());
    for (size_t i = 0; i < S.nodes.size(); ++i) {
      const SolveNode& N = S.nodes[i];
      nd[i] = NodeDev{N.first, N.c, N.r, 0, N.pf, N.pb, N.uoff, N.soff, N.poff};
    }
    UP(upload(h, &h->nodes, nd));
    std::vector<int2> tf, tb;
    h->level_fwd_off.push_back(0);
    h->level_bwd_off.push_back(0);
    for (const auto& lvl : S.level_nodes) {
      for (int32_t i : lvl) {
        const SolveNode& N = S.nodes[i];
        for (int r0 = 0; r0 < N.c + N.r; r0 += kRT) tf.push_back(make_int2(i, r0));
        for (int r0 = 0; r0 < N.c; r0 += kRT) tb.push_back(make_int2(i, r0));
      }
      h->level_fwd_off.push_back(static_cast<int32_t>(tf.size()));
      h->level_bwd_off.push_back(static_cast<int32_t>(tb.size()));
    }
    UP(upload(h, &h->tasks_fwd, tf));
    UP(upload(h, &h->tasks_bwd, tb));
  }
  UP(upload(h, &h->Pf, S.panel_f));
  std::vector<double>().swap(S.panel_f);
  UP(upload(h, &h->Pb, S.panel_b));
  std::vector<double>().swap(S.panel_b);
  UP(upload(h, &h->sidx, S.struct_idx));
  UP(upload(h, &h->pull_ptr, S.pull_ptr));
  UP(upload(h, &h->pull_idx, S.pull_idx));
  if (h->pins_given) {
    std::vector<double> pp(opt->pinned_pos, opt->pinned_pos + opt->n_pinned * d);
    UP(hipMemcpy(h->xC, pp.data(), pp.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  UP(hipDeviceSynchronize());
#undef UP
  const auto t1 = std::chrono::steady_clock::now();
  ffd_info& I = h->info;
  I.n_free = S.nF;
  I.n_pinned = S.nC;
  I.factor_nnz = S.factor_nnz;
  I.panel_entries = S.panel_entries;
  I.n_nodes = static_cast<int32_t>(S.nodes.size());
  I.n_levels = static_cast<int32_t>(S.level_nodes.size());
  I.t_geometry = S.t_geometry;
  I.t_order = S.t_order;
  I.t_symbolic = S.t_symbolic;
  I.t_numeric = S.t_numeric;
  I.t_upload = std::chrono::duration<double>(t1 - t0).count();
  I.factor_flops = S.factor_flops;
  *out = h;
  return FFD_OK;
}

ffd_status ffd_analyze(const ffd_mesh* mesh, const ffd_options* opt, ffd_info* info, double* selfcheck_residual) {
  if (!mesh || !opt || !info) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  if (opt->n_pinned < 0 || (opt->n_pinned > 0 && !opt->pinned_idx))
    return fail(FFD_ERR_INVALID_ARG, "bad pinned vertex list");
  std::vector<int32_t> pins;
  if (opt->n_pinned > 0) pins.assign(opt->pinned_idx, opt->pinned_idx + opt->n_pinned);
  else if (opt->auto_pin) pins.push_back(0);
  SetupInput in;
  in.d = mesh->simplex_dim;
  in.din = mesh->dim_in;
  in.n = mesh->n_vertices;
  in.m = mesh->n_elements;
  in.V = mesh->V;
  in.T = mesh->T;
  in.rho = opt->rho;
  in.n_pinned = static_cast<int64_t>(pins.size());
  in.pinned_idx = pins.data();
  in.leaf_size = opt->leaf_size;
  in.selfcheck = selfcheck_residual != nullptr;
  Setup S;
  std::string err;
  const int st = build_setup(in, S, err);
  if (st != OK) return fail(static_cast<ffd_status>(st), err);
  *info = ffd_info{};
  info->n_free = S.nF;
  info->n_pinned = S.nC;
  info->factor_nnz = S.factor_nnz;
  info->panel_entries = S.panel_entries;
  info->n_nodes = static_cast<int32_t>(S.nodes.size());
  info->n_levels = static_cast<int32_t>(S.level_nodes.size());
  info->t_geometry = S.t_geometry;
  info->t_order = S.t_order;
  info->t_symbolic = S.t_symbolic;
  info->t_numeric = S.t_numeric;
  info->factor_flops = S.factor_flops;
  if (selfcheck_residual) *selfcheck_residual = S.selfcheck_residual;
  return FFD_OK;
}

ffd_status ffd_get_info(ffd_handle h, ffd_info* info) {
  if (!h || !info) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  *info = h->info;
  info->device_bytes = h->device_bytes;
  return FFD_OK;
}

ffd_status ffd_init(ffd_handle h, const double* map0_dev, void* stream) {
  if (!h || !map0_dev) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  h->cur = 0;
  hipLaunchKernelGGL((h->d == 2 ? k_map_in<2> : k_map_in<3>), dim3(nblk(h->n)), dim3(kBlock), 0, s, h->n,
                     h->vnew2old_d, map0_dev, h->x[0]);
  // W^0 is used as given; the pins act through the W-step.  Without given pin
  // positions they are taken from W^0.
  if (!h->pins_given && h->nC > 0)
    hipLaunchKernelGGL((h->d == 2 ? k_pins_from_map<2> : k_pins_from_map<3>), dim3(nblk(h->nC)), dim3(kBlock), 0, s,
                       h->nF, h->nC, h->x[0], h->xC);
  do_init(h, s);
  HIP_TRY(hipGetLastError());
  h->k = 0;
  h->initialized = true;
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_set_pins(ffd_handle h, const double* pinned_pos_dev, void* stream) {
  if (!h || !pinned_pos_dev) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  if (h->nC == 0) return FFD_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(h->xC, pinned_pos_dev, h->nC * h->d * sizeof(double), hipMemcpyDeviceToDevice, s));
  h->pins_given = true;
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_iterate(ffd_handle h, int32_t n_iter, void* stream) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (!h->initialized) return fail(FFD_ERR_STATE, "ffd_iterate before ffd_init / ffd_set_state");
  if (n_iter < 0) return fail(FFD_ERR_INVALID_ARG, "negative iteration count");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ffd_status st = ensure_hist(h, h->k + n_iter, s);
  if (st != FFD_OK) return st;
  for (int32_t it = 0; it < n_iter; ++it) one_iteration(h, s, nullptr);
  HIP_TRY(hipGetLastError());
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_iterate_profiled(ffd_handle h, int32_t n_iter, void* stream, double* phase_ms_host) {
  if (!h || !phase_ms_host) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  if (!h->initialized) return fail(FFD_ERR_STATE, "ffd_iterate before ffd_init / ffd_set_state");
  if (n_iter <= 0) return fail(FFD_ERR_INVALID_ARG, "non-positive iteration count");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ffd_status st = ensure_hist(h, h->k + n_iter, s);
  if (st != FFD_OK) return st;
  const size_t need = static_cast<size_t>(n_iter) * 5 + 1;
  while (h->events.size() < need) {
    hipEvent_t ev;
    HIP_TRY(hipEventCreate(&ev));
    h->events.push_back(ev);
  }
  HIP_TRY(hipEventRecord(h->events[0], s));
  for (int32_t it = 0; it < n_iter; ++it) one_iteration(h, s, h->events.data() + 1 + static_cast<size_t>(it) * 5);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventSynchronize(h->events[need - 1]));
  for (int f = 0; f < FFD_PROFILE_FIELDS; ++f) phase_ms_host[f] = 0.0;
  for (int32_t it = 0; it < n_iter; ++it)
    for (int p = 0; p < 5; ++p) {
      float ms = 0.f;
      const size_t i = 1 + static_cast<size_t>(it) * 5 + p;
      HIP_TRY(hipEventElapsedTime(&ms, h->events[i - 1], h->events[i]));
      phase_ms_host[p] += ms;
    }
  float tot = 0.f;
  HIP_TRY(hipEventElapsedTime(&tot, h->events[0], h->events[need - 1]));
  phase_ms_host[5] = tot;
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_get_state(ffd_handle h, double* map_dev, void* Wel_dev, void* U_dev, void* P_dev, void* Lambda_dev,
                         void* stream) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (!h->initialized) return fail(FFD_ERR_STATE, "no state before ffd_init / ffd_set_state");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (map_dev)
    hipLaunchKernelGGL((h->d == 2 ? k_map_out<2> : k_map_out<3>), dim3(nblk(h->n)), dim3(kBlock), 0, s, h->n,
                       h->vnew2old_d, h->x[h->cur], map_dev);
  if (Wel_dev || U_dev || P_dev || Lambda_dev) {
    const unsigned g = nblk(h->m);
    if (h->prec == 32) {
      auto f = h->d == 2 ? k_state_out<2, float> : k_state_out<3, float>;
      hipLaunchKernelGGL(f, dim3(g), dim3(kBlock), 0, s, h->m, h->enew2old_d, static_cast<const float*>(h->U),
                         static_cast<const float*>(h->P), static_cast<const float*>(h->L), static_cast<float*>(U_dev),
                         static_cast<float*>(P_dev), static_cast<float*>(Lambda_dev), static_cast<float*>(Wel_dev));
    } else {
      auto f = h->d == 2 ? k_state_out<2, double> : k_state_out<3, double>;
      hipLaunchKernelGGL(f, dim3(g), dim3(kBlock), 0, s, h->m, h->enew2old_d, static_cast<const double*>(h->U),
                         static_cast<const double*>(h->P), static_cast<const double*>(h->L),
                         static_cast<double*>(U_dev), static_cast<double*>(P_dev), static_cast<double*>(Lambda_dev),
                         static_cast<double*>(Wel_dev));
    }
  }
  HIP_TRY(hipGetLastError());
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_set_state(ffd_handle h, const double* map_dev, const void* U_dev, const void* P_dev,
                         const void* Lambda_dev, int64_t k, void* stream) {
  if (!h || !map_dev || !U_dev || !P_dev || !Lambda_dev) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  if (k < 0) return fail(FFD_ERR_INVALID_ARG, "negative iteration counter");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ffd_status st = ensure_hist(h, k + 1, s);
  if (st != FFD_OK) return st;
  h->cur = 0;
  hipLaunchKernelGGL((h->d == 2 ? k_map_in<2> : k_map_in<3>), dim3(nblk(h->n)), dim3(kBlock), 0, s, h->n,
                     h->vnew2old_d, map_dev, h->x[0]);
  if (!h->pins_given && h->nC > 0)
    hipLaunchKernelGGL((h->d == 2 ? k_pins_from_map<2> : k_pins_from_map<3>), dim3(nblk(h->nC)), dim3(kBlock), 0, s,
                       h->nF, h->nC, h->x[0], h->xC);
  const unsigned g = nblk(h->m);
  if (h->prec == 32) {
    auto f = h->d == 2 ? k_state_in<2, float> : k_state_in<3, float>;
    hipLaunchKernelGGL(f, dim3(g), dim3(kBlock), 0, s, h->m, h->enew2old_d, static_cast<const float*>(U_dev),
                       static_cast<const float*>(P_dev), static_cast<const float*>(Lambda_dev),
                       static_cast<float*>(h->U), static_cast<float*>(h->P), static_cast<float*>(h->L));
  } else {
    auto f = h->d == 2 ? k_state_in<2, double> : k_state_in<3, double>;
    hipLaunchKernelGGL(f, dim3(g), dim3(kBlock), 0, s, h->m, h->enew2old_d, static_cast<const double*>(U_dev),
                       static_cast<const double*>(P_dev), static_cast<const double*>(Lambda_dev),
                       static_cast<double*>(h->U), static_cast<double*>(h->P), static_cast<double*>(h->L));
  }
  do_prepare(h, s);
  HIP_TRY(hipGetLastError());
  h->k = k;
  h->initialized = true;
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_get_history(ffd_handle h, int64_t first, int64_t count, double* out_host) {
  if (!h || (!out_host && count > 0)) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  if (first < 0 || count < 0 || first + count > h->k)
    return fail(FFD_ERR_INVALID_ARG, "history range outside the completed iterations");
  if (count == 0) return FFD_OK;
  HIP_TRY(hipStreamSynchronize(h->last_stream));
  HIP_TRY(hipMemcpy(out_host, h->hist + first * FFD_HIST_FIELDS, count * FFD_HIST_FIELDS * sizeof(double),
                    hipMemcpyDeviceToHost));
  return FFD_OK;
}

ffd_status ffd_get_iteration(ffd_handle h, int64_t* k) {
  if (!h || !k) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  *k = h->k;
  return FFD_OK;
}

ffd_status ffd_solve(ffd_handle h, const double* b_dev, double* x_dev, void* stream) {
  if (!h || !b_dev || !x_dev) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  do_solve(h, b_dev, x_dev, s);
  HIP_TRY(hipGetLastError());
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_get_vertex_order(ffd_handle h, int32_t* order_host) {
  if (!h || !order_host) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  std::memcpy(order_host, h->vnew2old.data(), h->vnew2old.size() * sizeof(int32_t));
  return FFD_OK;
}

void ffd_destroy(ffd_handle h) {
  if (!h) return;
  if (h->last_stream) (void)hipStreamSynchronize(h->last_stream);
  else (void)hipDeviceSynchronize();
  delete h;
}

}  // extern "C"
