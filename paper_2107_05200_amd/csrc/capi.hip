// C ABI of the flip-free ADMM solver (include/ffd.h): handle, device memory,
// and the launch sequence of one iteration of Algorithm 1:
//   K2 W-step right-hand side -> K4 forward solve levels -> K5 backward solve
//   levels -> K3 fused U/P/Lambda step -> finalize (history record).
// This file holds the extern "C" entry points; the runtime they use is one
// translation unit with it, in runtime/ (each header includes the previous):
// context (handle state) -> launch (one iteration) -> schedule (solve task
// lists) -> state (refactorisation, checkpoints, adjoint launches) -> create
// (handle set-up) -> graph (captured iterations) -> tune (autotuner timing).
#include "runtime/tune.hpp"

#include <mutex>

// Fixed scratch of ffd_iterate_noalloc: the per-block partial sums of the
// local step and their first-stage reduction live here instead of in the
// handle's buffers.  One copy per GPU, held until the process ends; every call
// on a GPU shares it (calls that overlap on one GPU race).  In host code the
// name is only a stand-in: the device address comes from hipGetSymbolAddress.
constexpr size_t kScratchDoubles = size_t(1) << 19;  // 4 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxScratchDevices = 64;
double* g_scratch_ptr[kMaxScratchDevices] = {};
std::mutex g_scratch_mutex;

// the current device's copy of `scratch`, looked up once per device
ffd_status scratch_for_current_device(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) return fail(FFD_ERR_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return FFD_OK;
}

// Checks every creating entry point shares, made before any array of the
// caller is read: the mesh's dimensions, the option values, the pinned list
// and the finiteness of the pinned positions.
ffd_status check_mesh_options(const ffd_mesh& M, const ffd_options& O) {
  const int d = M.simplex_dim, din = M.dim_in;
  if (!(d == 2 || d == 3) || !(din == d || (d == 2 && din == 3)))
    return fail(FFD_ERR_INVALID_ARG, "unsupported (simplex_dim, dim_in)");
  if (!(O.energy == 0 || O.energy == 1)) return fail(FFD_ERR_INVALID_ARG, "energy must be 0 or 1");
  if (!(O.precision == 32 || O.precision == 64)) return fail(FFD_ERR_INVALID_ARG, "precision must be 32 or 64");
  if (!(O.h_mode == 0 || O.h_mode == 1)) return fail(FFD_ERR_INVALID_ARG, "h_mode must be 0 or 1");
  if (O.n_pinned < 0 || (O.n_pinned > 0 && !O.pinned_idx)) return fail(FFD_ERR_INVALID_ARG, "bad pinned vertex list");
  if (O.n_pinned > 0 && O.pinned_pos)
    for (int64_t i = 0; i < O.n_pinned * d; ++i)
      if (!std::isfinite(O.pinned_pos[i])) return fail(FFD_ERR_NOT_FINITE, "non-finite pinned position");
  return FFD_OK;
}

}  // namespace

extern "C" {

const char* ffd_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

extern "C" {

ffd_status ffd_create(const ffd_mesh* mesh, const ffd_options* opt, ffd_handle* out) {
  if (!mesh || !opt || !out) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  const ffd_status chk = check_mesh_options(*mesh, *opt);
  if (chk != FFD_OK) return chk;
  const int d = mesh->simplex_dim;
  std::vector<int32_t> pins;
  bool auto_pinned = false;
  if (opt->n_pinned > 0) {
    pins.assign(opt->pinned_idx, opt->pinned_idx + opt->n_pinned);
  } else if (opt->auto_pin) {
    pins.push_back(0);
    auto_pinned = true;
  }
  std::vector<double> ppos;
  if (opt->n_pinned > 0 && opt->pinned_pos) ppos.assign(opt->pinned_pos, opt->pinned_pos + opt->n_pinned * d);
  return create_impl(*mesh, *opt, pins, ppos, auto_pinned, {}, {}, {}, out);
}

ffd_status ffd_create_constrained(const ffd_mesh* mesh, const ffd_options* opt, const ffd_constraints* con,
                                  ffd_handle* out) {
  if (!mesh || !opt || !con || !out) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (con->n_rows <= 0 || con->n_rows > kMaxConstraints || !con->row_ptr || !con->col_idx || !con->val || !con->rhs)
    return fail(FFD_ERR_INVALID_ARG, "constraints: 1 to 1024 rows with row_ptr, col_idx, val and rhs required");
  const ffd_status chk = check_mesh_options(*mesh, *opt);
  if (chk != FFD_OK) return chk;
  const int d = mesh->simplex_dim;
  for (int64_t i = 0; i < con->n_rows * d; ++i)
    if (!std::isfinite(con->rhs[i])) return fail(FFD_ERR_NOT_FINITE, "non-finite constraint right-hand side");
  std::vector<int32_t> pins;
  std::vector<double> ppos;
  if (opt->n_pinned > 0) {
    pins.assign(opt->pinned_idx, opt->pinned_idx + opt->n_pinned);
    if (opt->pinned_pos) ppos.assign(opt->pinned_pos, opt->pinned_pos + opt->n_pinned * d);
  }
  // with constraints no vertex is fixed automatically (the W-step text fixes
  // the first vertex only when there are no constraints)
  return create_impl(*mesh, *opt, pins, ppos, false, {}, {}, {}, out, false, con);
}

ffd_status ffd_set_constraint_rhs(ffd_handle h, const double* rhs_dev, void* stream) {
  if (!h || !rhs_dev) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  if (h->ncon == 0) return fail(FFD_ERR_STATE, "the handle has no general constraints");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(h->con_c, rhs_dev, static_cast<size_t>(h->ncon) * h->d * sizeof(double),
                         hipMemcpyDeviceToDevice, s));
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_tutte_map(const ffd_mesh* mesh, int64_t n_fixed, const int32_t* fixed_idx, const double* fixed_pos,
                         int32_t leaf_size, double* map_dev, void* stream) {
  if (!mesh || !map_dev || n_fixed <= 0 || !fixed_idx || !fixed_pos)
    return fail(FFD_ERR_INVALID_ARG, "NULL argument or no fixed vertex");
  const int d = mesh->simplex_dim;
  if (!(d == 2 || d == 3)) return fail(FFD_ERR_INVALID_ARG, "unsupported simplex_dim");
  for (int64_t i = 0; i < n_fixed * d; ++i)
    if (!std::isfinite(fixed_pos[i])) return fail(FFD_ERR_NOT_FINITE, "non-finite fixed position");
  ffd_options opt{};
  opt.energy = 0;
  opt.rho = 1.0;
  opt.precision = 64;
  opt.leaf_size = leaf_size;
  std::vector<int32_t> pins(fixed_idx, fixed_idx + n_fixed);
  std::vector<double> ppos(fixed_pos, fixed_pos + n_fixed * d);
  ffd_handle h = nullptr;
  ffd_status st = create_impl(*mesh, opt, pins, ppos, false, {}, {}, {}, &h, true);
  if (st != FFD_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // b = -L_FC x_C (the fixed rows go straight into the map), then the two
  // triangular solves into the free rows, then the caller's vertex order
  double* x = h->x[0];
  hipLaunchKernelGGL((d == 2 ? k_fixed_rhs<2> : k_fixed_rhs<3>), dim3(nblk(h->n)), dim3(kBlock), 0, s, h->nF, h->n,
                     h->pin_ptr, h->pin_col, h->pin_val, h->xC, h->b, x);
  do_solve(h, h->b, x, s);
  hipLaunchKernelGGL((d == 2 ? k_map_out<2> : k_map_out<3>), dim3(nblk(h->n)), dim3(kBlock), 0, s, h->n,
                     h->vnew2old_d, x, map_dev);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  ffd_destroy(h);
  if (e != hipSuccess) return fail(FFD_ERR_DEVICE, hipGetErrorString(e));
  return FFD_OK;
}

ffd_status ffd_batch_create(const ffd_mesh* meshes, const ffd_options* opts, int32_t n_meshes, ffd_handle* out) {
  if (!meshes || !opts || !out || n_meshes <= 0) return fail(FFD_ERR_INVALID_ARG, "NULL argument or no meshes");
  *out = nullptr;
  const ffd_options& o0 = opts[0];
  const int d = meshes[0].simplex_dim, din = meshes[0].dim_in;
  for (int32_t b = 0; b < n_meshes; ++b) {
    const ffd_status chk = check_mesh_options(meshes[b], opts[b]);
    if (chk != FFD_OK) return chk;
  }
  const bool with_pos = o0.n_pinned > 0 && o0.pinned_pos != nullptr;
  std::vector<double> V;
  std::vector<int32_t> T, pins;
  std::vector<double> ppos;
  std::vector<int8_t> energy;
  std::vector<int64_t> voff{0}, eoff{0};
  for (int32_t b = 0; b < n_meshes; ++b) {
    const ffd_mesh& M = meshes[b];
    const ffd_options& O = opts[b];
    if (M.simplex_dim != d || M.dim_in != din) return fail(FFD_ERR_INVALID_ARG, "meshes of a batch share d and dim_in");
    if (O.precision != o0.precision || O.h_mode != o0.h_mode || O.rho != o0.rho)
      return fail(FFD_ERR_INVALID_ARG, "meshes of a batch share precision, h_mode and rho");
    if (!M.V || !M.T || M.n_vertices <= 0 || M.n_elements <= 0) return fail(FFD_ERR_INVALID_ARG, "empty mesh");
    const int64_t vb = voff.back();
    if (vb + M.n_vertices > INT32_MAX / 2) return fail(FFD_ERR_INVALID_ARG, "batch too large");
    V.insert(V.end(), M.V, M.V + M.n_vertices * din);
    for (int64_t i = 0; i < M.n_elements * (d + 1); ++i) {
      if (M.T[i] < 0 || M.T[i] >= M.n_vertices) return fail(FFD_ERR_INVALID_ARG, "element index out of range");
      T.push_back(static_cast<int32_t>(M.T[i] + vb));
    }
    energy.insert(energy.end(), M.n_elements, static_cast<int8_t>(O.energy));
    if (O.n_pinned > 0) {
      if ((O.pinned_pos != nullptr) != with_pos)
        return fail(FFD_ERR_INVALID_ARG, "give pinned positions for all meshes of a batch or for none");
      for (int64_t i = 0; i < O.n_pinned; ++i) {
        if (O.pinned_idx[i] < 0 || O.pinned_idx[i] >= M.n_vertices)
          return fail(FFD_ERR_INVALID_ARG, "pinned index out of range");
        pins.push_back(static_cast<int32_t>(O.pinned_idx[i] + vb));
      }
      if (with_pos) ppos.insert(ppos.end(), O.pinned_pos, O.pinned_pos + O.n_pinned * d);
    } else if (O.auto_pin) {
      if (with_pos) return fail(FFD_ERR_INVALID_ARG, "an auto-pinned mesh in a batch with given pin positions");
      pins.push_back(static_cast<int32_t>(vb));
    }
    voff.push_back(vb + M.n_vertices);
    eoff.push_back(eoff.back() + M.n_elements);
  }
  ffd_mesh all{d, din, voff.back(), eoff.back(), V.data(), T.data()};
  ffd_options common = o0;
  return create_impl(all, common, pins, ppos, false, energy, voff, eoff, out);
}

ffd_status ffd_batch_layout(ffd_handle h, int64_t* vertex_offsets, int64_t* element_offsets) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (h->voff.empty()) {
    if (vertex_offsets) {
      vertex_offsets[0] = 0;
      vertex_offsets[1] = h->n;
    }
    if (element_offsets) {
      element_offsets[0] = 0;
      element_offsets[1] = h->m;
    }
    return FFD_OK;
  }
  if (vertex_offsets) std::memcpy(vertex_offsets, h->voff.data(), h->voff.size() * sizeof(int64_t));
  if (element_offsets) std::memcpy(element_offsets, h->eoff.data(), h->eoff.size() * sizeof(int64_t));
  return FFD_OK;
}

ffd_status ffd_analyze(const ffd_mesh* mesh, const ffd_options* opt, ffd_info* info, double* selfcheck_residual) {
  if (!mesh || !opt || !info) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  const ffd_status chk = check_mesh_options(*mesh, *opt);
  if (chk != FFD_OK) return chk;
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
  if (h->rescaled) {  // back to mu_i = rho w_i and its factor
    h->rescaled = false;
    h->graph_valid = false;
    const ffd_status st = refactor(h, nullptr, s);
    if (st != FFD_OK) return st;
  }
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
  for (int32_t it = 0; it < n_iter; ++it) one_iteration(h, s, nullptr, true, it == n_iter - 1);
  HIP_TRY(hipGetLastError());
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_iterate_noalloc(ffd_handle h, int32_t n_iter, void* stream) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (!h->initialized) return fail(FFD_ERR_STATE, "ffd_iterate_noalloc before ffd_init / ffd_set_state");
  if (n_iter < 0) return fail(FFD_ERR_INVALID_ARG, "negative iteration count");
  if (h->k + n_iter > h->hist_cap)
    return fail(FFD_ERR_INVALID_ARG, "the history holds " + std::to_string(h->hist_cap) + " records; " +
                                         std::to_string(h->k + n_iter) + " would need a larger one (allocation)");
  const int64_t nb2 = h->nparts > 2 * kFinalizeRows ? (h->nparts + kFinalizeRows - 1) / kFinalizeRows : 0;
  const size_t need = static_cast<size_t>(h->nparts + nb2) * kNumPartials;
  if (need > kScratchDoubles)
    return fail(FFD_ERR_INVALID_ARG, "the local step needs " + std::to_string(need) +
                                         " float64 of scratch; the fixed scratch holds " +
                                         std::to_string(kScratchDoubles));
  double* sp = nullptr;
  const ffd_status st = scratch_for_current_device(&sp);
  if (st != FFD_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the launches of ffd_iterate with the partial sums redirected to the
  // scratch (every block writes its partials before the reduction reads them,
  // so nothing needs clearing)
  double* const own = h->partials;
  double* const own2 = h->partials2;
  h->partials = sp;
  h->partials2 = sp + static_cast<size_t>(h->nparts) * kNumPartials;
  for (int32_t it = 0; it < n_iter; ++it) one_iteration(h, s, nullptr, true, it == n_iter - 1);
  h->partials = own;
  h->partials2 = own2;
  HIP_TRY(hipGetLastError());
  h->last_stream = s;
  return FFD_OK;
}

}  // extern "C"

extern "C" {

ffd_status ffd_iterate_graph(ffd_handle h, int32_t n_iter, void* stream) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (!h->initialized) return fail(FFD_ERR_STATE, "ffd_iterate_graph before ffd_init / ffd_set_state");
  if (n_iter < 0) return fail(FFD_ERR_INVALID_ARG, "negative iteration count");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ffd_status st = ensure_hist(h, h->k + n_iter, s);
  if (st != FFD_OK) return st;
  int32_t n = n_iter;
  if (n >= 2) {
    if (!h->graph_valid || h->graph_hist != h->hist) {
      st = capture_graph(h);
      if (st != FFD_OK) return st;
    }
    if (h->cur != h->graph_cur) {
      one_iteration(h, s, nullptr, true, false);
      --n;
    }
    const int32_t reps = n / 2;
    if (reps > 0) {
      hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, s, h->k_dev, h->k);
      for (int32_t r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(h->graph_exec, s));
      h->k += 2 * static_cast<int64_t>(reps);
      n -= 2 * reps;
    }
  }
  for (int32_t it = 0; it < n; ++it) one_iteration(h, s, nullptr, true, it == n - 1);
  HIP_TRY(hipGetLastError());
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_iterate_until(ffd_handle h, int32_t max_iter, int32_t check_every, double eps_abs, double eps_rel,
                             int32_t require_flip_free, int32_t use_graph, void* stream, int32_t* iters_done,
                             int32_t* converged) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (!h->initialized) return fail(FFD_ERR_STATE, "ffd_iterate_until before ffd_init / ffd_set_state");
  if (max_iter < 0 || check_every < 1 || !(eps_abs >= 0.0) || !(eps_rel >= 0.0))
    return fail(FFD_ERR_INVALID_ARG, "max_iter >= 0, check_every >= 1 and eps_abs, eps_rel >= 0 required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ffd_status st = ensure_hist(h, h->k + max_iter, s);
  if (st != FFD_OK) return st;
  if (!h->glam) HIP_TRY(h->alloc(reinterpret_cast<char**>(&h->glam), h->rsize() * h->m * (h->d + 1) * h->d));
  if (!h->gtl_part) HIP_TRY(h->alloc(&h->gtl_part, static_cast<size_t>((4 * h->n + kBlock - 1) / kBlock)));
  int32_t done = 0, conv = 0;
  while (done < max_iter) {
    const int32_t blk = std::min(check_every, max_iter - done);
    if (blk > 1) {
      if (use_graph) {
        st = ffd_iterate_graph(h, blk - 1, stream);
        if (st != FFD_OK) return st;
      } else {
        // the iteration before the check stores U^{k-1} for the Lambda-ratio proxy
        for (int32_t it = 0; it < blk - 1; ++it) one_iteration(h, s, nullptr, true, it == blk - 2);
      }
    }
    one_iteration(h, s, nullptr, true, true, false, true);
    done += blk;
    bool ok = false;
    st = check_termination(h, s, eps_abs, eps_rel, require_flip_free != 0, &ok);
    if (st != FFD_OK) return st;
    if (ok) {
      conv = 1;
      break;
    }
  }
  HIP_TRY(hipGetLastError());
  if (iters_done) *iters_done = done;
  if (converged) *converged = conv;
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_set_refactor_mode(ffd_handle h, int32_t device) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (device && !dense_lib().ok) return fail(FFD_ERR_STATE, "rocBLAS / rocSOLVER not available");
  h->device_refactor = device != 0;
  return FFD_OK;
}

ffd_status ffd_rescale(ffd_handle h, double rho_r, void* stream) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (!h->initialized || h->k < 1) return fail(FFD_ERR_STATE, "ffd_rescale needs an iteration after ffd_init");
  if (!(rho_r > 2.0) || !std::isfinite(rho_r)) return fail(FFD_ERR_INVALID_ARG, "rescaling factor must exceed 2");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ffd_status st = do_rescale(h, rho_r, s);
  h->last_stream = s;
  return st;
}

ffd_status ffd_run(ffd_handle h, int32_t max_iter, int32_t check_every, double eps_abs, double eps_rel,
                   int32_t require_flip_free, double rescale_rho, int32_t use_graph, void* stream, int32_t* iters_done,
                   int32_t* converged, int32_t* rescales_done) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (!h->initialized) return fail(FFD_ERR_STATE, "ffd_run before ffd_init / ffd_set_state");
  if (max_iter < 0 || check_every < 1 || !(eps_abs >= 0.0) || !(eps_rel >= 0.0) ||
      (rescale_rho != 0.0 && !(rescale_rho > 2.0)))
    return fail(FFD_ERR_INVALID_ARG, "max_iter >= 0, check_every >= 1, tolerances >= 0, rescale_rho 0 or > 2 required");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ffd_status st = ensure_hist(h, h->k + max_iter, s);
  if (st != FFD_OK) return st;
  if (!h->glam) HIP_TRY(h->alloc(reinterpret_cast<char**>(&h->glam), h->rsize() * h->m * (h->d + 1) * h->d));
  if (!h->gtl_part) HIP_TRY(h->alloc(&h->gtl_part, static_cast<size_t>((4 * h->n + kBlock - 1) / kBlock)));
  // rescaling events: after iterations 1..5 of this run, then every
  // 5 (3/2)^p iterations (p past events, rounded half up)
  auto next_event = [&](int32_t after) -> int64_t {
    if (rescale_rho == 0.0) return INT64_MAX;
    int64_t k = 0, q = 0;
    while (true) {
      k = q < 5 ? k + 1 : k + static_cast<int64_t>(std::floor(5.0 * std::pow(1.5, static_cast<double>(q)) + 0.5));
      if (k > after) return k;
      ++q;
    }
  };
  int32_t done = 0, conv = 0, nres = 0;
  auto plain = [&](int32_t n) -> ffd_status {
    if (n <= 0) return FFD_OK;
    if (use_graph) return ffd_iterate_graph(h, n, stream);
    for (int32_t it = 0; it < n; ++it) one_iteration(h, s, nullptr, true, it == n - 1);
    return FFD_OK;
  };
  // Algorithm 2's loop body: the iteration, the rescaling block if the
  // iteration is an event, then the termination test at check iterations on
  // the state as it stands (after the event's new mu and Lambda)
  while (done < max_iter) {
    const int64_t ev = next_event(done);
    const int64_t ck = (static_cast<int64_t>(done) / check_every + 1) * check_every;
    const int32_t target = static_cast<int32_t>(std::min<int64_t>({ev, ck, static_cast<int64_t>(max_iter)}));
    const bool is_check = target == ck, is_event = target == ev;
    st = plain(target - done - 1);
    if (st != FFD_OK) return st;
    one_iteration(h, s, nullptr, true, true, false, is_check);
    done = target;
    if (is_event) {
      st = do_rescale(h, rescale_rho, s, is_check ? h->glam : nullptr);
      if (st != FFD_OK) return st;
      ++nres;
    }
    if (!is_check) continue;
    bool ok = false;
    st = check_termination(h, s, eps_abs, eps_rel, require_flip_free != 0, &ok);
    if (st != FFD_OK) return st;
    if (ok) {
      conv = 1;
      break;
    }
  }
  HIP_TRY(hipGetLastError());
  if (iters_done) *iters_done = done;
  if (converged) *converged = conv;
  if (rescales_done) *rescales_done = nres;
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
  for (int32_t it = 0; it < n_iter; ++it)
    one_iteration(h, s, h->events.data() + 1 + static_cast<size_t>(it) * 5, true, it == n_iter - 1);
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

ffd_status ffd_profile_solve_levels(ffd_handle h, int32_t n_rep, void* stream, double* out_host, int32_t cap_levels,
                                   int32_t* n_levels) {
  if (!h || !out_host || !n_levels) return fail(FFD_ERR_INVALID_ARG, "NULL argument");
  if (n_rep <= 0) return fail(FFD_ERR_INVALID_ARG, "non-positive repetition count");
  const int nlev = static_cast<int>(h->hlevels.size());
  *n_levels = nlev;
  if (cap_levels < nlev) return fail(FFD_ERR_INVALID_ARG, "output holds fewer levels than the schedule has");
  if (h->solve_groups != 1) return fail(FFD_ERR_STATE, "per-level timing needs the single-stream schedule");
  if (h->nF == 0) return fail(FFD_ERR_STATE, "no free vertices");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t need = 2 * static_cast<size_t>(nlev) + 1;
  while (h->events.size() < need) {
    hipEvent_t ev;
    HIP_TRY(hipEventCreate(&ev));
    h->events.push_back(ev);
  }
  std::vector<double> ms(2 * nlev, 0.0);
  double* xs = h->x[1 - h->cur];  // the next map buffer: overwritten by the next W-step anyway
  const int top = h->solve_top;
  for (int rep = 0; rep <= n_rep; ++rep) {  // the first repetition is not timed
    HIP_TRY(hipEventRecord(h->events[0], s));
    for (int l = 0; l < nlev; ++l) {
      const LevelRun& r = l < top ? h->grun_fwd[0][l] : h->grun_fwd[1][l];
      if (h->d == 2) launch_fwd_level<2>(h, r, h->b, s, r.reduce_now);
      else launch_fwd_level<3>(h, r, h->b, s, r.reduce_now);
      HIP_TRY(hipEventRecord(h->events[1 + l], s));
    }
    for (int l = nlev - 1; l >= 0; --l) {
      const LevelRun& r = l >= top ? h->grun_bwd[1][l] : h->grun_bwd[0][l];
      if (h->d == 2) launch_bwd_level<2>(h, r, xs, s);
      else launch_bwd_level<3>(h, r, xs, s);
      HIP_TRY(hipEventRecord(h->events[1 + nlev + (nlev - 1 - l)], s));
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventSynchronize(h->events[need - 1]));
    if (rep == 0) continue;
    for (int l = 0; l < nlev; ++l) {
      float a = 0.f, b = 0.f;
      HIP_TRY(hipEventElapsedTime(&a, h->events[l], h->events[1 + l]));
      const int i = 1 + nlev + (nlev - 1 - l);
      HIP_TRY(hipEventElapsedTime(&b, h->events[i - 1], h->events[i]));
      ms[2 * l] += a;
      ms[2 * l + 1] += b;
    }
  }
  for (int l = 0; l < nlev; ++l) {
    double nnz = 0.0, cmax = 0.0, rmax = 0.0;
    for (int32_t i : h->hlevels[l]) {
      const SolveNode& N = h->hnodes[i];
      nnz += 0.5 * N.c * (N.c + 1.0) + static_cast<double>(N.c) * N.r;
      cmax = std::max(cmax, static_cast<double>(N.c));
      rmax = std::max(rmax, static_cast<double>(N.r));
    }
    const LevelRun& rf = l < top ? h->grun_fwd[0][l] : h->grun_fwd[1][l];
    const LevelRun& rb = l >= top ? h->grun_bwd[1][l] : h->grun_bwd[0][l];
    double* o = out_host + static_cast<size_t>(l) * FFD_LEVEL_FIELDS;
    o[0] = ms[2 * l] / n_rep;
    o[1] = ms[2 * l + 1] / n_rep;
    o[2] = 8.0 * nnz;
    o[3] = static_cast<double>(h->hlevels[l].size());
    o[4] = cmax;
    o[5] = rmax;
    o[6] = rf.nt;
    o[7] = rb.nt;
    o[8] = rf.nr;
    o[9] = rb.nr * (rb.reduce_now ? 1.0 : 0.0);
  }
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

ffd_status ffd_adjoint_forward(ffd_handle h, int32_t n_iter, int32_t checkpoint_every, void* stream) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (!h->initialized) return fail(FFD_ERR_STATE, "ffd_adjoint_forward before ffd_init / ffd_set_state");
  if (n_iter <= 0 || checkpoint_every <= 0) return fail(FFD_ERR_INVALID_ARG, "n_iter and checkpoint_every must be > 0");
  if (h->rescaled) return fail(FFD_ERR_STATE, "the adjoint differentiates mu_i = rho w_i: not after a rescaling");
  if (h->ncon > 0) return fail(FFD_ERR_STATE, "the adjoint is not built for general constraints");
  if (h->h_mode != 0)
    return fail(FFD_ERR_STATE, "the adjoint differentiates the U-step without the proximal term (h_mode 0)");
  hipStream_t s = static_cast<hipStream_t>(stream);
  ffd_status st = ensure_hist(h, h->k + n_iter, s);
  if (st != FFD_OK) return st;
  const int64_t nslots = (n_iter + checkpoint_every - 1) / checkpoint_every;
  const size_t sb = h->slot_bytes();
  if (nslots > h->adj_nslots || checkpoint_every != h->adj_every) {
    HIP_TRY(hipStreamSynchronize(s));
    for (char** pp : {&h->adj_ck, &h->adj_seg, &h->adj_fin})
      if (*pp) {
        for (auto& a : h->allocs)
          if (a == *pp) a = nullptr;
        (void)hipFree(*pp);
        *pp = nullptr;
      }
    HIP_TRY(h->alloc(&h->adj_ck, sb * nslots));
    HIP_TRY(h->alloc(&h->adj_seg, sb * checkpoint_every));  // recomputed states 1 .. every - 1
    HIP_TRY(h->alloc(&h->adj_fin, sb));
    h->adj_nslots = nslots;
  }
  h->adj_k0 = h->k;
  h->adj_K = n_iter;
  h->adj_every = checkpoint_every;
  for (int32_t it = 0; it < n_iter; ++it) {
    if (it % checkpoint_every == 0) HIP_TRY(save_state(h, h->adj_ck + sb * (it / checkpoint_every), s));
    one_iteration(h, s, nullptr);
  }
  HIP_TRY(hipGetLastError());
  h->last_stream = s;
  return FFD_OK;
}

ffd_status ffd_adjoint_backward(ffd_handle h, const void* Pbar_dev, int32_t energy_loss, double* pins_bar_dev,
                                double* V_bar_dev, void* stream) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (h->adj_k0 < 0 || h->k != h->adj_k0 + h->adj_K)
    return fail(FFD_ERR_STATE, "ffd_adjoint_backward needs ffd_adjoint_forward as the last iterations");
  if (V_bar_dev && h->din != h->d)
    return fail(FFD_ERR_INVALID_ARG, "rest-vertex gradients need dim_in == simplex_dim");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int d = h->d;
  const int64_t m = h->m, n = h->n;
  if (!h->Ubar) {
    HIP_TRY(h->alloc(&h->Ubar, m * d * d));
    HIP_TRY(h->alloc(&h->Pbar, m * d * d));
    HIP_TRY(h->alloc(&h->Lbar, m * d * d));
    HIP_TRY(h->alloc(&h->Bbar, m * d * d));
    HIP_TRY(h->alloc(&h->wbar, m));
    HIP_TRY(h->alloc(&h->gadj, m * (d + 1) * d));
    HIP_TRY(h->alloc(&h->lam, n * d));
    HIP_TRY(h->alloc(&h->xbar, std::max<int64_t>(h->nF, 1) * d));
    HIP_TRY(h->alloc(&h->pinsbar, std::max<int64_t>(h->nC, 1) * d));
    HIP_TRY(h->alloc(&h->vbar, n * d));
  }
  HIP_TRY(hipMemsetAsync(h->lam, 0, sizeof(double) * n * d, s));
  HIP_TRY(hipMemsetAsync(h->pinsbar, 0, sizeof(double) * std::max<int64_t>(h->nC, 1) * d, s));
  const size_t sb = h->slot_bytes();
  HIP_TRY(save_state(h, h->adj_fin, s));
  for (const auto& g : h->segs) SEG_CASES(launch_adj_seed, h, g, Pbar_dev, energy_loss, s)
  const int64_t K = h->adj_K, every = h->adj_every;
  const int64_t nseg = (K + every - 1) / every;
  for (int64_t seg = nseg - 1; seg >= 0; --seg) {
    const int64_t start = seg * every, len = std::min(every, K - start);
    // states of the segment: t = 0 is its checkpoint; 1 .. len - 1 are
    // recomputed from it; of the state after the segment only the map is read,
    // and it is the next checkpoint's (the final state's for the last
    // segment), bitwise what a recomputation would give.  With a checkpoint
    // every iteration nothing is recomputed.
    char* const ck = h->adj_ck + sb * seg;
    const double* const xlast = slot_view(h, seg + 1 < nseg ? h->adj_ck + sb * (seg + 1) : h->adj_fin).x;
    auto state = [&](int64_t t) { return slot_view(h, t == 0 ? ck : h->adj_seg + sb * t); };
    if (len > 1) HIP_TRY(load_state(h, ck, s));
    for (int64_t t = 1; t < len; ++t) {
      one_iteration(h, s, nullptr, false);
      HIP_TRY(save_state(h, h->adj_seg + sb * t, s));
    }
    for (int64_t t = len; t >= 1; --t) {
      const SlotView prev = state(t - 1);
      const double* xk = t == len ? xlast : state(t).x;
      for (const auto& g : h->segs) SEG_CASES(launch_adj_local, h, g, prev, xk, s)
      hipLaunchKernelGGL((d == 2 ? k_adj_gather<2> : k_adj_gather<3>), dim3(nblk(n)), dim3(kBlock), 0, s, h->nF, n,
                         h->av_ptr, h->av_idx, h->gadj, h->xbar, h->pinsbar, 1.0);
      do_solve(h, h->xbar, h->lam, s);
      ADJ_DISPATCH(launch_adj_wstep, h, prev, xk, s);
      if (h->nC > 0)
        hipLaunchKernelGGL((d == 2 ? k_adj_pins<2> : k_adj_pins<3>), dim3(nblk(h->nC)), dim3(kBlock), 0, s, h->nC,
                           h->lcf_ptr, h->lcf_col, h->lcf_val, h->lam, h->pinsbar);
    }
  }
  if (V_bar_dev) {
    ADJ_DISPATCH(launch_adj_vbar, h, s);
    // all rows: pass nF = 0 so every row is written to vbar
    hipLaunchKernelGGL((d == 2 ? k_adj_gather<2> : k_adj_gather<3>), dim3(nblk(n)), dim3(kBlock), 0, s, n, n,
                       h->av_ptr, h->av_idx, h->gadj, h->vbar, static_cast<double*>(nullptr), 0.0);
    hipLaunchKernelGGL((d == 2 ? k_map_out<2> : k_map_out<3>), dim3(nblk(n)), dim3(kBlock), 0, s, n, h->vnew2old_d,
                       h->vbar, V_bar_dev);
  }
  if (pins_bar_dev && h->nC > 0)
    HIP_TRY(hipMemcpyAsync(pins_bar_dev, h->pinsbar, sizeof(double) * h->nC * d, hipMemcpyDeviceToDevice, s));
  HIP_TRY(load_state(h, h->adj_fin, s));
  HIP_TRY(hipGetLastError());
  h->last_stream = s;
  return FFD_OK;
}

}  // extern "C"

extern "C" {

ffd_status ffd_autotune(ffd_handle h, const char* cache_path, void* stream, int32_t* choice_out) {
  if (!h) return fail(FFD_ERR_INVALID_ARG, "NULL handle");
  if (!h->initialized) return fail(FFD_ERR_STATE, "ffd_autotune before ffd_init / ffd_set_state");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const std::string key = tune_key(h);
  const size_t nlev = h->hlevels.size();
  int bs = 0, lpr = 0, groups = 1, topl = static_cast<int>(nlev);
  std::vector<LevelCfg> cf, cb;
  bool cached = false;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      std::string line;
      char buf[4096];
      while (std::fgets(buf, sizeof buf, f)) {
        line += buf;
        if (line.empty() || line.back() != '\n') continue;  // a line longer than the buffer
        std::istringstream in(line);
        line.clear();
        std::string k;
        int b2 = 0, l2 = 0;
        size_t n2 = 0;
        int g2 = 1, t2 = 0;
        if (!(in >> k >> b2 >> l2 >> n2 >> g2 >> t2) || k != key || n2 != nlev) continue;
        std::vector<LevelCfg> f2(nlev), h2(nlev);
        bool good = g2 >= 1 && g2 <= 8 && t2 >= 0 && t2 <= static_cast<int>(nlev);
        for (size_t l = 0; l < nlev && good; ++l)
          good = static_cast<bool>(in >> f2[l].mode >> f2[l].opt >> f2[l].chunk >> f2[l].nw >> f2[l].defer);
        for (size_t l = 0; l < nlev && good; ++l)
          good = static_cast<bool>(in >> h2[l].mode >> h2[l].opt >> h2[l].chunk >> h2[l].nw >> h2[l].defer);
        if (!good) continue;
        bs = b2;
        lpr = l2;
        cf = f2;
        cb = h2;
        groups = g2;
        topl = t2;
        cached = true;
      }
      std::fclose(f);
    }
  }
  // a configuration read from a file is checked before use
  auto valid = [](const LevelCfg& c) {
    return (c.mode == 0 || c.mode == 1) && (c.opt == 16 || c.opt == 32 || c.opt == 64) && c.chunk >= 0 &&
           (c.mode == 0 || c.chunk == 0) && (c.nw == 4 || c.nw == 8 || c.nw == 16) && (c.defer == 0 || c.defer == 1);
  };
  for (size_t l = 0; l < cf.size() && cached; ++l) cached = valid(cf[l]) && valid(cb[l]);
  if (!cached) {
    // coordinate search with the state saved and restored around it; the
    // timed iterations are not recorded in the history
    if (!h->adj_fin) HIP_TRY(h->alloc(&h->adj_fin, h->slot_bytes()));
    HIP_TRY(save_state(h, h->adj_fin, s));
    const int iters = 6;
    double best = 1e300;
    for (int cand : {256, 128, 64}) {
      set_local_block(h, cand);
      const double t = time_phase(h, s, 3, iters);
      if (t < best) {
        best = t;
        bs = cand;
      }
    }
    set_local_block(h, bs);
    best = 1e300;
    for (int cand : {4, 2, 8}) {
      h->wrhs_lpr = cand;
      h->graph_valid = false;
      const double t = time_phase(h, s, 0, iters);
      if (t < best) {
        best = t;
        lpr = cand;
      }
    }
    h->wrhs_lpr = lpr;
    // solve levels one at a time, both passes, from the default schedule
    h->cfg_fwd.clear();
    h->cfg_bwd.clear();
    h->solve_groups = 1;
    ffd_status st = build_solve_schedule(h);
    if (st != FFD_OK) return st;
    // forward levels are timed with the backward pass too: deferred forward
    // partials are added there
    auto timed = [&](int pass) {
      const double tb = time_solve_pass(h, s, false, 3);
      return pass == 0 ? time_solve_pass(h, s, true, 3) + tb : tb;
    };
    // two sweeps; each level's current choice is timed afresh before its
    // candidates (a stale minimum from earlier levels would favour it), and a
    // candidate must beat it by 0.5%
    for (int sweep = 0; sweep < 2; ++sweep)
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<LevelCfg>& cfg = pass == 0 ? h->cfg_fwd : h->cfg_bwd;
      for (size_t l = 0; l < nlev; ++l) {
        int64_t max_inner = 0;
        for (const OutBlock& o : level_blocks(h, h->hlevels[l], pass == 0, 64))
          max_inner = std::max<int64_t>(max_inner, o.hi - o.lo);
        std::vector<LevelCfg> cands;
        for (int opt : {64, 32, 16}) {
          if (max_inner <= 1024) cands.push_back(LevelCfg{1, opt, 0, 4, 0});
          for (int nw : {4, 8, 16})
            for (int chunk : {0, 2048, 1024, 512, 256})
              if ((chunk == 0 || chunk < max_inner) && (nw == 4 || chunk == 0 || chunk >= 1024))
                for (int defer : {0, 1})
                  if (defer == 0 || (chunk > 0 && (pass == 0 || l > 0))) cands.push_back(LevelCfg{0, opt, chunk, nw, defer});
        }
        const LevelCfg keep = cfg[l];
        st = build_solve_schedule(h);
        if (st != FFD_OK) return st;
        double tcur = 0.995 * timed(pass);
        LevelCfg bestc = keep;
        for (const LevelCfg& c : cands) {
          if (c == keep) continue;
          cfg[l] = c;
          st = build_solve_schedule(h);
          if (st != FFD_OK) return st;
          const double t = timed(pass);
          if (t < tcur) {
            tcur = t;
            bestc = c;
          }
        }
        cfg[l] = bestc;
      }
    }
    cf = h->cfg_fwd;
    cb = h->cfg_bwd;
    // then the forest below a top level split over 2..4 streams, kept only
    // when it beats one stream by more than 3% (run-to-run noise is ~2%)
    const double t_one = time_solve_pass(h, s, true, 3) + time_solve_pass(h, s, false, 3);
    double tbest = 0.97 * t_one;
    groups = 1;
    topl = static_cast<int>(nlev);
    HIP_TRY(ensure_workers(h, 4));
    for (int g = 2; g <= 4; ++g)
      for (int t = static_cast<int>(nlev) - 1; t >= std::max(1, static_cast<int>(nlev) - 6); --t) {
        h->solve_groups = g;
        h->solve_top = t;
        st = build_solve_schedule(h);
        if (st != FFD_OK) return st;
        const double tt = time_solve_pass(h, s, true, 3) + time_solve_pass(h, s, false, 3);
        if (tt < tbest) {
          tbest = tt;
          groups = g;
          topl = t;
        }
      }
    h->solve_groups = groups;
    h->solve_top = topl;
    st = build_solve_schedule(h);
    if (st != FFD_OK) return st;
    HIP_TRY(load_state(h, h->adj_fin, s));
    if (cache_path) {
      if (FILE* f = std::fopen(cache_path, "a")) {
        std::fprintf(f, "%s %d %d %zu %d %d", key.c_str(), bs, lpr, nlev, groups, topl);
        for (const LevelCfg& c : cf) std::fprintf(f, " %d %d %d %d %d", c.mode, c.opt, c.chunk, c.nw, c.defer);
        for (const LevelCfg& c : cb) std::fprintf(f, " %d %d %d %d %d", c.mode, c.opt, c.chunk, c.nw, c.defer);
        std::fprintf(f, "\n");
        std::fclose(f);
      }
    }
  }
  if (bs != 64 && bs != 128 && bs != 256) bs = 256;
  if (lpr != 2 && lpr != 4 && lpr != 8) lpr = 4;
  set_local_block(h, bs);
  h->wrhs_lpr = lpr;
  h->graph_valid = false;
  h->cfg_fwd = cf;
  h->cfg_bwd = cb;
  HIP_TRY(ensure_workers(h, groups));
  h->solve_groups = groups;
  h->solve_top = topl;
  ffd_status st = build_solve_schedule(h);
  if (st != FFD_OK) return st;
  HIP_TRY(hipStreamSynchronize(s));
  if (choice_out) {
    int32_t wave = 0, split = 0;
    for (const auto* v : {&cf, &cb})
      for (const LevelCfg& c : *v) {
        wave += c.mode == 1;
        split += c.chunk > 0;
      }
    choice_out[0] = bs;
    choice_out[1] = lpr;
    choice_out[2] = wave;
    choice_out[3] = split;
    choice_out[4] = h->solve_groups;
    choice_out[5] = h->solve_top;
  }
  h->last_stream = s;
  return FFD_OK;
}

void ffd_destroy(ffd_handle h) {
  if (!h) return;
  if (h->last_stream) (void)hipStreamSynchronize(h->last_stream);
  else (void)hipDeviceSynchronize();
  delete h;
}

}  // extern "C"
