// Handle creation shared by ffd_create, ffd_create_constrained,
// ffd_batch_create and ffd_tutte_map: host set-up, upload, default schedule.
// Part of the single translation unit capi.hip.
#pragma once

#include "state.hpp"

namespace {

// shared by ffd_create and ffd_batch_create: mesh is the (concatenated) mesh,
// opt the common options, pins in mesh indices, pin_pos empty = taken from W^0
ffd_status create_impl(const ffd_mesh& mesh_in, const ffd_options& opt, const std::vector<int32_t>& pins,
                       const std::vector<double>& pin_pos, bool auto_pinned, const std::vector<int8_t>& elem_energy,
                       const std::vector<int64_t>& voff, const std::vector<int64_t>& eoff, ffd_handle* out,
                       bool tutte = false, const ffd_constraints* con = nullptr) {
  const ffd_mesh* mesh = &mesh_in;
  const int d = mesh->simplex_dim;
  SetupInput in;
  in.d = d;
  in.din = mesh->dim_in;
  in.n = mesh->n_vertices;
  in.m = mesh->n_elements;
  in.V = mesh->V;
  in.T = mesh->T;
  in.rho = opt.rho;
  in.n_pinned = static_cast<int64_t>(pins.size());
  in.pinned_idx = pins.data();
  in.leaf_size = opt.leaf_size;
  in.elem_energy = elem_energy.empty() ? nullptr : elem_energy.data();
  in.tutte = tutte;
  in.device_top = dense_lib().ok;  // the large top fronts are factorised on the device
  if (con && con->n_rows > 0) {
    in.n_con = con->n_rows;
    in.con_ptr = con->row_ptr;
    in.con_col = con->col_idx;
    in.con_val = con->val;
  }
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
  h->prec = opt.precision;
  h->energy = opt.energy;
  h->h_mode = opt.h_mode;
  h->rho = opt.rho;
  h->n = S.n;
  h->m = S.m;
  h->nF = S.nF;
  h->nC = S.nC;
  h->pins_given = !pin_pos.empty();
  h->voff = voff;
  h->eoff = eoff;
  h->auto_pinned = auto_pinned;
  h->vnew2old = S.vnew2old;
  h->in_V.assign(mesh->V, mesh->V + mesh->n_vertices * mesh->dim_in);
  h->in_T.assign(mesh->T, mesh->T + mesh->n_elements * (d + 1));
  h->in_pins = pins;
  h->in_energy = elem_energy;
  h->in_leaf = opt.leaf_size;
  h->enew2old_h = S.enew2old;
  h->hstruct.reset(new Setup());
  h->hstruct->vnew2old = S.vnew2old;
  h->hstruct->vold2new = S.vold2new;
  h->hstruct->nodes = S.nodes;
  h->hstruct->children = S.children;
  h->hstruct->struct_idx = S.struct_idx;
  h->hstruct->panel_entries = S.panel_entries;
  if (in.n_con > 0) {
    h->ncon = in.n_con;
    h->in_con_ptr.assign(in.con_ptr, in.con_ptr + in.n_con + 1);
    h->in_con_col.assign(in.con_col, in.con_col + in.con_ptr[in.n_con]);
    h->in_con_val.assign(in.con_val, in.con_val + in.con_ptr[in.n_con]);
    h->con_ptr_h = S.con_ptr;
    h->con_col_h = S.con_col;
    h->con_val_h = S.con_val;
    h->con_gamma = S.con_gamma;
    h->ncon_rows = static_cast<int64_t>(S.cont_rows.size());
  }
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
  {
    if (elem_energy.empty()) {
      h->segs.push_back(ffd_ctx::Seg{0, m, opt.energy, 0});
    } else {
      if (S.m_energy0 > 0) h->segs.push_back(ffd_ctx::Seg{0, S.m_energy0, 0, 0});
      if (S.m_energy0 < m) h->segs.push_back(ffd_ctx::Seg{S.m_energy0, m, 1, 0});
    }
    int64_t pmax = 0;
    for (auto& g : h->segs) pmax += (g.e1 - g.e0 + 63) / 64;
    set_local_block(h, 256);
    UP(h->alloc(&h->partials, static_cast<size_t>(std::max<int64_t>(pmax, 1)) * kNumPartials));
    UP(h->alloc(&h->partials2, static_cast<size_t>((pmax + kFinalizeRows - 1) / kFinalizeRows + 1) * kNumPartials));
  }
  UP(upload(h, &h->dt_ptr, S.dt_ptr));
  UP(upload(h, &h->dt_idx, S.dt_idx));
  UP(upload(h, &h->pin_ptr, S.pin_ptr));
  UP(upload(h, &h->pin_col, S.pin_col));
  UP(upload(h, &h->pin_val, S.pin_val));
  h->n_pin_val = S.pin_val.size();
  h->n_lcf_val = S.lcf_val.size();
  UP(upload(h, &h->av_ptr, S.av_ptr));
  UP(upload(h, &h->av_idx, S.av_idx));
  UP(upload(h, &h->lcf_ptr, S.lcf_ptr));
  UP(upload(h, &h->lcf_col, S.lcf_col));
  UP(upload(h, &h->lcf_val, S.lcf_val));
  UP(h->alloc(&h->hist_scratch, FFD_HIST_FIELDS));
  {
    // the first history buffer comes with the handle, so iterations can run
    // without allocating until it fills
    const ffd_status hs = ensure_hist(h, 1, nullptr);
    if (hs != FFD_OK) return cleanup(hs);
  }
  {
    std::vector<int64_t> poff;
    const int64_t ptot = device_panel_offsets(S, poff);
    UP(h->alloc(&h->Prow, static_cast<size_t>(ptot)));
    UP(h->alloc(&h->Pcol, static_cast<size_t>(ptot)));
    UP(hipMemset(h->Prow, 0, static_cast<size_t>(ptot) * sizeof(double)));
    UP(hipMemset(h->Pcol, 0, static_cast<size_t>(ptot) * sizeof(double)));
    const ffd_status pst = upload_host_panels(h, S, poff, ptot, nullptr);
    if (pst != FFD_OK) return cleanup(pst);
    decltype(S.panel_f)().swap(S.panel_f);
    h->hpoff = poff;
    h->hnodes = S.nodes;
    h->hlevels = S.level_nodes;
    h->hparent.assign(S.nodes.size(), -1);
    for (size_t i = 0; i < S.children.size(); ++i)
      for (int32_t ch : S.children[i]) h->hparent[ch] = static_cast<int32_t>(i);
    h->solve_top = static_cast<int>(S.level_nodes.size());
    if (build_solve_schedule(h) != FFD_OK) return cleanup(FFD_ERR_OUT_OF_MEMORY);
  }
  UP(upload(h, &h->sidx, S.struct_idx));
  UP(upload(h, &h->pull_ptr, S.pull_ptr));
  UP(upload(h, &h->pull_idx, S.pull_idx));
  if (h->pins_given) UP(hipMemcpy(h->xC, pin_pos.data(), pin_pos.size() * sizeof(double), hipMemcpyHostToDevice));
  if (h->ncon > 0) {
    const std::vector<double> crhs(con->rhs, con->rhs + h->ncon * d);
    UP(upload(h, &h->con_ptr, S.con_ptr));
    UP(upload(h, &h->con_col, S.con_col));
    UP(upload(h, &h->con_val, S.con_val));
    UP(upload(h, &h->cont_rows, S.cont_rows));
    UP(upload(h, &h->cont_ptr, S.cont_ptr));
    UP(upload(h, &h->cont_con, S.cont_con));
    UP(upload(h, &h->cont_val, S.cont_val));
    UP(upload(h, &h->con_c, crhs));
    UP(h->alloc(&h->con_cp, static_cast<size_t>(h->ncon) * d));
    UP(h->alloc(&h->con_t, static_cast<size_t>(h->ncon) * d));
    UP(h->alloc(&h->con_lam, static_cast<size_t>(h->ncon) * d));
    UP(h->alloc(&h->con_Z, static_cast<size_t>(h->ncon) * static_cast<size_t>(std::max<int64_t>(S.nF, 1))));
    UP(h->alloc(&h->con_Sinv, static_cast<size_t>(h->ncon) * h->ncon));
    UP(h->alloc(&h->con_tmp, static_cast<size_t>(n) * d));
  }
  UP(hipDeviceSynchronize());
#undef UP
  if (in.device_top) {
    const ffd_status fst = device_factor_top(h, S, nullptr);
    if (fst != FFD_OK) return cleanup(fst);
  }
  if (h->ncon > 0) {
    const ffd_status cst = prepare_constraints(h, nullptr);
    if (cst != FFD_OK) return cleanup(cst);
  }
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

}  // namespace
