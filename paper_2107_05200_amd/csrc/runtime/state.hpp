// Refactorisation after a penalty rescaling event, the history buffer, state
// slots (checkpoints) and the adjoint launch helpers.  Part of the single
// translation unit capi.hip.
#pragma once

#include "devfactor.hpp"

namespace {

// Rebuilds the factor of L = G^T M G for per-element penalties mu_dev_order
// (device element order; nullptr: rho w_e) from the kept set-up input and
// structure (the ordering and the factor structure do not depend on the
// penalties; the result is checked against them) and writes the new panels
// and pinned-coupling values into the existing buffers.  Synchronous.
ffd_status refactor(ffd_ctx* h, const std::vector<double>* mu_dev_order, hipStream_t s) {
  std::vector<double> mu_in;
  SetupInput in;
  in.d = h->d;
  in.din = h->din;
  in.n = h->n;
  in.m = h->m;
  in.V = h->in_V.data();
  in.T = h->in_T.data();
  in.rho = h->rho;
  in.n_pinned = static_cast<int64_t>(h->in_pins.size());
  in.pinned_idx = h->in_pins.data();
  in.leaf_size = h->in_leaf;
  in.elem_energy = h->in_energy.empty() ? nullptr : h->in_energy.data();
  if (h->ncon > 0) {
    in.n_con = h->ncon;
    in.con_ptr = h->in_con_ptr.data();
    in.con_col = h->in_con_col.data();
    in.con_val = h->in_con_val.data();
  }
  if (mu_dev_order) {
    mu_in.resize(h->m);
    for (int64_t e = 0; e < h->m; ++e) mu_in[h->enew2old_h[e]] = (*mu_dev_order)[e];
    in.mu_elem = mu_in.data();
  }
  // the top fronts on the device when the dense libraries load; the ordering
  // and symbolic structure of the set-up are reused
  in.device_top = h->device_refactor && dense_lib().ok;
  in.structure = h->hstruct.get();
  Setup S;
  std::string err;
  const int st = build_setup(in, S, err);
  if (st != OK) return fail(static_cast<ffd_status>(st), err);
  bool same = S.nodes.size() == h->hnodes.size() && S.pin_val.size() == h->n_pin_val &&
              S.lcf_val.size() == h->n_lcf_val && S.panel_entries == h->info.panel_entries;
  for (size_t i = 0; same && i < S.nodes.size(); ++i)
    same = S.nodes[i].first == h->hnodes[i].first && S.nodes[i].c == h->hnodes[i].c && S.nodes[i].r == h->hnodes[i].r;
  std::vector<int64_t> poff;
  int64_t ptot = 0;
  if (same) {
    ptot = device_panel_offsets(S, poff);
    same = poff == h->hpoff;
  }
  if (!same) return fail(FFD_ERR_STATE, "the factor structure changed on refactorisation");
  // on the caller's stream, after its pending work; every node's segment is
  // rewritten (the top fronts by the device below), padding included
  HIP_TRY(hipStreamSynchronize(s));
  const ffd_status pst = upload_host_panels(h, S, poff, ptot, s);
  if (pst != FFD_OK) return pst;
  if (!S.pin_val.empty())
    HIP_TRY(hipMemcpyAsync(h->pin_val, S.pin_val.data(), S.pin_val.size() * sizeof(double), hipMemcpyHostToDevice, s));
  if (!S.lcf_val.empty())
    HIP_TRY(hipMemcpyAsync(h->lcf_val, S.lcf_val.data(), S.lcf_val.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (in.device_top) {
    const ffd_status st2 = device_factor_top(h, S, s);
    if (st2 != FFD_OK) return st2;
  }
  if (h->ncon > 0) {
    h->con_gamma = S.con_gamma;
    h->graph_valid = false;  // gamma is a kernel argument
    return prepare_constraints(h, s);
  }
  return FFD_OK;
}

// one rescaling event on the device, then the factor for the new penalties;
// glam (may be null): receives the corner vectors of the rescaled Lambda
ffd_status do_rescale(ffd_ctx* h, double rho_r, hipStream_t s, void* glam = nullptr) {
  if (!h->rho_e) {
    HIP_TRY(h->alloc(reinterpret_cast<char**>(&h->rho_e), h->rsize() * h->m));
    HIP_TRY(h->alloc(&h->mu_dev, static_cast<size_t>(h->m)));
  }
  if (!h->rescaled) {
    if (h->prec == 32) {
      std::vector<float> r(h->m, static_cast<float>(h->rho));
      HIP_TRY(hipMemcpyAsync(h->rho_e, r.data(), r.size() * sizeof(float), hipMemcpyHostToDevice, s));
      HIP_TRY(hipStreamSynchronize(s));
    } else {
      std::vector<double> r(h->m, h->rho);
      HIP_TRY(hipMemcpyAsync(h->rho_e, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    h->rescaled = true;
    h->graph_valid = false;
  }
  for (const auto& g : h->segs) SEG_CASES(launch_rescale, h, g, rho_r, glam, s)
  std::vector<double> mu(h->m);
  HIP_TRY(hipMemcpyAsync(mu.data(), h->mu_dev, mu.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return refactor(h, &mu, s);
}

// Tables of the per-problem termination test (on first use): each problem's
// element and vertex lists in device numbering (null lists for a plain
// handle: the identity) cut into pieces of at most kDiagPiece entries.
constexpr int32_t kDiagPiece = 4096;

ffd_status build_diag(ffd_ctx* h) {
  if (h->diag_pieces) return FFD_OK;
  const int64_t nprob = h->voff.empty() ? 1 : static_cast<int64_t>(h->voff.size()) - 1;
  std::vector<int32_t> elist, vlist, eptr(nprob + 1, 0), vptr(nprob + 1, 0);
  if (nprob > 1) {
    std::vector<int32_t> ep(h->m), vp(h->n);
    for (int64_t e = 0; e < h->m; ++e)
      ep[e] = static_cast<int32_t>(std::upper_bound(h->eoff.begin(), h->eoff.end(), h->enew2old_h[e]) - h->eoff.begin() - 1);
    for (int64_t v = 0; v < h->n; ++v)
      vp[v] = static_cast<int32_t>(std::upper_bound(h->voff.begin(), h->voff.end(), h->vnew2old[v]) - h->voff.begin() - 1);
    for (int64_t e = 0; e < h->m; ++e) ++eptr[ep[e] + 1];
    for (int64_t v = 0; v < h->n; ++v) ++vptr[vp[v] + 1];
    for (int64_t c = 0; c < nprob; ++c) {
      eptr[c + 1] += eptr[c];
      vptr[c + 1] += vptr[c];
    }
    elist.resize(h->m);
    vlist.resize(h->n);
    std::vector<int32_t> fe(eptr.begin(), eptr.end() - 1), fv(vptr.begin(), vptr.end() - 1);
    for (int64_t e = 0; e < h->m; ++e) elist[fe[ep[e]]++] = static_cast<int32_t>(e);
    for (int64_t v = 0; v < h->n; ++v) vlist[fv[vp[v]]++] = static_cast<int32_t>(v);
  } else {
    eptr[1] = static_cast<int32_t>(h->m);
    vptr[1] = static_cast<int32_t>(h->n);
  }
  std::vector<DiagPiece> pieces;
  std::vector<int32_t> pptr{0};
  h->diag_m.assign(nprob, 0);
  for (int64_t c = 0; c < nprob; ++c) {
    for (int32_t q = eptr[c]; q < eptr[c + 1]; q += kDiagPiece)
      pieces.push_back(DiagPiece{0, q, std::min(q + kDiagPiece, eptr[c + 1]), 0});
    for (int32_t q = vptr[c]; q < vptr[c + 1]; q += kDiagPiece)
      pieces.push_back(DiagPiece{1, q, std::min(q + kDiagPiece, vptr[c + 1]), 0});
    pptr.push_back(static_cast<int32_t>(pieces.size()));
    h->diag_m[c] = eptr[c + 1] - eptr[c];
  }
  if (!elist.empty()) HIP_TRY(upload(h, &h->diag_elist, elist));
  if (!vlist.empty()) HIP_TRY(upload(h, &h->diag_vlist, vlist));
  HIP_TRY(upload(h, &h->diag_piece_ptr, pptr));
  HIP_TRY(h->alloc(&h->diag_part, pieces.size() * kDiagFields));
  HIP_TRY(h->alloc(&h->diag_out, static_cast<size_t>(nprob) * kDiagFields));
  HIP_TRY(upload(h, &h->diag_pieces, pieces));
  h->diag_npieces = static_cast<int32_t>(pieces.size());
  h->diag_nprob = static_cast<int32_t>(nprob);
  return FFD_OK;
}

template <int D, typename R>
void launch_diag(ffd_ctx* h, hipStream_t s) {
  hipLaunchKernelGGL((k_diag_pieces<D, R>), dim3(h->diag_npieces), dim3(kBlock), 0, s, h->diag_pieces,
                     h->diag_elist, h->diag_vlist, h->m, h->T, h->B64, static_cast<const R*>(h->w),
                     static_cast<R>(h->rho), static_cast<const R*>(h->rescaled ? h->rho_e : nullptr),
                     h->x[h->cur], h->x[1 - h->cur], static_cast<const R*>(h->U), static_cast<const R*>(h->P),
                     static_cast<const R*>(h->glam), h->av_ptr, h->av_idx, h->diag_part);
}

// Algorithm 2's termination test on the state as it stands (after the
// iteration and any rescaling of it; U and the corner vectors of Lambda in
// glam must be current): eq. primaldualthresholds and, with flip_free, no
// flipped element, for every problem with its own sqrt(d m).  Synchronises.
ffd_status check_termination(ffd_ctx* h, hipStream_t s, double eps_abs, double eps_rel, bool flip_free, bool* conv) {
  ffd_status st = build_diag(h);
  if (st != FFD_OK) return st;
  if (h->d == 2) {
    if (h->prec == 32) launch_diag<2, float>(h, s);
    else launch_diag<2, double>(h, s);
  } else {
    if (h->prec == 32) launch_diag<3, float>(h, s);
    else launch_diag<3, double>(h, s);
  }
  hipLaunchKernelGGL(k_diag_problems, dim3((h->diag_nprob + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     h->diag_piece_ptr, h->diag_nprob, h->diag_part, h->diag_out);
  HIP_TRY(hipGetLastError());
  std::vector<double> out(static_cast<size_t>(h->diag_nprob) * kDiagFields);
  HIP_TRY(hipMemcpyAsync(out.data(), h->diag_out, out.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  bool all = true;
  for (int32_t c = 0; c < h->diag_nprob && all; ++c) {
    const double* v = out.data() + static_cast<size_t>(c) * kDiagFields;
    const double base = eps_abs * std::sqrt(static_cast<double>(h->d) * static_cast<double>(h->diag_m[c]));
    const bool prim = std::sqrt(v[0]) < base + eps_rel * std::max(std::sqrt(v[2]), std::sqrt(v[3]));
    const bool dual = std::sqrt(v[1]) < base + eps_rel * std::sqrt(v[5]);
    all = prim && dual && (!flip_free || v[4] == 0.0);
  }
  *conv = all;
  return FFD_OK;
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


// ---------------------------------------------------------------------------
// adjoint helpers
// ---------------------------------------------------------------------------
struct SlotView {
  void *U, *P, *L, *gn, *g;
  double* x;
};

SlotView slot_view(ffd_ctx* h, char* base) {
  const size_t nU = h->d == 2 ? 2 : 9, nP = h->d == 2 ? 3 : 6, rs = h->rsize(), m = h->m, d = h->d;
  SlotView v;
  v.U = base;
  v.P = base + rs * m * nU;
  v.L = base + rs * m * (nU + nP);
  v.gn = base + rs * m * (nU + nP + d * d);
  v.g = base + rs * m * (nU + nP + d * d + 1);
  const size_t el = rs * m * h->slot_elem_entries();
  v.x = reinterpret_cast<double*>(base + ((el + 255) / 256) * 256);
  return v;
}

// Element state and map (U, P, Lambda, |grad f|^2, corner vectors, map):
// copies from slot `from` (nullptr: the live state) to slot `to` (nullptr:
// the live state) and, when `to2` is given, to that slot as well, all in one
// launch.
hipError_t copy_state3(ffd_ctx* h, char* from, char* to, char* to2, hipStream_t s) {
  const size_t nU = h->d == 2 ? 2 : 9, nP = h->d == 2 ? 3 : 6, rs = h->rsize(), m = h->m, d = h->d;
  auto parts = [&](char* slot, void* (&p)[6]) {
    if (!slot) {
      void* live[6] = {h->U, h->P, h->L, h->gn, h->g, h->x[h->cur]};
      for (int i = 0; i < 6; ++i) p[i] = live[i];
    } else {
      const SlotView v = slot_view(h, slot);
      void* saved[6] = {v.U, v.P, v.L, v.gn, v.g, v.x};
      for (int i = 0; i < 6; ++i) p[i] = saved[i];
    }
  };
  const size_t bytes[6] = {rs * m * nU, rs * m * nP, rs * m * d * d, rs * m, rs * m * (d + 1) * d,
                           sizeof(double) * h->n * d};
  void *src[6], *dst[6], *dst2[6];
  parts(from, src);
  parts(to, dst);
  if (to2) parts(to2, dst2);
  CopyJobs J{};
  size_t most = 0;
  for (int i = 0; i < 6; ++i) {
    if (bytes[i] % 4 != 0) return hipErrorInvalidValue;  // the copy kernel moves 4-byte words
    J.src[J.n] = static_cast<const char*>(src[i]);
    J.dst[J.n] = static_cast<char*>(dst[i]);
    J.bytes[J.n++] = static_cast<int64_t>(bytes[i]);
    if (to2) {
      J.src[J.n] = static_cast<const char*>(src[i]);
      J.dst[J.n] = static_cast<char*>(dst2[i]);
      J.bytes[J.n++] = static_cast<int64_t>(bytes[i]);
    }
    most = std::max(most, bytes[i]);
  }
  const int64_t blocks = std::min<int64_t>(2048, std::max<int64_t>(1, static_cast<int64_t>(most / 16 + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_copy_jobs, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, J);
  return hipGetLastError();
}

hipError_t save_state(ffd_ctx* h, char* slot, hipStream_t s) { return copy_state3(h, nullptr, slot, nullptr, s); }
hipError_t load_state(ffd_ctx* h, char* slot, hipStream_t s) { return copy_state3(h, slot, nullptr, nullptr, s); }

template <int D, typename R, int E>
void launch_adj_seed(ffd_ctx* h, const ffd_ctx::Seg& g, const void* Pbar_ext, int energy_loss, hipStream_t s) {
  hipLaunchKernelGGL((k_adj_seed<D, R, E>), dim3(nblk(g.e1 - g.e0)), dim3(kBlock), 0, s, h->m, g.e0, g.e1,
                     static_cast<const R*>(h->P),
                     static_cast<const R*>(h->w), energy_loss, static_cast<const R*>(Pbar_ext), h->enew2old_d,
                     h->Ubar, h->Pbar, h->Lbar, h->Bbar, h->wbar);
}

template <int D, typename R, int E>
void launch_adj_local(ffd_ctx* h, const ffd_ctx::Seg& g, const SlotView& prev, const double* x, hipStream_t s) {
  hipLaunchKernelGGL((k_adj_local<D, R, E>), dim3(nblk(g.e1 - g.e0)), dim3(kBlock), 0, s, h->m, g.e0, g.e1, h->T,
                     static_cast<const R*>(h->B), h->B64, static_cast<R>(h->rho), x, static_cast<const R*>(prev.U),
                     static_cast<const R*>(prev.P), static_cast<const R*>(prev.L), h->Ubar, h->Pbar, h->Lbar, h->Bbar,
                     h->gadj);
}

template <int D, typename R, int E>
void launch_adj_wstep(ffd_ctx* h, const SlotView& prev, const double* x, hipStream_t s) {
  hipLaunchKernelGGL((k_adj_wstep<D, R>), dim3(nblk(h->m)), dim3(kBlock), 0, s, h->m, h->T, h->B64,
                     static_cast<const R*>(h->w), static_cast<R>(h->rho), x, h->lam, static_cast<const R*>(prev.U),
                     static_cast<const R*>(prev.P), static_cast<const R*>(prev.L), h->Ubar, h->Pbar, h->Lbar, h->Bbar,
                     h->wbar);
}

template <int D, typename R, int E>
void launch_adj_vbar(ffd_ctx* h, hipStream_t s) {
  hipLaunchKernelGGL((k_adj_vbar<D, R>), dim3(nblk(h->m)), dim3(kBlock), 0, s, h->m, h->B64,
                     static_cast<const R*>(h->w), h->Bbar, h->wbar, h->gadj);
}

#define ADJ_DISPATCH(FN, ...)                                                        \
  do {                                                                               \
    switch (h->d * 100 + h->prec + h->energy) {                                      \
      case 232: FN<2, float, 0>(__VA_ARGS__); break;                                 \
      case 233: FN<2, float, 1>(__VA_ARGS__); break;                                 \
      case 264: FN<2, double, 0>(__VA_ARGS__); break;                                \
      case 265: FN<2, double, 1>(__VA_ARGS__); break;                                \
      case 332: FN<3, float, 0>(__VA_ARGS__); break;                                 \
      case 333: FN<3, float, 1>(__VA_ARGS__); break;                                 \
      case 364: FN<3, double, 0>(__VA_ARGS__); break;                                \
      case 365: FN<3, double, 1>(__VA_ARGS__); break;                                \
    }                                                                                \
  } while (0)

}  // namespace
