// Launch helpers of one iteration of Algorithm 1 (dispatch on dimension,
// precision and energy), the level-by-level solve passes with their stream
// groups, the constraint terms of the W-step and one_iteration itself.
// Part of the single translation unit capi.hip.
#pragma once

#include "context.hpp"

namespace {

// --------------------------------------------------------------------------
// launch helpers (dispatch on d, precision, energy)
// --------------------------------------------------------------------------

template <int D, typename R, int E>
void launch_init(ffd_ctx* h, const ffd_ctx::Seg& g, hipStream_t s) {
  hipLaunchKernelGGL((k_init<D, R, E>), dim3(nblk(g.e1 - g.e0)), dim3(kBlock), 0, s, h->m, g.e0, g.e1, h->T, h->B64,
                     static_cast<const R*>(h->B), static_cast<const R*>(h->w), static_cast<R>(h->rho), h->x[h->cur],
                     static_cast<R*>(h->U), static_cast<R*>(h->P), static_cast<R*>(h->L), static_cast<R*>(h->gn),
                     static_cast<R*>(h->g));
}

template <int D, typename R, int E>
void launch_prepare(ffd_ctx* h, const ffd_ctx::Seg& g, hipStream_t s) {
  hipLaunchKernelGGL((k_prepare<D, R, E>), dim3(nblk(g.e1 - g.e0)), dim3(kBlock), 0, s, h->m, g.e0, g.e1,
                     static_cast<const R*>(h->B), static_cast<const R*>(h->w), static_cast<R>(h->rho),
                     static_cast<const R*>(h->rescaled ? h->rho_e : nullptr), static_cast<const R*>(h->U),
                     static_cast<const R*>(h->P),
                     static_cast<const R*>(h->L), static_cast<R*>(h->gn), static_cast<R*>(h->g));
}

template <int D, typename R, int E>
void launch_rescale(ffd_ctx* h, const ffd_ctx::Seg& g, double rho_r, void* glam, hipStream_t s) {
  hipLaunchKernelGGL((k_rescale<D, R, E>), dim3(nblk(g.e1 - g.e0)), dim3(kBlock), 0, s, h->m, g.e0, g.e1, h->T,
                     static_cast<const R*>(h->B), static_cast<const R*>(h->w), static_cast<R*>(h->rho_e),
                     h->x[h->cur], h->x[1 - h->cur], static_cast<const R*>(h->U), static_cast<const R*>(h->P),
                     static_cast<R*>(h->L), static_cast<const R*>(h->gn), static_cast<R*>(h->g), rho_r, h->mu_dev,
                     static_cast<R*>(glam));
}

template <int D, typename R, int E, int BS, bool PROX, bool DIAG>
void launch_local_k(ffd_ctx* h, const ffd_ctx::Seg& g, const double* xnew, const double* xold, int store_u,
                    void* glam, hipStream_t s) {
  hipLaunchKernelGGL((k_local<D, R, E, BS, PROX, DIAG>), dim3(static_cast<unsigned>((g.e1 - g.e0 + BS - 1) / BS)),
                     dim3(BS), 0, s, h->m, g.e0, g.e1, h->T, static_cast<const R*>(h->B), static_cast<const R*>(h->w),
                     static_cast<R>(h->rho), static_cast<const R*>(h->rescaled ? h->rho_e : nullptr), store_u, xnew,
                     xold, static_cast<R*>(h->U), static_cast<R*>(h->P), static_cast<R*>(h->L),
                     static_cast<R*>(h->gn), static_cast<R*>(h->g), h->partials + g.pb0 * kNumPartials,
                     static_cast<R*>(glam));
}

template <int D, typename R, int E, int BS>
void launch_local_bs(ffd_ctx* h, const ffd_ctx::Seg& g, const double* xnew, const double* xold, int store_u,
                     void* glam, hipStream_t s) {
  if (h->h_mode == 1) {
    if (glam) launch_local_k<D, R, E, BS, true, true>(h, g, xnew, xold, store_u, glam, s);
    else launch_local_k<D, R, E, BS, true, false>(h, g, xnew, xold, store_u, glam, s);
  } else {
    if (glam) launch_local_k<D, R, E, BS, false, true>(h, g, xnew, xold, store_u, glam, s);
    else launch_local_k<D, R, E, BS, false, false>(h, g, xnew, xold, store_u, glam, s);
  }
}

template <int D, typename R, int E>
void launch_local(ffd_ctx* h, const ffd_ctx::Seg& g, const double* xnew, const double* xold, int store_u,
                  void* glam, hipStream_t s) {
  if (h->local_bs == 64) launch_local_bs<D, R, E, 64>(h, g, xnew, xold, store_u, glam, s);
  else if (h->local_bs == 128) launch_local_bs<D, R, E, 128>(h, g, xnew, xold, store_u, glam, s);
  else launch_local_bs<D, R, E, 256>(h, g, xnew, xold, store_u, glam, s);
}

// partial-sum block offsets of the energy ranges for the local-step block size
void set_local_block(ffd_ctx* h, int bs) {
  h->graph_valid = false;
  h->local_bs = bs;
  int64_t pb = 0;
  for (auto& g : h->segs) {
    g.pb0 = pb;
    pb += (g.e1 - g.e0 + bs - 1) / bs;
  }
  h->nparts = pb;
}

template <int D, typename R, int LPR>
void launch_wrhs_l(ffd_ctx* h, double* xnew, hipStream_t s) {
  hipLaunchKernelGGL((k_wrhs<D, R, LPR>), dim3(nblk(LPR * h->n)), dim3(kBlock), 0, s, h->nF, h->n, h->dt_ptr,
                     h->dt_idx, static_cast<const R*>(h->g), h->pin_ptr, h->pin_col, h->pin_val, h->xC, h->b, xnew);
}

template <int D, typename R>
void launch_wrhs(ffd_ctx* h, double* xnew, hipStream_t s) {
  if (h->wrhs_lpr == 2) launch_wrhs_l<D, R, 2>(h, xnew, s);
  else if (h->wrhs_lpr == 8) launch_wrhs_l<D, R, 8>(h, xnew, s);
  else launch_wrhs_l<D, R, 4>(h, xnew, s);
}

template <int D, int OPT, int NW>
void launch_fwd_block(ffd_ctx* h, const LevelRun& r, const SolveTask* tasks, const double* b, hipStream_t s) {
  hipLaunchKernelGGL((k_solve_fwd<D, OPT, NW>), dim3(r.nt), dim3(NW * 64), 0, s, tasks, h->Pcol, h->pull_ptr,
                     h->pull_idx, b, h->y, h->ub, h->fpart);
}

inline const int32_t* bwd_sidx(const ffd_ctx* h) { return h->sidx_coded ? h->sidx_def : h->sidx; }

template <int D, int OPT, int NW>
void launch_bwd_block(ffd_ctx* h, const LevelRun& r, const SolveTask* tasks, double* x, hipStream_t s) {
  const int grid = r.nt + (r.ny + r.nx + NW - 1) / NW;
  hipLaunchKernelGGL((k_solve_bwd<D, OPT, NW>), dim3(grid), dim3(NW * 64), 0, s, tasks, r.nt, h->Prow, bwd_sidx(h),
                     h->y, x, h->solve_part, h->yred + r.y0, r.ny, h->fpart, h->xred + r.x0, r.nx, h->solve_part);
}

template <int D, int OPT>
void launch_fwd_opt(ffd_ctx* h, const LevelRun& r, const SolveTask* tasks, const double* b, hipStream_t s) {
  if (r.mode == 1)
    hipLaunchKernelGGL((k_solve_fwd_wave<D, OPT>), dim3((r.nt + 3) / 4), dim3(kBlock), 0, s, tasks, r.nt, h->Pcol,
                       h->pull_ptr, h->pull_idx, b, h->y, h->ub);
  else if (r.nw == 16)
    launch_fwd_block<D, OPT, 16>(h, r, tasks, b, s);
  else if (r.nw == 8)
    launch_fwd_block<D, OPT, 8>(h, r, tasks, b, s);
  else
    launch_fwd_block<D, OPT, 4>(h, r, tasks, b, s);
}

template <int D, int OPT>
void launch_bwd_opt(ffd_ctx* h, const LevelRun& r, const SolveTask* tasks, double* x, hipStream_t s) {
  if (r.mode == 1)
    hipLaunchKernelGGL((k_solve_bwd_wave<D, OPT>), dim3((r.nt + r.ny + r.nx + 3) / 4), dim3(kBlock), 0, s, tasks,
                       r.nt, h->Prow, bwd_sidx(h), h->y, x, h->yred + r.y0, r.ny, h->fpart, h->xred + r.x0, r.nx,
                       h->solve_part);
  else if (r.nw == 16)
    launch_bwd_block<D, OPT, 16>(h, r, tasks, x, s);
  else if (r.nw == 8)
    launch_bwd_block<D, OPT, 8>(h, r, tasks, x, s);
  else
    launch_bwd_block<D, OPT, 4>(h, r, tasks, x, s);
}

// reduce: add the split partials now (otherwise a backward launch adds them)
template <int D>
void launch_fwd_level(ffd_ctx* h, const LevelRun& r, const double* b, hipStream_t s, bool reduce) {
  const SolveTask* tasks = h->tasks_fwd + r.t0;
  if (r.nt > 0) {
    if (r.opt == 16) launch_fwd_opt<D, 16>(h, r, tasks, b, s);
    else if (r.opt == 32) launch_fwd_opt<D, 32>(h, r, tasks, b, s);
    else launch_fwd_opt<D, 64>(h, r, tasks, b, s);
  }
  if (reduce && r.nr > 0)
    hipLaunchKernelGGL((k_solve_fwd_reduce<D>), dim3((r.nr + 3) / 4), dim3(kBlock), 0, s, h->red_fwd + r.r0, r.nr,
                       h->pull_ptr, h->pull_idx, h->y, h->ub, h->fpart);
}

template <int D>
void launch_bwd_level(ffd_ctx* h, const LevelRun& r, double* x, hipStream_t s) {
  const SolveTask* tasks = h->tasks_bwd + r.t0;
  if (r.nt > 0 || r.ny > 0 || r.nx > 0) {
    if (r.opt == 16) launch_bwd_opt<D, 16>(h, r, tasks, x, s);
    else if (r.opt == 32) launch_bwd_opt<D, 32>(h, r, tasks, x, s);
    else launch_bwd_opt<D, 64>(h, r, tasks, x, s);
  }
  if (r.nr > 0 && r.reduce_now)  // otherwise the next backward launch adds them
    hipLaunchKernelGGL((k_solve_bwd_reduce<D>), dim3((r.nr + 3) / 4), dim3(kBlock), 0, s, h->red_bwd + r.r0, r.nr, x,
                       h->solve_part);
}

// stream of group g (group 0 and the top levels run on the caller's stream)
inline hipStream_t group_stream(ffd_ctx* h, int g, hipStream_t s) { return g == 0 ? s : h->wstreams[g - 1]; }

template <int D>
void launch_solve_fwd(ffd_ctx* h, const double* b, hipStream_t s) {
  const int G = h->solve_groups, top = h->solve_top;
  if (G > 1) {
    (void)hipEventRecord(h->fork_ev[0], s);
    for (int g = 1; g < G; ++g) (void)hipStreamWaitEvent(h->wstreams[g - 1], h->fork_ev[0], 0);
  }
  const int nlev = static_cast<int>(h->hlevels.size());
  for (int l = 0; l < top; ++l)
    for (int g = 0; g < G; ++g)
      launch_fwd_level<D>(h, h->grun_fwd[g][l], b, group_stream(h, g, s), h->grun_fwd[g][l].reduce_now);
  if (G > 1)
    for (int g = 1; g < G; ++g) {
      (void)hipEventRecord(h->join_ev[0][g], h->wstreams[g - 1]);
      (void)hipStreamWaitEvent(s, h->join_ev[0][g], 0);
    }
  for (int l = top; l < nlev; ++l) launch_fwd_level<D>(h, h->grun_fwd[G][l], b, s, h->grun_fwd[G][l].reduce_now);
}

template <int D>
void launch_solve_bwd(ffd_ctx* h, double* x, hipStream_t s) {
  const int G = h->solve_groups, top = h->solve_top;
  const int nlev = static_cast<int>(h->hlevels.size());
  for (int l = nlev - 1; l >= top; --l) launch_bwd_level<D>(h, h->grun_bwd[G][l], x, s);
  if (G > 1) {
    (void)hipEventRecord(h->fork_ev[1], s);
    for (int g = 1; g < G; ++g) (void)hipStreamWaitEvent(h->wstreams[g - 1], h->fork_ev[1], 0);
  }
  for (int l = top - 1; l >= 0; --l)
    for (int g = 0; g < G; ++g) launch_bwd_level<D>(h, h->grun_bwd[g][l], x, group_stream(h, g, s));
  if (G > 1)
    for (int g = 1; g < G; ++g) {
      (void)hipEventRecord(h->join_ev[1][g], h->wstreams[g - 1]);
      (void)hipStreamWaitEvent(s, h->join_ev[1][g], 0);
    }
}

template <int D>
void launch_solve(ffd_ctx* h, const double* b, double* x, hipStream_t s) {
  launch_solve_fwd<D>(h, b, s);
  launch_solve_bwd<D>(h, x, s);
}

#define SEG_CASES(FN, ...)                                                  \
  switch (h->d * 100 + h->prec + g.energy) {                                \
    case 232: FN<2, float, 0>(__VA_ARGS__); break;                          \
    case 233: FN<2, float, 1>(__VA_ARGS__); break;                          \
    case 264: FN<2, double, 0>(__VA_ARGS__); break;                         \
    case 265: FN<2, double, 1>(__VA_ARGS__); break;                         \
    case 332: FN<3, float, 0>(__VA_ARGS__); break;                          \
    case 333: FN<3, float, 1>(__VA_ARGS__); break;                          \
    case 364: FN<3, double, 0>(__VA_ARGS__); break;                         \
    case 365: FN<3, double, 1>(__VA_ARGS__); break;                         \
  }

void do_init(ffd_ctx* h, hipStream_t s) {
  for (const auto& g : h->segs) SEG_CASES(launch_init, h, g, s)
}

void do_prepare(ffd_ctx* h, hipStream_t s) {
  for (const auto& g : h->segs) SEG_CASES(launch_prepare, h, g, s)
}

void do_local(ffd_ctx* h, const double* xnew, const double* xold, int store_u, hipStream_t s,
              void* glam = nullptr) {
  for (const auto& g : h->segs) SEG_CASES(launch_local, h, g, xnew, xold, store_u, glam, s)
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

// the constraint terms of the W-step: c' = c - A_C x_C and b += gamma A_F^T c'
// before the solve, x_F -= Z S^{-1} (A x - c) after it
template <int D>
void con_before_solve_d(ffd_ctx* h, hipStream_t s) {
  hipLaunchKernelGGL(k_con_shift<D>, dim3(nblk(h->ncon)), dim3(kBlock), 0, s, h->ncon, h->nF, h->con_ptr,
                     h->con_col, h->con_val, h->con_c, h->xC, h->con_cp);
  hipLaunchKernelGGL(k_con_addq<D>, dim3(nblk(h->ncon_rows)), dim3(kBlock), 0, s, h->ncon_rows, h->cont_rows,
                     h->cont_ptr, h->cont_con, h->cont_val, h->con_gamma, h->con_cp, h->b);
}
template <int D>
void con_after_solve_d(ffd_ctx* h, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_con_resid<D>, dim3(nblk(h->ncon)), dim3(kBlock), 0, s, h->ncon, h->con_ptr, h->con_col,
                     h->con_val, h->con_c, x, h->con_t);
  hipLaunchKernelGGL(k_con_lambda<D>, dim3(nblk(h->ncon)), dim3(kBlock), 0, s, h->ncon, h->con_Sinv, h->con_t,
                     h->con_lam);
  if (h->nF > 0)
    hipLaunchKernelGGL(k_con_correct<D>, dim3(nblk(h->nF)), dim3(kBlock), 0, s, h->nF, h->ncon, h->con_Z,
                       h->con_lam, x);
}
void con_before_solve(ffd_ctx* h, hipStream_t s) {
  if (h->d == 2) con_before_solve_d<2>(h, s);
  else con_before_solve_d<3>(h, s);
}
void con_after_solve(ffd_ctx* h, double* x, hipStream_t s) {
  if (h->d == 2) con_after_solve_d<2>(h, x, s);
  else con_after_solve_d<3>(h, x, s);
}

// Z = L~^{-1} A_F^T by solves of D columns at a time, S = A_F Z on the device,
// S^{-1} on the host (Cholesky with a relative pivot floor: dependent rows
// are an error).  Synchronous; uses b and con_tmp as scratch.
ffd_status prepare_constraints(ffd_ctx* h, hipStream_t s) {
  const int d = h->d;
  const int64_t nF = h->nF, nc = h->ncon;
  std::vector<double> rhs(static_cast<size_t>(nF) * d, 0.0);
  for (int64_t a0 = 0; a0 < nc; a0 += d) {
    for (int k = 0; k < d && a0 + k < nc; ++k)
      for (int64_t q = h->con_ptr_h[a0 + k]; q < h->con_ptr_h[a0 + k + 1]; ++q)
        if (h->con_col_h[q] < nF) rhs[static_cast<size_t>(h->con_col_h[q]) * d + k] = h->con_val_h[q];
    HIP_TRY(hipMemcpyAsync(h->b, rhs.data(), rhs.size() * sizeof(double), hipMemcpyHostToDevice, s));
    do_solve(h, h->b, h->con_tmp, s);
    hipLaunchKernelGGL((d == 2 ? k_con_zcols<2> : k_con_zcols<3>), dim3(nblk(nF)), dim3(kBlock), 0, s, nF, nc, a0,
                       h->con_tmp, h->con_Z);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    for (int k = 0; k < d && a0 + k < nc; ++k)
      for (int64_t q = h->con_ptr_h[a0 + k]; q < h->con_ptr_h[a0 + k + 1]; ++q)
        if (h->con_col_h[q] < nF) rhs[static_cast<size_t>(h->con_col_h[q]) * d + k] = 0.0;
  }
  hipLaunchKernelGGL(k_con_gram, dim3(nblk(nc * nc)), dim3(kBlock), 0, s, nF, nc, h->con_ptr, h->con_col, h->con_val,
                     h->con_Z, h->con_Sinv);
  HIP_TRY(hipGetLastError());
  std::vector<double> S(static_cast<size_t>(nc) * nc), X(static_cast<size_t>(nc) * nc, 0.0);
  HIP_TRY(hipMemcpyAsync(S.data(), h->con_Sinv, S.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  // symmetrise, then S = C C^T (C lower, row-major in place)
  double dmax = 0.0;
  for (int64_t i = 0; i < nc; ++i) {
    for (int64_t j = 0; j < i; ++j) S[i * nc + j] = S[j * nc + i] = 0.5 * (S[i * nc + j] + S[j * nc + i]);
    dmax = std::max(dmax, S[i * nc + i]);
  }
  for (int64_t j = 0; j < nc; ++j) {
    double dj = S[j * nc + j];
    for (int64_t l = 0; l < j; ++l) dj -= S[j * nc + l] * S[j * nc + l];
    if (!(dj > 1e-12 * dmax) || !std::isfinite(dj))
      return fail(FFD_ERR_SINGULAR_SYSTEM, "constraint row " + std::to_string(j) +
                                               " depends on the others (with the pins): the constraint system is singular");
    dj = std::sqrt(dj);
    S[j * nc + j] = dj;
    for (int64_t i = j + 1; i < nc; ++i) {
      double t = S[i * nc + j];
      for (int64_t l = 0; l < j; ++l) t -= S[i * nc + l] * S[j * nc + l];
      S[i * nc + j] = t / dj;
    }
  }
  // X = C^{-1} (lower), then S^{-1} = X^T X
  for (int64_t j = 0; j < nc; ++j) {
    X[j * nc + j] = 1.0 / S[j * nc + j];
    for (int64_t i = j + 1; i < nc; ++i) {
      double t = 0.0;
      for (int64_t l = j; l < i; ++l) t += S[i * nc + l] * X[l * nc + j];
      X[i * nc + j] = -t / S[i * nc + i];
    }
  }
  std::vector<double> Si(static_cast<size_t>(nc) * nc);
  for (int64_t i = 0; i < nc; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      double t = 0.0;
      for (int64_t l = i; l < nc; ++l) t += X[l * nc + i] * X[l * nc + j];
      Si[i * nc + j] = Si[j * nc + i] = t;
    }
  HIP_TRY(hipMemcpyAsync(h->con_Sinv, Si.data(), Si.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return FFD_OK;
}

// one iteration of Algorithm 1; with ev != nullptr an event is recorded after
// each of the five phases
// store_u: write the rotation and |grad f|^2 of this iteration even where the
// next iteration does not read them (3D with h = 0); they are state outputs, so
// the last iteration of a call and every iteration whose state is saved store
// them (2D and h_mode 1 always store them)
// dev_k: the history record index comes from the device counter (graph capture)
// diag: also record |G^T Lambda| (history field 9; needs h->glam and h->gtl_part)
void one_iteration(ffd_ctx* h, hipStream_t s, hipEvent_t* ev, bool record = true, bool store_u = true,
                   bool dev_k = false, bool diag = false) {
  double* xold = h->x[h->cur];
  double* xnew = h->x[1 - h->cur];
  do_wrhs(h, xnew, s);
  if (h->ncon > 0) con_before_solve(h, s);
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
  if (h->ncon > 0) con_after_solve(h, xnew, s);
  if (ev) (void)hipEventRecord(ev[2], s);
  do_local(h, xnew, xold, store_u ? 1 : 0, s, diag ? h->glam : nullptr);
  if (ev) (void)hipEventRecord(ev[3], s);
  double* rec = dev_k ? h->hist : record ? h->hist + h->k * FFD_HIST_FIELDS : h->hist_scratch;
  int64_t* kd = dev_k ? h->k_dev : nullptr;
  const int nf = diag ? kNumPartials : kNumSums;  // the maxima exist on diagnostic iterations only
  if (h->nparts > 2 * kFinalizeRows) {
    const int64_t nb2 = (h->nparts + kFinalizeRows - 1) / kFinalizeRows;
    hipLaunchKernelGGL(k_partials_reduce, dim3(static_cast<unsigned>(nb2)), dim3(kBlock), 0, s, h->partials,
                       h->nparts, h->partials2, nf);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, h->partials2, nb2, rec, kd, FFD_HIST_FIELDS, nf);
  } else {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, h->partials, h->nparts, rec, kd, FFD_HIST_FIELDS,
                       nf);
  }
  if (diag && !dev_k) {
    const int64_t nb = (4 * h->n + kBlock - 1) / kBlock;
    if (h->d == 2) {
      if (h->prec == 32)
        hipLaunchKernelGGL((k_gtlam<2, float>), dim3(nb), dim3(kBlock), 0, s, h->n, h->av_ptr, h->av_idx,
                           static_cast<const float*>(h->glam), h->gtl_part);
      else
        hipLaunchKernelGGL((k_gtlam<2, double>), dim3(nb), dim3(kBlock), 0, s, h->n, h->av_ptr, h->av_idx,
                           static_cast<const double*>(h->glam), h->gtl_part);
    } else {
      if (h->prec == 32)
        hipLaunchKernelGGL((k_gtlam<3, float>), dim3(nb), dim3(kBlock), 0, s, h->n, h->av_ptr, h->av_idx,
                           static_cast<const float*>(h->glam), h->gtl_part);
      else
        hipLaunchKernelGGL((k_gtlam<3, double>), dim3(nb), dim3(kBlock), 0, s, h->n, h->av_ptr, h->av_idx,
                           static_cast<const double*>(h->glam), h->gtl_part);
    }
    hipLaunchKernelGGL(k_gtlam_finalize, dim3(1), dim3(kBlock), 0, s, h->gtl_part, nb, rec + 9);
  }
  if (ev) (void)hipEventRecord(ev[4], s);
  h->cur = 1 - h->cur;
  if (record) h->k += 1;
}

}  // namespace
