// Timing helpers of the autotuner and its cache key.  Part of the single
// translation unit capi.hip.
#pragma once

#include "graph.hpp"

namespace {

// time `iters` iterations (not recorded) and return the summed milliseconds of
// phase `phase` (0 right-hand side, 1+2 solve, 3 local step)
double time_phase(ffd_ctx* h, hipStream_t s, int phase, int iters) {
  const size_t need = static_cast<size_t>(iters) * 5 + 1;
  while (h->events.size() < need) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return 1e30;
    h->events.push_back(ev);
  }
  for (int it = 0; it < 2; ++it) one_iteration(h, s, nullptr, false, true);
  (void)hipEventRecord(h->events[0], s);
  for (int it = 0; it < iters; ++it) one_iteration(h, s, h->events.data() + 1 + static_cast<size_t>(it) * 5, false, true);
  if (hipEventSynchronize(h->events[need - 1]) != hipSuccess) return 1e30;
  double tot = 0.0;
  for (int it = 0; it < iters; ++it)
    for (int p = 0; p < 5; ++p) {
      const bool want = phase == 1 ? (p == 1 || p == 2) : p == phase;
      if (!want) continue;
      float ms = 0.f;
      const size_t i = 1 + static_cast<size_t>(it) * 5 + p;
      (void)hipEventElapsedTime(&ms, h->events[i - 1], h->events[i]);
      tot += ms;
    }
  return tot;
}

// milliseconds of one forward (or backward) solve pass on the current
// right-hand side, the smallest of `reps` timed passes after one untimed one
double time_solve_pass(ffd_ctx* h, hipStream_t s, bool fwd, int reps) {
  while (h->events.size() < 2) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return 1e30;
    h->events.push_back(ev);
  }
  double* xs = h->x[1 - h->cur];
  double best = 1e30;
  for (int r = 0; r <= reps; ++r) {
    (void)hipEventRecord(h->events[0], s);
    if (fwd) {
      if (h->d == 2) launch_solve_fwd<2>(h, h->b, s);
      else launch_solve_fwd<3>(h, h->b, s);
    } else {
      if (h->d == 2) launch_solve_bwd<2>(h, xs, s);
      else launch_solve_bwd<3>(h, xs, s);
    }
    (void)hipEventRecord(h->events[1], s);
    if (hipEventSynchronize(h->events[1]) != hipSuccess) return 1e30;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, h->events[0], h->events[1]);
    if (r > 0) best = std::min(best, static_cast<double>(ms));
  }
  return best;
}

std::string tune_key(ffd_ctx* h) {
  hipDeviceProp_t prop;
  std::string arch = hipGetDeviceProperties(&prop, h->dev) == hipSuccess ? prop.gcnArchName : "unknown";
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  int64_t mb = 1, nb = 1;
  while (mb < h->m) mb *= 2;
  while (nb < h->info.factor_nnz) nb *= 2;
  std::string energy = h->segs.size() > 1 ? "mixed" : std::to_string(h->segs.empty() ? 0 : h->segs[0].energy);
  return arch + "|d" + std::to_string(h->d) + "|e" + energy + "|p" + std::to_string(h->prec) + "|m" +
         std::to_string(mb) + "|nnz" + std::to_string(nb) + "|lv" + std::to_string(h->hlevels.size()) + "|h" +
         std::to_string(h->h_mode);
}

}  // namespace
