// Task lists of the level-scheduled triangular solves: output blocks per
// level, default and autotuned per-level configurations, XCD-aware task order,
// split inner ranges with their reductions, stream groups.  Part of the
// single translation unit capi.hip.
#pragma once

#include "launch.hpp"

namespace {

// Output blocks of one level of one pass: (node, first output, inner range).
struct OutBlock {
  int32_t node, out0, lo, hi;
};

std::vector<OutBlock> level_blocks(const ffd_ctx* h, const std::vector<int32_t>& lvl, bool fwd, int opt) {
  std::vector<OutBlock> obs;
  for (int32_t i : lvl) {
    const SolveNode& N = h->hnodes[i];
    const int nf = N.c + N.r;
    if (fwd) {
      for (int o0 = 0; o0 < nf; o0 += opt) obs.push_back(OutBlock{i, o0, 0, std::min(N.c, o0 + opt)});
    } else {
      for (int o0 = 0; o0 < N.c; o0 += opt) obs.push_back(OutBlock{i, o0, o0, nf});
    }
  }
  // longest inner ranges first: the blocks that take longest start first
  std::stable_sort(obs.begin(), obs.end(),
                   [](const OutBlock& a, const OutBlock& b) { return a.hi - a.lo > b.hi - b.lo; });
  return obs;
}

// Default configuration of a level: four-wave blocks of 64 outputs; a level
// with fewer than 512 blocks splits inner ranges into the largest chunks
// (4096 .. 256) that give it 512 tasks.
LevelCfg default_level_cfg(const ffd_ctx* h, const std::vector<int32_t>& lvl, bool fwd) {
  constexpr int64_t kMinTasks = 512;
  LevelCfg c;
  const std::vector<OutBlock> obs = level_blocks(h, lvl, fwd, 64);
  if (static_cast<int64_t>(obs.size()) >= kMinTasks) return c;
  c.chunk = 256;
  for (int64_t kc = 4096; kc >= 256; kc /= 2) {
    int64_t nt = 0;
    for (const OutBlock& o : obs) nt += (o.hi - o.lo + kc - 1) / kc;
    if (nt >= kMinTasks) {
      c.chunk = static_cast<int32_t>(kc);
      break;
    }
  }
  return c;
}

template <typename T_>
hipError_t upload_cap(ffd_ctx* h, T_** dst, size_t* cap, const std::vector<T_>& src) {
  if (src.size() > *cap) {
    if (*dst) {
      for (auto& a : h->allocs)
        if (a == *dst) a = nullptr;
      (void)hipFree(*dst);
      *dst = nullptr;
    }
    const size_t n = src.size() + src.size() / 4 + 16;
    hipError_t e = h->alloc(dst, n);
    if (e != hipSuccess) {
      *cap = 0;
      return e;
    }
    *cap = n;
  }
  if (src.empty()) return hipSuccess;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T_), hipMemcpyHostToDevice);
}

// worker streams (default priority) and fork / join events for g groups
hipError_t ensure_workers(ffd_ctx* h, int g) {
  g = std::min(g, 8);
  while (static_cast<int>(h->wstreams.size()) < g - 1) {
    hipStream_t w = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&w, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    h->wstreams.push_back(w);
  }
  for (int p = 0; p < 2; ++p) {
    if (!h->fork_ev[p]) {
      hipError_t e = hipEventCreateWithFlags(&h->fork_ev[p], hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    for (int i = 1; i < g; ++i)
      if (!h->join_ev[p][i]) {
        hipError_t e = hipEventCreateWithFlags(&h->join_ev[p][i], hipEventDisableTiming);
        if (e != hipSuccess) return e;
      }
  }
  return hipSuccess;
}

// Reorders the main tasks of one level run (from t0 on) so that the tasks of
// a node run on one XCD, whose L2 then serves the inner vector they all
// stage: blocks go to the 8 XCDs round-robin by index, so lane x of 8 takes
// block indices x, x + 8, ...  A node's tasks go to one lane in pieces of at
// most a lane's share (a level of one node still spreads over all eight),
// pieces onto the lane with the fewest tasks; each lane keeps the
// longest-first order; g tasks form a block (one wave each in wave mode);
// lanes are padded with empty tasks (no outputs).
void xcd_order(std::vector<SolveTask>& tasks, size_t t0, int g) {
  constexpr int X = 8;
  const size_t nt = tasks.size() - t0;
  if (nt < static_cast<size_t>(2 * X * g)) return;
  std::vector<std::vector<SolveTask>> byn;
  std::unordered_map<int64_t, size_t> slot_of;  // node (first row) -> its list
  for (size_t t = t0; t < tasks.size(); ++t) {
    const auto it = slot_of.emplace(tasks[t].first, byn.size());
    if (it.second) byn.emplace_back();
    byn[it.first->second].push_back(tasks[t]);
  }
  std::stable_sort(byn.begin(), byn.end(),
                   [](const std::vector<SolveTask>& a, const std::vector<SolveTask>& b) { return a.size() > b.size(); });
  const size_t cap = std::max<size_t>(g, (nt + X - 1) / X);
  std::vector<std::vector<SolveTask>> lane(X);
  for (const auto& nd : byn)
    for (size_t o = 0; o < nd.size(); o += cap) {
      size_t x = 0;
      for (size_t y2 = 1; y2 < X; ++y2)
        if (lane[y2].size() < lane[x].size()) x = y2;
      lane[x].insert(lane[x].end(), nd.begin() + o, nd.begin() + std::min(nd.size(), o + cap));
    }
  size_t groups = 0;
  for (auto& l : lane) {
    std::stable_sort(l.begin(), l.end(), [](const SolveTask& a, const SolveTask& b) { return a.hi - a.lo > b.hi - b.lo; });
    groups = std::max(groups, (l.size() + g - 1) / g);
  }
  SolveTask empty{};
  empty.slot = -1;
  tasks.resize(t0);
  for (size_t k = 0; k < groups; ++k)
    for (int x = 0; x < X; ++x)
      for (int u = 0; u < g; ++u) {
        const size_t i = k * g + u;
        tasks.push_back(i < lane[x].size() ? lane[x][i] : empty);
      }
}

// Builds the task lists of both passes from cfg_fwd / cfg_bwd (defaults for
// levels without one) and uploads them.  Waits for the device first: the
// task buffers may be in use by earlier launches.
ffd_status build_solve_schedule(ffd_ctx* h) {
  h->graph_valid = false;
  const size_t nlev = h->hlevels.size();
  if (h->cfg_fwd.size() != nlev || h->cfg_bwd.size() != nlev) {
    h->cfg_fwd.resize(nlev);
    h->cfg_bwd.resize(nlev);
    for (size_t l = 0; l < nlev; ++l) {
      h->cfg_fwd[l] = default_level_cfg(h, h->hlevels[l], true);
      h->cfg_bwd[l] = default_level_cfg(h, h->hlevels[l], false);
    }
  }
  auto task_of = [&](const OutBlock& o, bool fwd, int32_t lo, int32_t hi, int32_t slot, int32_t nk) {
    const SolveNode& N = h->hnodes[o.node];
    const int32_t nf = N.c + N.r;
    SolveTask t{};
    // the task's tile of the panel copy: base shifted so that output i sits
    // at pf + i + j * ld (outputs of one task never cross a tile)
    const int64_t tile = (o.out0 / kPanelTile) * kPanelTile, nout = fwd ? nf : N.c, nin = fwd ? N.c : nf;
    t.pf = h->hpoff[o.node] + tile * nin - tile;
    t.poff = N.poff;
    t.uoff = N.uoff;
    t.soff = N.soff;
    t.ld = static_cast<int32_t>(std::min<int64_t>(kPanelTile, nout - tile));
    t.first = N.first;
    t.c = N.c;
    t.nf = nf;
    t.out0 = o.out0;
    t.lo = lo;
    t.hi = hi;
    t.slot = slot;
    t.nk = nk;
    return t;
  };
  // groups of the forest below solve_top: whole subtrees, balanced greedily
  // by panel bytes (largest subtree first onto the lightest group)
  const int G = std::max(1, std::min(h->solve_groups, 1 + static_cast<int>(h->wstreams.size())));
  const int top = G > 1 ? std::max(0, std::min(h->solve_top, static_cast<int>(nlev))) : static_cast<int>(nlev);
  const int nn = static_cast<int>(h->hnodes.size());
  std::vector<int32_t> group(nn, G);
  if (G == 1) {
    std::fill(group.begin(), group.end(), 0);
  } else {
    std::vector<double> sub(nn, 0.0);
    for (int i = 0; i < nn; ++i) {  // postorder: children before parents
      const SolveNode& N = h->hnodes[i];
      sub[i] += static_cast<double>(N.c + N.r) * N.c;
      if (h->hparent[i] >= 0) sub[h->hparent[i]] += sub[i];
    }
    std::vector<int32_t> roots;
    for (int i = 0; i < nn; ++i)
      if (h->hnodes[i].level < top && (h->hparent[i] < 0 || h->hnodes[h->hparent[i]].level >= top)) roots.push_back(i);
    std::stable_sort(roots.begin(), roots.end(), [&](int32_t a, int32_t b) { return sub[a] > sub[b]; });
    std::vector<double> load(G, 0.0);
    for (int32_t r : roots) {
      const int g = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
      group[r] = g;
      load[g] += sub[r];
    }
    for (int i = nn - 1; i >= 0; --i)  // parents before children
      if (h->hnodes[i].level < top && group[i] == G) group[i] = group[h->hparent[i]];
  }
  std::vector<SolveTask> tf, tb, rf, rb;
  int64_t total_slots = 1;  // backward split partials: a region per level and group (a deferring
                            // level's partials are read by the next launch)
  int64_t fslots = 1;       // forward split partials: kept until the backward pass
  h->grun_fwd.assign(G + 1, std::vector<LevelRun>(nlev));
  h->grun_bwd.assign(G + 1, std::vector<LevelRun>(nlev));
  for (int g = 0; g <= G; ++g) {
    for (size_t l = 0; l < nlev; ++l) {
      if ((g < G) != (static_cast<int>(l) < top)) continue;
      std::vector<int32_t> nodes;
      for (int32_t i : h->hlevels[l])
        if (group[i] == g) nodes.push_back(i);
      if (nodes.empty()) continue;
      for (int pass = 0; pass < 2; ++pass) {
        const bool fwd = pass == 0;
        const LevelCfg& cfg = fwd ? h->cfg_fwd[l] : h->cfg_bwd[l];
        std::vector<SolveTask>& tasks = fwd ? tf : tb;
        std::vector<SolveTask>& red = fwd ? rf : rb;
        LevelRun& run = fwd ? h->grun_fwd[g][l] : h->grun_bwd[g][l];
        const std::vector<OutBlock> obs = level_blocks(h, nodes, fwd, cfg.opt);
        run.mode = cfg.mode;
        run.opt = cfg.opt;
        run.nw = cfg.nw;
        run.t0 = static_cast<int32_t>(tasks.size());
        run.r0 = static_cast<int32_t>(red.size());
        int32_t slots = 0;
        const int32_t base = static_cast<int32_t>(fwd ? fslots : total_slots);
        for (const OutBlock& o : obs) {
          const int64_t len = o.hi - o.lo;
          // forward: only blocks of y rows split (update rows feed the parents
          // within the pass and stay whole)
          const bool may_split =
              cfg.mode == 0 && cfg.chunk > 0 && (!fwd || !cfg.defer || o.out0 + cfg.opt <= h->hnodes[o.node].c);
          const int32_t nk = may_split ? static_cast<int32_t>((len + cfg.chunk - 1) / cfg.chunk) : 1;
          if (nk <= 1) {
            tasks.push_back(task_of(o, fwd, o.lo, o.hi, -1, 1));
            continue;
          }
          const int32_t b0 = base + slots;
          slots += nk;
          for (int32_t q = 0; q < nk; ++q)
            tasks.push_back(task_of(o, fwd, static_cast<int32_t>(o.lo + q * cfg.chunk),
                                    static_cast<int32_t>(std::min<int64_t>(o.hi, o.lo + static_cast<int64_t>(q + 1) * cfg.chunk)),
                                    b0 + q, nk));
          red.push_back(task_of(o, fwd, 0, cfg.opt, b0, nk));  // hi: outputs of the block
        }
        if (h->xcd_lanes) xcd_order(tasks, static_cast<size_t>(run.t0), cfg.mode == 1 ? 4 : 1);
        run.nt = static_cast<int32_t>(tasks.size()) - run.t0;
        run.nr = static_cast<int32_t>(red.size()) - run.r0;
        // a backward level defers to the next backward launch of its stream
        // (there is none after level 0, nor after the top group's lowest
        // level when the forest below runs on several streams)
        const bool bwd_defer = !fwd && cfg.defer && l >= 1 && (g < G || static_cast<int>(l) - 1 >= top) &&
                               run.nr > 0 && base + slots <= kDeferSlotLimit;
        run.reduce_now = fwd ? (!cfg.defer || l + 1 == nlev) : !bwd_defer;
        if (bwd_defer)
          for (int32_t q = 0; q < run.nr; ++q)
            if (red[run.r0 + q].nk > kDeferNkMax) run.reduce_now = true;
        if (fwd) fslots += slots;
        else total_slots += slots;
      }
    }
  }
  const int64_t max_slots = total_slots;
  // forward y-row reductions of level l run in the backward launch of level
  // l + 1 of the same stream group; those of the forest groups' level top - 1
  // in the top group's launch of level top (before the fork); the highest
  // level's in a launch of their own at the end of the forward pass
  std::vector<SolveTask> yr;
  auto attach = [&](LevelRun& br, int gsrc, size_t lsrc) {
    const LevelRun& fr = h->grun_fwd[gsrc][lsrc];
    if (fr.reduce_now) return;
    for (int32_t q = 0; q < fr.nr; ++q) yr.push_back(rf[fr.r0 + q]);
    br.ny += fr.nr;
  };
  for (int g = 0; g <= G; ++g)
    for (size_t l = 1; l < nlev; ++l) {
      if ((g < G) != (static_cast<int>(l) < top)) continue;
      LevelRun& br = h->grun_bwd[g][l];
      br.y0 = static_cast<int32_t>(yr.size());
      br.ny = 0;
      if (g == G && static_cast<int>(l) == top) {
        for (int gf = 0; gf < G; ++gf) attach(br, gf, l - 1);
      } else {
        attach(br, g, l - 1);
      }
    }
  // deferred backward reductions: appended to the next backward launch of
  // the same stream, whose structure lists read those rows from the partials
  std::vector<SolveTask> xr;
  std::vector<int32_t> coded;
  {
    const std::vector<int32_t>& sidx_h = h->hstruct->struct_idx;
    std::vector<int32_t> rowcode;
    for (int g = 0; g <= G; ++g)
      for (size_t l = 1; l < nlev; ++l) {
        if ((g < G) != (static_cast<int>(l) < top)) continue;
        const LevelRun& br = h->grun_bwd[g][l];
        if (br.reduce_now || br.nr == 0) continue;
        LevelRun& nx = h->grun_bwd[g][l - 1];
        nx.x0 = static_cast<int32_t>(xr.size());
        nx.nx = br.nr;
        if (coded.empty()) coded = sidx_h;
        if (rowcode.empty()) rowcode.assign(static_cast<size_t>(h->nF), 0);
        for (int32_t q = 0; q < br.nr; ++q) {
          const SolveTask& t = rb[br.r0 + q];
          xr.push_back(t);
          for (int32_t ln = 0; ln < t.hi && t.out0 + ln < t.c; ++ln)
            rowcode[t.first + t.out0 + ln] =
                -(1 + static_cast<int32_t>((static_cast<uint32_t>(t.slot) << 12) | (static_cast<uint32_t>(ln) << 6) |
                                           static_cast<uint32_t>(t.nk - 1)));
        }
        for (int32_t i : h->hlevels[l - 1]) {
          if (group[i] != g) continue;
          const SolveNode& N = h->hnodes[i];
          for (int64_t e = N.soff; e < N.soff + N.r; ++e)
            if (rowcode[sidx_h[e]] != 0) coded[e] = rowcode[sidx_h[e]];
        }
        for (int32_t q = 0; q < br.nr; ++q) {
          const SolveTask& t = rb[br.r0 + q];
          for (int32_t ln = 0; ln < t.hi && t.out0 + ln < t.c; ++ln) rowcode[t.first + t.out0 + ln] = 0;
        }
      }
  }
  h->sidx_coded = !coded.empty();
  h->solve_groups = G;
  h->solve_top = top;
  if (hipDeviceSynchronize() != hipSuccess) return fail(FFD_ERR_DEVICE, "device error before a schedule upload");
  bool ok = upload_cap(h, &h->tasks_fwd, &h->cap_tf, tf) == hipSuccess &&
            upload_cap(h, &h->tasks_bwd, &h->cap_tb, tb) == hipSuccess &&
            upload_cap(h, &h->red_fwd, &h->cap_rf, rf) == hipSuccess &&
            upload_cap(h, &h->red_bwd, &h->cap_rb, rb) == hipSuccess &&
            upload_cap(h, &h->yred, &h->cap_yr, yr) == hipSuccess &&
            upload_cap(h, &h->xred, &h->cap_xr, xr) == hipSuccess &&
            upload_cap(h, &h->sidx_def, &h->cap_sd, coded) == hipSuccess;
  if (ok && static_cast<size_t>(fslots) > h->cap_fslots) {
    if (h->fpart) {
      for (auto& a : h->allocs)
        if (a == h->fpart) a = nullptr;
      (void)hipFree(h->fpart);
      h->fpart = nullptr;
    }
    ok = h->alloc(&h->fpart, static_cast<size_t>(fslots) * kSolveOutMax * h->d) == hipSuccess;
    h->cap_fslots = ok ? static_cast<size_t>(fslots) : 0;
  }
  if (ok && static_cast<size_t>(max_slots) > h->cap_slots) {
    if (h->solve_part) {
      for (auto& a : h->allocs)
        if (a == h->solve_part) a = nullptr;
      (void)hipFree(h->solve_part);
      h->solve_part = nullptr;
    }
    ok = h->alloc(&h->solve_part, static_cast<size_t>(max_slots) * kSolveOutMax * h->d) == hipSuccess;
    h->cap_slots = ok ? static_cast<size_t>(max_slots) : 0;
  }
  if (!ok) return fail(FFD_ERR_OUT_OF_MEMORY, "solve schedule upload failed");
  return FFD_OK;
}

}  // namespace
