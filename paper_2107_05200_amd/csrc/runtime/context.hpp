// Handle state of the flip-free ADMM runtime: error reporting, the per-level
// launch configuration of the triangular solves and the device context
// ffd_ctx (buffers, schedules, graph, penalties, constraints, adjoint state).
// Part of the single translation unit capi.hip (helpers live in anonymous
// namespaces); include only from there.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>  // types only: the library is loaded on first use

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../../include/ffd.h"
#include "../adjoint.hpp"
#include "../host/setup.hpp"
#include "../kernels.hpp"

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

constexpr int64_t kHistCap0 = 1 << 14;

inline unsigned nblk(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }


}  // namespace

// Launch configuration of one solve level of one pass: mode 0 = blocks of nw
// waves per task, 1 = one wave per task; opt = outputs per task (64, 32, 16);
// chunk > 0 splits inner ranges longer than chunk (block mode only); the
// partials are added right after the level, or (forward, defer) only for
// blocks of y rows, by the backward pass.
struct LevelCfg {
  int32_t mode = 0, opt = 64, chunk = 0, nw = 4;  // nw: waves per block (block mode: 4, 8, 16)
  // forward: split y-row blocks only and add their partials in the backward
  // pass; backward (split levels above the lowest): the next backward launch
  // reads the partials and writes the rows
  int32_t defer = 0;
  bool operator==(const LevelCfg& o) const {
    return mode == o.mode && opt == o.opt && chunk == o.chunk && nw == o.nw && defer == o.defer;
  }
};
struct LevelRun {
  int32_t mode = 0, opt = 64, nw = 4, t0 = 0, nt = 0, r0 = 0, nr = 0;  // tasks [t0, t0+nt), reductions [r0, r0+nr)
  int32_t y0 = 0, ny = 0;  // backward runs: pending forward y-row reductions [y0, y0+ny) of yred
  int32_t x0 = 0, nx = 0;  // backward runs: the level above's pending x-row reductions [x0, x0+nx) of xred
  bool reduce_now = true;  // add the split partials right after the level
};

struct ffd_ctx {
  int d = 0, din = 0, prec = 32, energy = 0, h_mode = 0;
  double rho = 0;
  int64_t n = 0, m = 0, nF = 0, nC = 0;
  bool pins_given = false, auto_pinned = false, initialized = false;
  int64_t k = 0;          // completed iterations
  struct Seg {
    int64_t e0, e1;   // element range of one energy (elements are grouped by energy)
    int energy;
    int64_t pb0;      // first partial-sum block of the range
  };
  std::vector<Seg> segs;
  std::vector<int64_t> voff, eoff;  // batch layout: vertex / element offsets per mesh (empty: one mesh)
  // launch shapes (chosen by ffd_autotune)
  int local_bs = 256;              // threads per block of the local step
  int wrhs_lpr = 4;                // lanes per vertex row of the right-hand side
  std::vector<SolveNode> hnodes;   // host copies for rebuilding the solve schedule
  std::vector<std::vector<int32_t>> hlevels;
  int64_t nparts = 0;     // partial-sum blocks of one local step
  int cur = 0;            // index of the buffer holding W^k
  int dev = 0;
  hipStream_t last_stream = nullptr;
  ffd_info info{};
  // host copies
  std::vector<int32_t> vnew2old;
  // device buffers
  int32_t *T = nullptr, *vnew2old_d = nullptr, *enew2old_d = nullptr;
  double* B64 = nullptr;
  void *B = nullptr, *w = nullptr;
  double *x[2] = {nullptr, nullptr}, *xC = nullptr;
  void *U = nullptr, *P = nullptr, *L = nullptr, *gn = nullptr, *g = nullptr;
  double *b = nullptr, *y = nullptr, *ub = nullptr, *partials = nullptr, *hist = nullptr;
  double* partials2 = nullptr;  // first-stage sums of the partials (many local-step blocks)
  int64_t hist_cap = 0;
  int32_t *dt_ptr = nullptr, *dt_idx = nullptr, *pin_ptr = nullptr, *pin_col = nullptr;
  double* pin_val = nullptr;
  std::vector<int64_t> hpoff;  // device panel offset of every node
  // two captured iterations replayed by ffd_iterate_graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  bool graph_valid = false;      // captured with the current launch shapes and buffers
  int graph_cur = 0;             // map buffer holding W^k when the graph starts
  double* graph_hist = nullptr;  // history buffer the graph writes to
  int64_t* k_dev = nullptr;      // device copy of the iteration counter
  void* glam = nullptr;          // corner vectors of Lambda (diagnostic iterations)
  // penalty rescaling: per-element mu_e / w_e on the device (nullptr: rho for
  // every element), the new mu_e of a rescaling event, and the host copy of
  // the set-up input the factor is rebuilt from
  void* rho_e = nullptr;
  double* mu_dev = nullptr;
  bool rescaled = false;
  std::vector<double> in_V;
  std::vector<int32_t> in_T, in_pins, enew2old_h;
  std::vector<int8_t> in_energy;
  int in_leaf = 0;
  size_t n_pin_val = 0, n_lcf_val = 0;
  std::unique_ptr<Setup> hstruct;  // ordering and symbolic structure, reused by refactorisations
  double* gtl_part = nullptr;    // per-block partial sums of |G^T Lambda|^2
  // termination test per problem (each mesh of a batch; a plain handle is one):
  // pieces of the problems' element and vertex lists, their partial sums and
  // the per-problem sums (k_diag_pieces / k_diag_problems); element count per problem
  DiagPiece* diag_pieces = nullptr;
  int32_t *diag_elist = nullptr, *diag_vlist = nullptr, *diag_piece_ptr = nullptr;
  double *diag_part = nullptr, *diag_out = nullptr;
  int32_t diag_npieces = 0, diag_nprob = 0;
  std::vector<int64_t> diag_m;
  // general linear constraints A W = c: rows of A (device numbering; host and
  // device copies), the transposed free part over the rows it touches, the
  // right-hand sides c, per-iteration c', A y - c', lambda, the precomputed
  // Z = L~^{-1} A_F^T (column-major) and S^{-1}, and a solve scratch vector
  int64_t ncon = 0, ncon_rows = 0;
  double con_gamma = 0;
  std::vector<int64_t> con_ptr_h, in_con_ptr;
  std::vector<int32_t> con_col_h, in_con_col;
  std::vector<double> con_val_h, in_con_val;
  int64_t* con_ptr = nullptr;
  int32_t *con_col = nullptr, *cont_rows = nullptr, *cont_ptr = nullptr, *cont_con = nullptr;
  double *con_val = nullptr, *cont_val = nullptr, *con_c = nullptr, *con_cp = nullptr, *con_t = nullptr;
  double *con_lam = nullptr, *con_Z = nullptr, *con_Sinv = nullptr, *con_tmp = nullptr;
  // dense-library handle of the device refactorisation (created on first use)
  bool device_refactor = true;  // factorise the top fronts of a refactorisation on the device
  rocblas_handle blas = nullptr;
  rocblas_status (*blas_destroy)(rocblas_handle) = nullptr;
  std::vector<LevelCfg> cfg_fwd, cfg_bwd;  // per-level launch configuration of both solve passes
  // The forest below level solve_top is split into solve_groups groups of
  // whole subtrees, each solved on its own stream (group 0 on the caller's);
  // levels >= solve_top run on the caller's stream after the join.
  int solve_groups = 1, solve_top = 0;
  bool xcd_lanes = true;  // level tasks grouped per node onto one XCD (see xcd_order)
  std::vector<int32_t> hparent;                  // parent node (-1: root)
  std::vector<std::vector<LevelRun>> grun_fwd, grun_bwd;  // [group][level]; group solve_groups = top levels
  std::vector<hipStream_t> wstreams;             // worker streams of groups 1..
  hipEvent_t fork_ev[2] = {nullptr, nullptr}, join_ev[2][8] = {};
  double *Prow = nullptr, *Pcol = nullptr;  // factor panels, row- and column-major copies
  int32_t *sidx = nullptr, *pull_ptr = nullptr, *pull_idx = nullptr;
  SolveTask *tasks_fwd = nullptr, *tasks_bwd = nullptr, *red_fwd = nullptr, *red_bwd = nullptr;
  size_t cap_tf = 0, cap_tb = 0, cap_rf = 0, cap_rb = 0, cap_slots = 0;  // capacities (entries)
  SolveTask* yred = nullptr;  // forward y-row reductions, in the order the backward launches run them
  SolveTask* xred = nullptr;  // deferred backward x-row reductions, likewise
  size_t cap_xr = 0, cap_sd = 0;
  int32_t* sidx_def = nullptr;  // structure lists with deferred rows coded (read instead of sidx
  bool sidx_coded = false;      // by the backward launches when sidx_coded)
  double* fpart = nullptr;    // forward split partials (kept until the backward pass adds them)
  size_t cap_yr = 0, cap_fslots = 0;
  double* solve_part = nullptr;                   // backward split-K partials, a region per level
  int64_t device_bytes = 0;
  std::vector<void*> allocs;
  std::vector<hipEvent_t> events;
  double* hist_scratch = nullptr;  // history record target of recomputed iterations
  // adjoint: incidence of all vertex rows, L_CF, checkpoints and adjoint state
  int32_t *av_ptr = nullptr, *av_idx = nullptr, *lcf_ptr = nullptr, *lcf_col = nullptr;
  double* lcf_val = nullptr;
  int64_t adj_k0 = -1, adj_K = 0, adj_every = 0, adj_nslots = 0;
  char* adj_ck = nullptr;    // checkpoint slots
  char* adj_seg = nullptr;   // per-iteration states of one segment (every + 1 slots)
  char* adj_fin = nullptr;   // the state after the K iterations
  double *Ubar = nullptr, *Pbar = nullptr, *Lbar = nullptr, *Bbar = nullptr, *wbar = nullptr;
  double *gadj = nullptr, *lam = nullptr, *xbar = nullptr, *pinsbar = nullptr, *vbar = nullptr;
  // one saved state: U, P, Lambda, |grad f(P)|^2, the next right-hand side's
  // corner vectors (so a restored state continues bit for bit), and the map
  size_t slot_elem_entries() const {
    const size_t nU = d == 2 ? 2 : 9, nP = d == 2 ? 3 : 6;
    return nU + nP + static_cast<size_t>(d) * d + 1 + static_cast<size_t>(d + 1) * d;
  }
  size_t slot_bytes() const {
    const size_t el = rsize() * m * slot_elem_entries();
    return ((el + 255) / 256) * 256 + static_cast<size_t>(n) * d * sizeof(double);
  }

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
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (hipStream_t w : wstreams) (void)hipStreamDestroy(w);
    for (int p = 0; p < 2; ++p) {
      if (fork_ev[p]) (void)hipEventDestroy(fork_ev[p]);
      for (hipEvent_t e : join_ev[p])
        if (e) (void)hipEventDestroy(e);
    }
    for (hipEvent_t ev : events) (void)hipEventDestroy(ev);
    if (blas && blas_destroy) (void)blas_destroy(blas);
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

}  // namespace
