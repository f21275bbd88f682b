// One-time host setup of the flip-free ADMM solver: element geometry, the
// global matrix L = G^T M G, pin elimination, nested-dissection ordering and
// the FP64 multifrontal Cholesky factor of L_FF stored as per-node panels
// with explicitly inverted diagonal blocks, plus the tables the GPU kernels
// read (CSR of D^T, level schedule, extend-add pull lists).
#pragma once
#include <cstdint>
#include <memory>
#include <utility>
#include <string>
#include <vector>

namespace ffd {

enum Status : int {
  OK = 0,
  ERR_INVALID_ARG = -1,
  ERR_DEGENERATE_ELEMENT = -2,
  ERR_SINGULAR_SYSTEM = -3,
  ERR_NOT_FINITE = -4,
  ERR_DEVICE = -5,
  ERR_OUT_OF_MEMORY = -6,
  ERR_STATE = -7,
};

struct SetupInput {
  int d = 2;        // simplex dimension (2 triangles, 3 tets); output dimension == d
  int din = 2;      // source dimension (d, or 3 with d == 2)
  int64_t n = 0, m = 0;
  const double* V = nullptr;     // n x din row-major
  const int32_t* T = nullptr;    // m x (d+1) row-major
  double rho = 10.0;             // mu_i = rho * w_i
  const double* mu_elem = nullptr;  // optional per-element mu_i (input order, m entries; replaces rho * w_i)
  bool tutte = false;            // factor the edge Laplacian of Tutte's energy instead of G^T M G
  // general linear constraints A W = c beyond the pins (eq. solvinginw): the
  // rows of A in CSR over input vertex indices; the factorised matrix becomes
  // L_FF + gamma A_F^T A_F, which has the same minimiser on the constraint set
  int64_t n_con = 0;
  const int64_t* con_ptr = nullptr;  // n_con + 1
  const int32_t* con_col = nullptr;
  const double* con_val = nullptr;
  int64_t n_pinned = 0;
  const int32_t* pinned_idx = nullptr;
  int leaf_size = 0;             // 0: automatic
  const int8_t* elem_energy = nullptr;  // optional per-element energy (0 or 1), m entries
  bool selfcheck = false;        // solve with the panels on the host and record the residual
  bool device_top = false;       // leave the nodes above the host subtrees to the device (Setup::top)
  // refactorisation: the ordering and symbolic structure of an earlier set-up
  // of the same mesh, pins and constraints (vnew2old, vold2new, nodes,
  // children, struct_idx, panel_entries); only the values are computed
  // (panel_f, top, pin_val, lcf_val, con_gamma), the other tables are left empty
  const struct Setup* structure = nullptr;
};

// One node of the nested-dissection tree; its columns are the contiguous free
// indices [first, first + c); its row structure below the diagonal block is
// the sorted list struct_idx[soff .. soff + r).
struct SolveNode {
  int32_t first = 0, c = 0, r = 0, level = 0;
  int64_t pf = 0;    // forward panel [Linv; -M], (c + r) x c column-major, ld = c + r
  int64_t uoff = 0;  // first row of this node's update vector in the update buffer
  int64_t soff = 0;  // offset into struct_idx
  int64_t poff = 0;  // offset into pull_ptr (c + r + 1 entries)
};

// Allocator whose resize leaves doubles uninitialised: the panels of a large
// factor are written once by the factorisation threads (first touch there),
// never zero-filled first.
template <typename T>
struct UninitAlloc : std::allocator<T> {
  template <typename U>
  struct rebind {
    using other = UninitAlloc<U>;
  };
  UninitAlloc() = default;
  template <typename U>
  UninitAlloc(const UninitAlloc<U>&) noexcept {}
  template <typename U>
  void construct(U* p) noexcept {
    ::new (static_cast<void*>(p)) U;
  }
  template <typename U, typename... A>
  void construct(U* p, A&&... a) {
    ::new (static_cast<void*>(p)) U(std::forward<A>(a)...);
  }
};

// A node above the host-factorised subtrees whose front the device assembles
// and factorises (SetupInput::device_top): the entries of L in its columns and
// the update matrices of its children.
struct TopChild {
  int32_t node = 0;
  bool host = false;          // factorised on the host: its update matrix is upd
  std::vector<int32_t> rel;   // front position of each of the child's update rows
  std::vector<double> upd;    // r x r column-major, lower triangle valid (host children)
};
struct TopNode {
  int32_t node = 0;
  std::vector<int64_t> lidx;  // front entries p + j * (c + r), lower part, from L
  std::vector<double> lval;
  std::vector<TopChild> kids;
};

struct Setup {
  int d = 0, din = 0;
  int64_t n = 0, m = 0, nF = 0, nC = 0;
  double rho = 0;
  // elements in the device order, vertices in the device numbering
  std::vector<double> B;        // m x d x d, B_i = Dm_i^{-T}
  std::vector<double> w;        // m
  std::vector<int32_t> T;       // m x (d+1)
  std::vector<int32_t> vnew2old, vold2new, enew2old;
  int64_t m_energy0 = 0;        // elements of energy 0 (they come first when elem_energy is given)
  // D^T over free rows: entries e*(d+1)+corner, rows ordered by element index
  std::vector<int32_t> dt_ptr, dt_idx;
  // L_FC over free rows: pinned slot and value
  std::vector<int32_t> pin_ptr, pin_col;
  std::vector<double> pin_val;
  // incidences of every vertex (free and pinned rows), entries e*(d+1)+corner
  std::vector<int32_t> av_ptr, av_idx;
  // L_CF over pinned rows: free column and value
  std::vector<int32_t> lcf_ptr, lcf_col;
  std::vector<double> lcf_val;
  // constraints: rows of A with columns in the device numbering (>= nF:
  // pinned), gamma, and the transposed free part over the free rows it touches
  double con_gamma = 0;
  std::vector<int64_t> con_ptr;
  std::vector<int32_t> con_col;
  std::vector<double> con_val;
  std::vector<int32_t> cont_rows, cont_ptr, cont_con;
  std::vector<double> cont_val;
  // factor of L_FF (+ gamma A_F^T A_F)
  std::vector<SolveNode> nodes;
  std::vector<std::vector<int32_t>> children;
  // [Linv; -M] per node (the backward pass reads it transposed); every node the
  // host factorises is written whole, the regions of S.top are not initialised
  std::vector<double, UninitAlloc<double>> panel_f;
  std::vector<int32_t> struct_idx;
  std::vector<int32_t> pull_ptr, pull_idx;
  std::vector<std::vector<int32_t>> level_nodes;
  std::vector<TopNode> top;     // device_top: the nodes left for the device, in postorder (panels zero)
  int64_t ubuf_rows = 0;
  // statistics
  double t_geometry = 0, t_order = 0, t_symbolic = 0, t_numeric = 0;
  double factor_flops = 0;
  int64_t factor_nnz = 0;     // nonzeros of the Cholesky factor (dense node blocks)
  int64_t panel_entries = 0;  // float64 entries of the panels
  double selfcheck_residual = -1;  // |L_FF x - b| / |b| of a host solve with the panels
};

// Returns a Status; on error fills err.
int build_setup(const SetupInput& in, Setup& out, std::string& err);

// Device panel copies, both at offset off[s] (even) for node s with c
// columns and nf = c + r rows, tiled by kPanelTile outputs so that a solve
// task (at most kPanelTile consecutive outputs) reads one contiguous tile:
// the forward copy holds entry (output row i, inner column j) of tile
// t = i / kPanelTile, height h = min(kPanelTile, nf - t kPanelTile), at
// t kPanelTile c + j h + (i - t kPanelTile); the backward copy entry (output
// column j, inner row p) at panel_tile_index(j, p, c, nf) likewise.
// device_panel_offsets fills off and returns the length of each copy.
constexpr int64_t kPanelTile = 64;
inline int64_t panel_tile_index(int64_t out, int64_t in, int64_t nout, int64_t nin) {
  const int64_t t = out / kPanelTile, base = t * kPanelTile;
  const int64_t h = nout - base < kPanelTile ? nout - base : kPanelTile;
  return base * nin + in * h + (out - base);
}
int64_t device_panel_offsets(const Setup& S, std::vector<int64_t>& off);

// Compact host copies of the panels of the nodes not in S.top (off, tot from
// device_panel_offsets): node s's segment of each copy (its device layout,
// padding zero) at coff[s] (-1 for top nodes); runs of consecutive such
// nodes are contiguous both here and on the device.  Returns the compact
// length (the arrays are allocated here).
int64_t build_host_panels(const Setup& S, const std::vector<int64_t>& off, int64_t tot, std::vector<int64_t>& coff,
                          std::unique_ptr<double[]>& prow, std::unique_ptr<double[]>& pcol);

// Element geometry only (B_i = Dm_i^{-T}, w_i) in the input element order.
int element_geometry(int d, int din, int64_t m, const double* V, int64_t n, const int32_t* T,
                     std::vector<double>& B, std::vector<double>& w, std::string& err);

}  // namespace ffd
