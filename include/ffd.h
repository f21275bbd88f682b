/*
 * ffd.h -- C ABI of the MI355X (gfx950) flip-free ADMM solver.
 *
 * The solver runs the three-block ADMM of Stein, Li & Solomon, "A Splitting
 * Scheme for Flip-Free Distortion Energies" (Algorithm 1 with the fixed
 * penalties of the loop of Algorithm 2): the W-step (eq. solvinginw, a solve
 * with the fixed matrix L = G^T M G factored once), the U-step (Procrustes,
 * eqs. proximalfunctionu / optimizationinudecoupled), the P-step (eqs.
 * optimizinginp / rootfindinginp with the per-eigenvalue roots of the
 * supplement) and the Lambda-step (eq. lambdaupdate), with the primal and
 * dual residuals of eq. primaldualerror.
 *
 * Conventions
 *  - Status: every call returns ffd_status (0 = OK, < 0 = error) and leaves
 *    the handle unchanged on error; ffd_last_error() gives a thread-local
 *    message.  Numerical trouble (flipped Jacobians, non-finite values) is not
 *    an error: it is recorded in the history.
 *  - Ownership: host inputs are copied by ffd_create; the caller keeps them.
 *    Device buffers passed to the other calls belong to the caller and must
 *    hold the documented number of elements.  The handle owns its own device
 *    and host memory and frees it in ffd_destroy.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  A call after ffd_create only enqueues work on that stream
 *    (no host synchronisation) unless its comment says that it synchronises
 *    (ffd_get_history, the loops with a termination test, rescaling, the
 *    timing and tuning calls).
 *  - Layouts: the map (W of the paper) is n x d row-major float64 in the
 *    caller's vertex order.  Element arrays (U, P, Lambda, W_el = U P) are
 *    m x d x d row-major in the caller's element order, float32 when the
 *    handle was created with precision 32 and float64 with precision 64.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef FFD_H
#define FFD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ffd_ctx* ffd_handle;

typedef enum {
  FFD_SYMMETRIC_DIRICHLET = 0, /* f(X) = 1/2 (|X|^2 + |X^-1|^2)   (Table 1)                    */
  FFD_SYMMETRIC_GRADIENT = 1   /* f(X) = 1/2 |X|^2 - log det X    (eq. symmetricgradient...)   */
} ffd_energy;

typedef enum {
  FFD_OK = 0,
  FFD_ERR_INVALID_ARG = -1,        /* bad sizes, indices, options or NULL pointers              */
  FFD_ERR_DEGENERATE_ELEMENT = -2, /* an element with zero (or non-finite) area / volume         */
  FFD_ERR_SINGULAR_SYSTEM = -3,    /* a connected component without a pin: L_FF is singular     */
  FFD_ERR_NOT_FINITE = -4,         /* NaN / Inf in V or pinned positions                          */
  FFD_ERR_DEVICE = -5,             /* a HIP runtime call failed                                   */
  FFD_ERR_OUT_OF_MEMORY = -6,
  FFD_ERR_STATE = -7               /* call out of order (e.g. ffd_iterate before ffd_init)        */
} ffd_status;

/* One mesh (Section "Preliminaries"): n source vertices V (n x dim_in,
 * row-major float64) and m elements T (m x (simplex_dim+1), int32).  The
 * output dimension equals simplex_dim (square Jacobians, Def. "Piecewise
 * constant Jacobian"); dim_in = 3 with simplex_dim = 2 is a UV map of a surface
 * (intrinsic gradient, supplement "Computing the Jacobian Map"). */
typedef struct {
  int32_t simplex_dim; /* d: 2 = triangles, 3 = tetrahedra          */
  int32_t dim_in;      /* d or (3 when d == 2)                       */
  int64_t n_vertices;
  int64_t n_elements;
  const double* V;     /* host, n_vertices x dim_in                  */
  const int32_t* T;    /* host, n_elements x (d + 1)                 */
} ffd_mesh;

/* Options.  mu_i = rho * w_i with w_i the element area / volume (the
 * penalties of eq. augmentedlagrangian; per element after ffd_rescale).  Pins are the
 * linear constraints A W = b of eq. solvinginw restricted to fixed vertices;
 * with no pins and auto_pin = 1 vertex 0 is fixed at its initial position (the
 * W-step text fixes the first vertex when there are no constraints). */
typedef struct {
  int32_t energy;            /* ffd_energy                                                   */
  double rho;                /* > 0                                                           */
  int32_t h_mode;            /* proximal weight of eq. proximalfunctionu: 0 = off (h = 0)     */
  int32_t precision;         /* 32 or 64: arithmetic of the element steps; the factor, the
                                W-step right-hand side, the map and all sums are float64      */
  int64_t n_pinned;
  const int32_t* pinned_idx; /* host, n_pinned distinct vertex indices                        */
  const double* pinned_pos;  /* host, n_pinned x d row-major, may be NULL (then taken from the
                                initial map in ffd_init)                                      */
  int32_t auto_pin;          /* 1: pin vertex 0 when n_pinned == 0                             */
  int32_t leaf_size;         /* nested-dissection leaf size; 0 = automatic: 60 (tets) or 64
                                (triangles) for the largest connected component of the free
                                vertices, 32 for components of at most a quarter of its size */
} ffd_options;

/* Set-up statistics (filled by ffd_create / ffd_get_info). */
typedef struct {
  int64_t n_free, n_pinned;
  int64_t factor_nnz;       /* nonzeros of the Cholesky factor of L_FF                         */
  int64_t panel_entries;    /* float64 entries of one copy of the solve panels                 */
  int32_t n_nodes, n_levels;
  double t_geometry, t_order, t_symbolic, t_numeric, t_upload; /* seconds                       */
  double factor_flops;
  int64_t device_bytes;     /* device memory owned by the handle                              */
} ffd_info;

/* History record per iteration (FFD_HIST_FIELDS float64):
 *  0 e_prim   sqrt(sum_i |J_i - U_i P_i|^2)                  (eq. primaldualerror)
 *  1 e_dual   sqrt(sum_i mu_i^2 |J_i^k - J_i^{k-1}|^2)       (eq. primaldualerror)
 *  2 E_P      sum_i w_i f(P_i)
 *  3 E_map    sum_i w_i f(J_i), +inf if any det J_i <= 0     (eq. genericdeformationenergy)
 *  4 Phi      augmented Lagrangian at (W^k, U^k, P^k, Lambda^k) (eq. augmentedlagrangian)
 *  5 flips    number of elements with det J_i <= 0
 *  6 nonfinite number of elements whose Lambda is not finite
 *  7 norm_GW  |G W^k|                                         (eq. primaldualthresholds)
 *  8 norm_P   |P^k|                                           (eq. primaldualthresholds)
 *  9 norm_GtLam  |G^T Lambda^k| over all vertex rows (eq. primaldualthresholds),
 *             recorded at the check iterations of ffd_iterate_until / ffd_run,
 *             NaN elsewhere
 * 10 max_grad_f  max_i |grad f(P_i^k)| (the proxy for B_i of Condition "gradf"
 *             plotted with the UV-mapping bounds); at the check iterations of
 *             ffd_iterate_until / ffd_run, NaN elsewhere
 * 11 max_lambda_ratio  max_i |L1 - L0| / |1/2 (L1 - L0 + U1 L1^T U1 - U0 L0^T U0)|
 *             with L0, U0 = Lambda_i, U_i before and L1, U1 after the iteration
 *             (the proxy for gamma^(1/2) of Condition "lambdabound"; +inf where
 *             the denominator vanishes and the numerator does not); at the check
 *             iterations of ffd_iterate_until / ffd_run, NaN elsewhere
 * J_i = (G W^k)_i.  Iterations are numbered from 1 after ffd_init. */
#define FFD_HIST_FIELDS 12

/* Host set-up: geometry (B_i, w_i), L = G^T M G, pin elimination, nested
 * dissection, FP64 multifrontal Cholesky of L_FF, then upload to the current
 * HIP device.  Synchronous.  On success *out is a new handle. */
ffd_status ffd_create(const ffd_mesh* mesh, const ffd_options* opt, ffd_handle* out);

/* General linear constraints A W = c on the map (eq. solvinginw; the W-step
 * text), beyond pins: rows of A in CSR over vertex indices (distinct columns
 * per row, at least one free vertex per row), c = rhs (host, n_rows x
 * simplex_dim row-major; the same row of A acts on every output
 * coordinate).  At most 1024 rows. */
typedef struct {
  int64_t n_rows;
  const int64_t* row_ptr; /* host, n_rows + 1, row_ptr[0] = 0 */
  const int32_t* col_idx; /* host, vertex indices                 */
  const double* val;      /* host                                 */
  const double* rhs;      /* host, n_rows x simplex_dim           */
} ffd_constraints;

/* As ffd_create, with general constraints.  The W-step then returns the
 * constrained minimiser of eq. solvinginw: the host factorises
 * L_FF + gamma A_F^T A_F (gamma > 0 scales A to L's diagonal; the
 * minimiser on the constraint set is the same for any gamma, and the matrix
 * is definite when the constraints and pins fix every component's
 * translation), and the device adds the KKT correction x = y - Z lambda with
 * Z = L~^{-1} A_F^T (n_rows x n_free float64 kept on the device) and the
 * explicit inverse of S = A_F Z.  No vertex is fixed automatically (the first
 * vertex is fixed only when there are no constraints).  ffd_solve solves
 * with the factorised matrix; the adjoint entry points refuse such a handle
 * (FFD_ERR_STATE).  Errors: as ffd_create; FFD_ERR_SINGULAR_SYSTEM when the
 * rows are dependent (with the pins) or a component's translation stays free. */
ffd_status ffd_create_constrained(const ffd_mesh* mesh, const ffd_options* opt, const ffd_constraints* con,
                                  ffd_handle* out);

/* New right-hand sides c (device, n_rows x simplex_dim float64) for the next
 * W-steps; stream-ordered. */
ffd_status ffd_set_constraint_rhs(ffd_handle h, const double* rhs_dev, void* stream);

/* Minimiser of Tutte's energy (supplement "Tutte's Energy", Table 1): the sum
 * over the mesh edges (i, j) of |W_i - W_j|^2 / |V_i - V_j|, with the n_fixed
 * vertices fixed_idx held at fixed_pos (host, n_fixed x simplex_dim
 * row-major), e.g. the boundary on a convex curve for a flip-free 2D
 * initial map, or on a target surface for a volume (there it may flip
 * elements).  The edge Laplacian is factorised on the host with the same
 * ordering and factor form as L = G^T M G and solved on the device with the
 * W-step's solve kernels; map_dev (device, n_vertices x simplex_dim float64,
 * input vertex order) receives the whole map.  Synchronous on `stream`.
 * Errors: as ffd_create (a connected component without a fixed vertex:
 * FFD_ERR_SINGULAR_SYSTEM; a zero-length edge: FFD_ERR_DEGENERATE_ELEMENT). */
ffd_status ffd_tutte_map(const ffd_mesh* mesh, int64_t n_fixed, const int32_t* fixed_idx, const double* fixed_pos,
                         int32_t leaf_size, double* map_dev, void* stream);

/* Batched form: n_meshes independent meshes (same simplex_dim and dim_in;
 * options with the same precision, h_mode and rho; energy, pins and
 * auto_pin per mesh; pinned positions given for all meshes or for none) in
 * one handle.  Their vertices and elements are concatenated in mesh order:
 * every other call works on the concatenated arrays (map: sum n x d, element
 * arrays: sum m x d x d) and one ffd_iterate advances all meshes together
 * (one launch sequence; the meshes' factors form one block-diagonal factor
 * whose level schedules are merged level by level; elements are grouped by
 * energy so each launch is single-energy).  History records sum over all
 * meshes. */
ffd_status ffd_batch_create(const ffd_mesh* meshes, const ffd_options* opts, int32_t n_meshes, ffd_handle* out);

/* Offsets of each mesh's vertices and elements in the concatenated arrays
 * (n_meshes + 1 entries each, host; a plain handle reports one mesh). */
ffd_status ffd_batch_layout(ffd_handle h, int64_t* vertex_offsets, int64_t* element_offsets);

/* Host-only analysis: runs the set-up of ffd_create (geometry, global
 * matrix, ordering, factorisation) without touching a device and returns its
 * statistics; *selfcheck_residual (may be NULL) receives |L_FF x - b| / |b| of
 * a host solve with the factor panels for a fixed right-hand side.  For
 * checking inputs and the factorisation on machines without a GPU. */
ffd_status ffd_analyze(const ffd_mesh* mesh, const ffd_options* opt, ffd_info* info,
                       double* selfcheck_residual);

/* Statistics of a created handle. */
ffd_status ffd_get_info(ffd_handle h, ffd_info* info);

/* Initialisation (Section "Implementation", "Initializing U, P, Lambda"):
 * U0, P0 from the SVD of J0 = G map0 with the flip and epsilon rules;
 * Lambda0 = 0.  map0 (device, n x d float64) is W^0 as given: the pins act
 * through the W-step of the first iteration; when no pinned positions were
 * given they are taken from map0. */
ffd_status ffd_init(ffd_handle h, const double* map0_dev, void* stream);

/* Replace the pinned positions (device, n_pinned x d float64, in the order of
 * options.pinned_idx).  Takes effect at the next W-step. */
ffd_status ffd_set_pins(ffd_handle h, const double* pinned_pos_dev, void* stream);

/* Run n_iter iterations of Algorithm 1, appending n_iter history records. */
ffd_status ffd_iterate(ffd_handle h, int32_t n_iter, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ffd_iterate
 * without any allocation.  The local step's per-block partial sums go to a
 * fixed 4 MiB scratch array of the library (one per GPU, kept until the
 * process ends, looked up with hipGetSymbolAddress on the first call on a
 * device) instead of the handle's buffer; results are bitwise those of
 * ffd_iterate.  All calls on one GPU share that scratch, so calls that
 * overlap on one GPU (other streams, other threads, other handles) race.
 * Errors: FFD_ERR_INVALID_ARG when the handle's history cannot hold
 * n_iter more records (ffd_iterate would grow it) or when the local step
 * needs more than the scratch holds ((ceil(m / block) + blocks / 256) x 11
 * float64: about 12M elements at the default 256-element block, 3M at the
 * 64-element block the autotuner picks for the tet cube); FFD_ERR_STATE
 * before ffd_init. */
ffd_status ffd_iterate_noalloc(ffd_handle h, int32_t n_iter, void* stream);

/* As ffd_iterate, with the launches of two iterations captured once into a
 * HIP graph (on a stream of the handle's own) and replayed on `stream`
 * (Algorithm 1's loop body has a fixed launch sequence, so one capture serves
 * every replay).  Results are bitwise those of ffd_iterate.  The graph is
 * captured again after anything that changes launch shapes or buffers
 * (ffd_autotune, a larger history); an odd iteration is run directly. */
ffd_status ffd_iterate_graph(ffd_handle h, int32_t n_iter, void* stream);

/* Algorithm 2's loop with its termination test: up to max_iter iterations;
 * every check_every-th iteration (and the last) also records |G^T Lambda|
 * (history field 9, otherwise NaN) and the loop stops once the state meets
 * both thresholds of eq. primaldualthresholds,
 *   e_prim < eps_abs sqrt(d m) + eps_rel max(|G W|, |P|),
 *   e_dual < eps_abs sqrt(d m) + eps_rel |G^T Lambda|,
 * and, with require_flip_free, no element of the map has det J <= 0 (the
 * paper's added condition).  The test is evaluated in float64 from the state
 * after the check iteration, per problem: on a batched handle every mesh is
 * tested on its own (its m, its elements and vertex rows), and the loop stops
 * when all meshes pass.  The paper uses eps_abs = 1e-6, eps_rel = 1e-5
 * (5e-10, 5e-9 for deformations).  use_graph: the iterations between checks
 * replay the captured graph (ffd_iterate_graph).  Synchronises `stream` at
 * every check.  iters_done / converged (host, may be NULL): iterations run,
 * 1 if the test was met.  Errors: FFD_ERR_INVALID_ARG for max_iter < 0,
 * check_every < 1 or negative tolerances. */
ffd_status ffd_iterate_until(ffd_handle h, int32_t max_iter, int32_t check_every, double eps_abs, double eps_rel,
                             int32_t require_flip_free, int32_t use_graph, void* stream, int32_t* iters_done,
                             int32_t* converged);

/* One penalty rescaling event (Section "Implementation", "Rescaling mu_i and
 * Lambda") after the last iteration: per element, mu_i is multiplied by
 * rho_r / 2 if e_prim_i > rho_r e_dual_i and divided by it if e_dual_i >
 * rho_r e_prim_i (the paper uses rho_r = 5), never below half the bound of
 * Prop. "Sufficient decrease" (gamma = 1, epsilon = 0; F_i of the Lipschitz
 * lemma with B_i = sqrt(5 (1 + |grad f(P_i)|^2)), F_i^2 capped at
 * eps_m^(-1/4)); Lambda_i is divided by the same factor, and L = G^T M G is
 * factorised again on the host (same ordering and structure) and uploaded.
 * Synchronous.  From then on the handle uses the per-element penalties until
 * the next ffd_init, which returns to mu_i = rho w_i; the adjoint entry
 * points refuse a rescaled handle (FFD_ERR_STATE).  Errors: FFD_ERR_STATE
 * before the first iteration, FFD_ERR_INVALID_ARG for rho_r <= 2. */
ffd_status ffd_rescale(ffd_handle h, double rho_r, void* stream);

/* Where ffd_rescale refactorises: device = 1 (default when rocBLAS and
 * rocSOLVER load) factorises the large top fronts of the nested-dissection
 * tree on the device (assembly kernels plus rocSOLVER potrf / trtri and
 * rocBLAS trsm / syrk / trmm) and the subtrees below them on the host;
 * device = 0 factorises everything on the host.  Results agree to rounding.
 * Errors: FFD_ERR_STATE for device = 1 without the libraries. */
ffd_status ffd_set_refactor_mode(ffd_handle h, int32_t device);

/* Algorithm 2: up to max_iter iterations from the current state with
 * rescaling events (rescale_rho > 2; 0 = none) after iterations 1..5 of the
 * run and then every 5 (3/2)^p iterations (p = past events, rounded half up),
 * and the termination test of ffd_iterate_until at every check_every-th
 * iteration, taken in Algorithm 2's order: after the rescaling block of the
 * same iteration, on the state as it stands (an event's new mu_i enter
 * e_dual and its rescaled Lambda enters |G^T Lambda|).  Per problem on a
 * batched handle, as in ffd_iterate_until.  iters_done / converged /
 * rescales_done (host, may be NULL). */
ffd_status ffd_run(ffd_handle h, int32_t max_iter, int32_t check_every, double eps_abs, double eps_rel,
                   int32_t require_flip_free, double rescale_rho, int32_t use_graph, void* stream, int32_t* iters_done,
                   int32_t* converged, int32_t* rescales_done);

/* As ffd_iterate, with a HIP event recorded on `stream` between the phases
 * of every iteration; on return (after synchronising the stream)
 * phase_ms_host[0..4] hold the summed milliseconds of the phases
 *   0 W-step right-hand side, 1 forward triangular solve, 2 backward
 *   triangular solve, 3 fused U/P/Lambda step, 4 history reduction,
 * and phase_ms_host[5] the total from the first to the last event. */
#define FFD_PROFILE_FIELDS 6
ffd_status ffd_iterate_profiled(ffd_handle h, int32_t n_iter, void* stream, double* phase_ms_host);

/* Per-level timing of the W-step's two triangular-solve passes (the
 * back-substitution of eq. solvinginw with the level-scheduled factor): n_rep
 * timed solves of the current right-hand side (after one untimed one), with
 * a HIP event on `stream` after every level of each pass; the solution goes
 * to the map buffer the next W-step overwrites, so the state is unchanged.
 * out_host (host, cap_levels x FFD_LEVEL_FIELDS float64) per level l from the
 * leaves up: 0 forward ms, 1 backward ms (averages per solve; a level's
 * launches include its split-partial reduction), 2 algorithmic bytes of the
 * level's factor entries (8 (c (c + 1) / 2 + c r) per node, read once per
 * pass), 3 nodes, 4 largest c, 5 largest r, 6 forward tasks, 7 backward
 * tasks, 8 forward reduction tasks, 9 backward reduction tasks run right
 * after the level.  *n_levels receives the level count.  Synchronises.
 * Errors: FFD_ERR_INVALID_ARG when cap_levels is smaller than the level
 * count, FFD_ERR_STATE for a schedule split over several streams. */
#define FFD_LEVEL_FIELDS 10
ffd_status ffd_profile_solve_levels(ffd_handle h, int32_t n_rep, void* stream, double* out_host, int32_t cap_levels,
                                   int32_t* n_levels);

/* Copy the state out; any pointer may be NULL.  map: n x d float64; Wel, U,
 * P, Lambda: m x d x d in the handle's precision. */
ffd_status ffd_get_state(ffd_handle h, double* map_dev, void* Wel_dev, void* U_dev, void* P_dev,
                         void* Lambda_dev, void* stream);

/* Overwrite the state (resume or teacher forcing): map is W^k (n x d
 * float64, used as W^{k-1} by the dual residual of the next iteration); U,
 * P (symmetric; the mean of P and P^T is used), Lambda: m x d x d in the
 * handle's precision.  The next W-step right-hand side is rebuilt from them.
 * The iteration counter becomes k; history records before k are undefined. */
ffd_status ffd_set_state(ffd_handle h, const double* map_dev, const void* U_dev, const void* P_dev,
                         const void* Lambda_dev, int64_t k, void* stream);

/* Copy history records [first, first + count) to host memory
 * (count x FFD_HIST_FIELDS float64).  Synchronises the handle's last stream. */
ffd_status ffd_get_history(ffd_handle h, int64_t first, int64_t count, double* out_host);

/* Number of completed iterations since ffd_init. */
ffd_status ffd_get_iteration(ffd_handle h, int64_t* k);

/* Solve L_FF x = b for the free vertices with the handle's factor (the
 * back-substitution of the W-step).  b, x: device, n_free x d float64 in the
 * handle's internal free-vertex order (see ffd_get_vertex_order). */
ffd_status ffd_solve(ffd_handle h, const double* b_dev, double* x_dev, void* stream);

/* Internal vertex order: order_host[j] = caller index of internal vertex j
 * (free vertices first, then the pins in options order). */
ffd_status ffd_get_vertex_order(ffd_handle h, int32_t* order_host);

/* Adjoint, forward part: run n_iter iterations of Algorithm 1 from the
 * current state (as ffd_iterate, appending history) and keep a device
 * checkpoint of the state every checkpoint_every iterations, for
 * ffd_adjoint_backward, which recomputes checkpoint_every - 1 iterations per
 * checkpoint.  Memory: ceil(n_iter / checkpoint_every) + checkpoint_every + 1
 * copies of the element state and map (U, P, Lambda, |grad f|^2, corner
 * vectors, map); checkpoint_every = 1 keeps every state and recomputes
 * nothing.  The adjoint differentiates the iteration with
 * mu_i = rho w_i, no general constraints and no proximal term: a rescaled
 * handle, a constrained one and one with h_mode 1 give FFD_ERR_STATE. */
ffd_status ffd_adjoint_forward(ffd_handle h, int32_t n_iter, int32_t checkpoint_every, void* stream);

/* Adjoint, reverse part: gradients of a loss of the final element state
 * with respect to the pinned targets and the rest vertices, through the
 * n_iter iterations of the last ffd_adjoint_forward (which must be the last
 * iterations run).  The iterations are recomputed segment by segment from the
 * checkpoints (Algorithm 1 steps: the W-step by implicit differentiation of
 * eq. solvinginw with the same factor, the polar U-step, the spectral P-step
 * of eq. rootfindinginp, the Lambda-step of eq. lambdaupdate).
 *  Pbar_dev: optional (NULL) device m x d x d in the handle's precision and
 *    the caller's element order, the gradient of the loss with respect to P^K;
 *  energy_loss: 1 adds the loss sum_i w_i f(P_i^K) (its P and w terms);
 *  pins_bar_dev: optional device n_pinned x d float64 output (pinned targets);
 *  V_bar_dev: optional device n x dim_in float64 output (rest vertices; needs
 *    dim_in == simplex_dim and assumes W^0 = V, for which the initial state
 *    does not depend on V).
 * The gradients do not depend on checkpoint_every (bitwise).  The handle's
 * state is left as it was after the forward part. */
ffd_status ffd_adjoint_backward(ffd_handle h, const void* Pbar_dev, int32_t energy_loss, double* pins_bar_dev,
                                double* V_bar_dev, void* stream);

/* Autotuner: picks the launch shapes of the handle's kernels by timing them
 * with HIP events on `stream` from the current state (which is saved before
 * and restored after; the timed iterations are not recorded): the local-step
 * block size (64 / 128 / 256 elements), the lanes per vertex row of the
 * right-hand side (2 / 4 / 8); level by level for both triangular-solve
 * passes, the task shape (blocks of 4 / 8 / 16 waves or one wave per task,
 * 64 / 32 / 16 outputs per task, inner-range splitting: none, 2048 .. 256,
 * with the partials added right away, or, for forward blocks of y rows, by
 * the backward pass, or, for backward levels above the lowest, by the next
 * backward launch, which reads the pending rows from the partials); and the
 * number of streams (1 .. 4, the caller's stream plus streams of the handle,
 * all of default priority) over which the subtrees below a top level are
 * spread.  With cache_path (may be NULL) the choice is read from / appended
 * to a text file, one line per key "arch|d|energy|precision|element
 * bucket|factor bucket|levels|h" followed by the block size, lanes per row,
 * level count, stream count, top level and five numbers (mode, outputs,
 * chunk, waves, deferred) per level and pass.  choice_out (may be NULL): 6 int32 (block size,
 * lanes per row, solve levels run one wave per task, solve levels with split
 * inner ranges (both passes counted), streams, top level).  Element results
 * do not depend on the choice; history sums and the solve's rounding order
 * may change in the last bits (deferral and the stream count change nothing). */
ffd_status ffd_autotune(ffd_handle h, const char* cache_path, void* stream, int32_t* choice_out);

void ffd_destroy(ffd_handle h);

const char* ffd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FFD_H */
