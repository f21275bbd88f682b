"""Thin ctypes binding of libffd.so (include/ffd.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory (tensors passed by ``data_ptr()``) and streams
(``torch.cuda.current_stream().cuda_stream``).  A missing library is an error,
never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffd.so")
HIST_FIELDS = 12
HIST_NAMES = ("e_prim", "e_dual", "E_P", "E_map", "Phi", "flips", "nonfinite",
              "norm_GW", "norm_P", "norm_GtLam", "max_grad_f", "max_lambda_ratio")

STATUS = {0: "FFD_OK", -1: "FFD_ERR_INVALID_ARG", -2: "FFD_ERR_DEGENERATE_ELEMENT",
          -3: "FFD_ERR_SINGULAR_SYSTEM", -4: "FFD_ERR_NOT_FINITE", -5: "FFD_ERR_DEVICE",
          -6: "FFD_ERR_OUT_OF_MEMORY", -7: "FFD_ERR_STATE"}


class FFDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Mesh(C.Structure):
    _fields_ = [("simplex_dim", C.c_int32), ("dim_in", C.c_int32), ("n_vertices", C.c_int64),
                ("n_elements", C.c_int64), ("V", C.POINTER(C.c_double)), ("T", C.POINTER(C.c_int32))]


class Options(C.Structure):
    _fields_ = [("energy", C.c_int32), ("rho", C.c_double), ("h_mode", C.c_int32),
                ("precision", C.c_int32), ("n_pinned", C.c_int64),
                ("pinned_idx", C.POINTER(C.c_int32)), ("pinned_pos", C.POINTER(C.c_double)),
                ("auto_pin", C.c_int32), ("leaf_size", C.c_int32)]


class Constraints(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("rhs", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("n_free", C.c_int64), ("n_pinned", C.c_int64), ("factor_nnz", C.c_int64),
                ("panel_entries", C.c_int64), ("n_nodes", C.c_int32), ("n_levels", C.c_int32),
                ("t_geometry", C.c_double), ("t_order", C.c_double), ("t_symbolic", C.c_double),
                ("t_numeric", C.c_double), ("t_upload", C.c_double), ("factor_flops", C.c_double),
                ("device_bytes", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None

_PROTOS = {
    "ffd_create": (C.c_int, [C.POINTER(Mesh), C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "ffd_analyze": (C.c_int, [C.POINTER(Mesh), C.POINTER(Options), C.POINTER(Info), C.POINTER(C.c_double)]),
    "ffd_get_info": (C.c_int, [C.c_void_p, C.POINTER(Info)]),
    "ffd_init": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ffd_set_pins": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ffd_iterate": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "ffd_iterate_graph": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "ffd_iterate_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "ffd_iterate_until": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_int32,
                                    C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ffd_rescale": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p]),
    "ffd_create_constrained": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ffd_set_refactor_mode": (C.c_int, [C.c_void_p, C.c_int32]),
    "ffd_set_constraint_rhs": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ffd_tutte_map": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "ffd_run": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.c_double, C.c_int32,
                          C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ffd_iterate_profiled": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_double)]),
    "ffd_profile_solve_levels": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_double), C.c_int32,
                                           C.POINTER(C.c_int32)]),
    "ffd_get_state": (C.c_int, [C.c_void_p] + [C.c_void_p] * 5 + [C.c_void_p]),
    "ffd_set_state": (C.c_int, [C.c_void_p] + [C.c_void_p] * 4 + [C.c_int64, C.c_void_p]),
    "ffd_get_history": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_double)]),
    "ffd_get_iteration": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "ffd_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ffd_get_vertex_order": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "ffd_adjoint_forward": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]),
    "ffd_adjoint_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ffd_batch_create": (C.c_int, [C.POINTER(Mesh), C.POINTER(Options), C.c_int32, C.POINTER(C.c_void_p)]),
    "ffd_batch_layout": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "ffd_autotune": (C.c_int, [C.c_void_p, C.c_char_p, C.c_void_p, C.POINTER(C.c_int32)]),
    "ffd_destroy": (None, [C.c_void_p]),
    "ffd_last_error": (C.c_char_p, []),
}


def load(path: str = LIB_PATH):
    """Load libffd.so (built in-tree by paper_2107_05200_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2107_05200_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st: int):
    if st != 0:
        raise FFDError(st, load().ffd_last_error().decode())


def _dptr(t) -> int:
    return 0 if t is None else t.data_ptr()


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _mesh_struct(V: np.ndarray, T: np.ndarray):
    V = np.ascontiguousarray(V, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    ms = Mesh(T.shape[1] - 1, V.shape[1], V.shape[0], T.shape[0],
              V.ctypes.data_as(C.POINTER(C.c_double)), T.ctypes.data_as(C.POINTER(C.c_int32)))
    return ms, (V, T)


def _options_struct(d, energy, rho, pinned_idx, pinned_pos, precision, h_mode, auto_pin, leaf_size):
    pi = np.ascontiguousarray(pinned_idx if pinned_idx is not None else np.zeros(0), dtype=np.int32)
    pp = None if pinned_pos is None else np.ascontiguousarray(pinned_pos, dtype=np.float64).reshape(-1, d)
    op = Options(int(energy), float(rho), int(h_mode), int(precision), pi.shape[0],
                 pi.ctypes.data_as(C.POINTER(C.c_int32)) if pi.size else None,
                 pp.ctypes.data_as(C.POINTER(C.c_double)) if pp is not None and pp.size else None,
                 int(auto_pin), int(leaf_size))
    return op, (pi, pp)


def analyze(V, T, energy=0, rho=10.0, pinned_idx=None, pinned_pos=None, auto_pin=1, leaf_size=0):
    """Host-only set-up statistics and factor self-check (no device)."""
    lib = load()
    ms, keep1 = _mesh_struct(V, T)
    op, keep2 = _options_struct(T.shape[1] - 1, energy, rho, pinned_idx, pinned_pos, 32, 0, auto_pin, leaf_size)
    info = Info()
    res = C.c_double(-1.0)
    _check(lib.ffd_analyze(C.byref(ms), C.byref(op), C.byref(info), C.byref(res)))
    out = info.as_dict()
    out["selfcheck_residual"] = res.value
    return out


def tutte_map(V, T, fixed_idx, fixed_pos, leaf_size=0, stream=None):
    """Minimiser of Tutte's energy with the vertices fixed_idx held at
    fixed_pos (host factor, device solve); returns a (n, d) float64 tensor on
    the current device in the input vertex order."""
    import torch
    lib = load()
    V = np.asarray(V)
    T = np.asarray(T)
    d = T.shape[1] - 1
    ms, keep1 = _mesh_struct(V, T)
    fi = np.ascontiguousarray(fixed_idx, dtype=np.int32)
    fp = np.ascontiguousarray(fixed_pos, dtype=np.float64).reshape(-1, d)
    if fp.shape[0] != fi.shape[0]:
        raise ValueError("fixed_pos needs one row per fixed vertex")
    out = torch.empty((V.shape[0], d), dtype=torch.float64, device=torch.device("cuda", torch.cuda.current_device()))
    _check(lib.ffd_tutte_map(C.byref(ms), fi.shape[0], fi.ctypes.data_as(C.c_void_p), fp.ctypes.data_as(C.c_void_p),
                             int(leaf_size), C.c_void_p(out.data_ptr()), _stream(stream)))
    return out


class Solver:
    """One mesh on the current HIP device.

    precision 32: element steps in float32 (factor, right-hand side, map and
    sums in float64); precision 64: everything float64."""

    def __init__(self, V, T, energy=0, rho=10.0, pinned_idx=None, pinned_pos=None, precision=32,
                 h_mode=0, auto_pin=1, leaf_size=0, constraints=None):
        """constraints: optional (A, c) with A a (rows, n) matrix (dense or
        scipy sparse) and c (rows, d): general linear constraints A W = c."""
        import torch
        self.lib = load()
        V = np.asarray(V)
        T = np.asarray(T)
        self.d = T.shape[1] - 1
        self.din = V.shape[1]
        self.n = V.shape[0]
        self.m = T.shape[0]
        self.precision = precision
        self.dtype = torch.float32 if precision == 32 else torch.float64
        self.n_pinned = 0 if pinned_idx is None else len(pinned_idx)
        ms, keep1 = _mesh_struct(V, T)
        op, keep2 = _options_struct(self.d, energy, rho, pinned_idx, pinned_pos, precision, h_mode,
                                    auto_pin, leaf_size)
        h = C.c_void_p()
        self.n_constraints = 0
        if constraints is None:
            _check(self.lib.ffd_create(C.byref(ms), C.byref(op), C.byref(h)))
        else:
            import scipy.sparse as sp
            A = sp.csr_matrix(constraints[0], dtype=np.float64)
            A.sort_indices()
            rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
            ci = np.ascontiguousarray(A.indices, dtype=np.int32)
            va = np.ascontiguousarray(A.data, dtype=np.float64)
            rh = np.ascontiguousarray(constraints[1], dtype=np.float64).reshape(A.shape[0], self.d)
            con = Constraints(A.shape[0], rp.ctypes.data, ci.ctypes.data, va.ctypes.data, rh.ctypes.data)
            _check(self.lib.ffd_create_constrained(C.byref(ms), C.byref(op), C.byref(con), C.byref(h)))
            self.n_constraints = A.shape[0]
        self.h = h
        if self.n_pinned == 0 and auto_pin and constraints is None:
            self.n_pinned = 1
        self.device = torch.device("cuda", torch.cuda.current_device())

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.ffd_destroy(h)
            self.h = None

    def close(self):
        self.__del__()

    def info(self) -> dict:
        inf = Info()
        _check(self.lib.ffd_get_info(self.h, C.byref(inf)))
        return inf.as_dict()

    def _dev(self, a, dtype):
        import torch
        if isinstance(a, torch.Tensor):
            return a.to(device=self.device, dtype=dtype).contiguous()
        return torch.as_tensor(np.asarray(a), dtype=dtype, device=self.device).contiguous()

    def init(self, map0, stream=None):
        import torch
        x0 = self._dev(map0, torch.float64).reshape(self.n, self.d)
        _check(self.lib.ffd_init(self.h, C.c_void_p(x0.data_ptr()), _stream(stream)))
        self._keep = x0
        return self

    def set_pins(self, pos, stream=None):
        import torch
        p = self._dev(pos, torch.float64).reshape(-1, self.d)
        _check(self.lib.ffd_set_pins(self.h, C.c_void_p(p.data_ptr()), _stream(stream)))
        self._keep_pins = p

    def iterate(self, n_iter: int = 1, stream=None, graph: bool = False):
        """n_iter iterations; graph=True replays a captured HIP graph (same results)."""
        fn = self.lib.ffd_iterate_graph if graph else self.lib.ffd_iterate
        _check(fn(self.h, int(n_iter), _stream(stream)))
        return self

    def iterate_noalloc(self, n_iter: int = 1, stream=None):
        """n_iter iterations with no device allocation (ffd_iterate_noalloc):
        the local step's partial sums use the library's fixed scratch."""
        _check(self.lib.ffd_iterate_noalloc(self.h, int(n_iter), _stream(stream)))
        return self

    def iterate_until(self, max_iter: int, check_every: int = 10, eps_abs: float = 1e-6, eps_rel: float = 1e-5,
                      flip_free: bool = True, graph: bool = True, stream=None):
        """Iterate until the thresholds of eq. primaldualthresholds hold at a
        check (every check_every iterations) or max_iter is reached; returns
        (iterations run, converged)."""
        done, conv = C.c_int32(0), C.c_int32(0)
        _check(self.lib.ffd_iterate_until(self.h, int(max_iter), int(check_every), float(eps_abs), float(eps_rel),
                                          int(bool(flip_free)), int(bool(graph)), _stream(stream),
                                          C.byref(done), C.byref(conv)))
        return done.value, bool(conv.value)

    def set_constraint_rhs(self, c, stream=None):
        """New right-hand sides c (rows, d) of the general constraints."""
        import torch
        cs = self._dev(c, torch.float64).reshape(self.n_constraints, self.d)
        _check(self.lib.ffd_set_constraint_rhs(self.h, C.c_void_p(cs.data_ptr()), _stream(stream)))
        self._keep_rhs = cs
        return self

    def set_refactor_mode(self, device: bool):
        """Refactorise the top fronts on the device (True) or on the host."""
        _check(self.lib.ffd_set_refactor_mode(self.h, int(bool(device))))
        return self

    def rescale(self, rho_r: float = 5.0, stream=None):
        """One penalty rescaling event (new per-element mu, Lambda, factor)."""
        _check(self.lib.ffd_rescale(self.h, float(rho_r), _stream(stream)))
        return self

    def run(self, max_iter: int, check_every: int = 10, eps_abs: float = 1e-6, eps_rel: float = 1e-5,
            flip_free: bool = True, rescale_rho: float = 5.0, graph: bool = True, stream=None):
        """Algorithm 2 (rescaling schedule and termination test); returns
        (iterations run, converged, rescaling events)."""
        done, conv, nres = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        _check(self.lib.ffd_run(self.h, int(max_iter), int(check_every), float(eps_abs), float(eps_rel),
                                int(bool(flip_free)), float(rescale_rho), int(bool(graph)), _stream(stream),
                                C.byref(done), C.byref(conv), C.byref(nres)))
        return done.value, bool(conv.value), nres.value

    def iterate_profiled(self, n_iter: int, stream=None) -> dict:
        """Iterate with per-phase HIP events; returns summed milliseconds per phase."""
        out = (C.c_double * 6)()
        _check(self.lib.ffd_iterate_profiled(self.h, int(n_iter), _stream(stream), out))
        names = ("wrhs", "solve_fwd", "solve_bwd", "local", "finalize", "total")
        return {k: out[i] for i, k in enumerate(names)}

    def profile_solve_levels(self, n_rep: int = 10, stream=None) -> list:
        """Per-level timing of both triangular-solve passes (ffd_profile_solve_levels):
        one dict per level from the leaves up."""
        cap = 64
        out = (C.c_double * (cap * 10))()
        nl = C.c_int32(0)
        _check(self.lib.ffd_profile_solve_levels(self.h, int(n_rep), _stream(stream), out, cap, C.byref(nl)))
        names = ("fwd_ms", "bwd_ms", "bytes", "nodes", "c_max", "r_max", "fwd_tasks", "bwd_tasks",
                 "fwd_reduce_tasks", "bwd_reduce_tasks")
        return [{k: out[l * 10 + i] for i, k in enumerate(names)} for l in range(nl.value)]

    def get_state(self, stream=None):
        """Returns dict of device tensors: map (n, d) float64; U, P, Lam, Wel (m, d, d)."""
        import torch
        d, m = self.d, self.m
        out = {"map": torch.empty((self.n, d), dtype=torch.float64, device=self.device)}
        for k in ("Wel", "U", "P", "Lam"):
            out[k] = torch.empty((m, d, d), dtype=self.dtype, device=self.device)
        _check(self.lib.ffd_get_state(self.h, C.c_void_p(out["map"].data_ptr()),
                                      C.c_void_p(out["Wel"].data_ptr()), C.c_void_p(out["U"].data_ptr()),
                                      C.c_void_p(out["P"].data_ptr()), C.c_void_p(out["Lam"].data_ptr()),
                                      _stream(stream)))
        return out

    def set_state(self, x, U, P, Lam, k: int = 0, stream=None):
        import torch
        xs = self._dev(x, torch.float64).reshape(self.n, self.d)
        Us = self._dev(U, self.dtype).reshape(self.m, self.d, self.d)
        Ps = self._dev(P, self.dtype).reshape(self.m, self.d, self.d)
        Ls = self._dev(Lam, self.dtype).reshape(self.m, self.d, self.d)
        _check(self.lib.ffd_set_state(self.h, C.c_void_p(xs.data_ptr()), C.c_void_p(Us.data_ptr()),
                                      C.c_void_p(Ps.data_ptr()), C.c_void_p(Ls.data_ptr()), int(k),
                                      _stream(stream)))
        self._keep_state = (xs, Us, Ps, Ls)

    def iteration(self) -> int:
        k = C.c_int64()
        _check(self.lib.ffd_get_iteration(self.h, C.byref(k)))
        return k.value

    def history(self, first: int = 0, count: int | None = None) -> np.ndarray:
        if count is None:
            count = self.iteration() - first
        out = np.empty((count, HIST_FIELDS), dtype=np.float64)
        _check(self.lib.ffd_get_history(self.h, first, count, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def vertex_order(self) -> np.ndarray:
        o = np.empty(self.n, dtype=np.int32)
        _check(self.lib.ffd_get_vertex_order(self.h, o.ctypes.data_as(C.POINTER(C.c_int32))))
        return o

    def autotune(self, cache_path: str | None = None, stream=None) -> dict:
        """Pick launch shapes by timing them (state saved and restored)."""
        out = (C.c_int32 * 6)()
        _check(self.lib.ffd_autotune(self.h, cache_path.encode() if cache_path else None, _stream(stream), out))
        return {"local_block": out[0], "wrhs_lanes": out[1], "solve_wave_levels": out[2],
                "solve_split_levels": out[3], "solve_streams": out[4], "solve_top_level": out[5]}

    def adjoint_forward(self, n_iter: int, checkpoint_every: int = 10, stream=None):
        """n_iter iterations with checkpoints every checkpoint_every (for adjoint_backward)."""
        _check(self.lib.ffd_adjoint_forward(self.h, int(n_iter), int(checkpoint_every), _stream(stream)))
        return self

    def adjoint_backward(self, Pbar=None, energy_loss: bool = True, stream=None):
        """Gradients (pins_bar (n_pinned, d), V_bar (n, d), float64 device tensors) of
        sum_i w_i f(P_i^K) (energy_loss) plus <Pbar, P^K> through the last adjoint_forward.
        V_bar is None for a surface map (rest vertices in 3D, map in 2D)."""
        import torch
        pb = torch.zeros((max(self.n_pinned, 1), self.d), dtype=torch.float64, device=self.device)
        vb = torch.zeros((self.n, self.d), dtype=torch.float64, device=self.device) if self.din == self.d else None
        Pt = None if Pbar is None else self._dev(Pbar, self.dtype).reshape(self.m, self.d, self.d)
        _check(self.lib.ffd_adjoint_backward(self.h, C.c_void_p(_dptr(Pt)), int(bool(energy_loss)),
                                             C.c_void_p(pb.data_ptr()), C.c_void_p(_dptr(vb)),
                                             _stream(stream)))
        return pb[: self.n_pinned], vb

    def solve(self, b, stream=None):
        """x = L_FF^{-1} b in the internal free-vertex order (n_free, d) float64."""
        import torch
        bb = self._dev(b, torch.float64).reshape(-1, self.d)
        x = torch.zeros((self.n, self.d), dtype=torch.float64, device=self.device)
        _check(self.lib.ffd_solve(self.h, C.c_void_p(bb.data_ptr()), C.c_void_p(x.data_ptr()), _stream(stream)))
        return x[: bb.shape[0]]


class BatchSolver(Solver):
    """Many meshes in one handle (ffd_batch_create): arrays are the meshes'
    arrays concatenated in order; ``layout()`` gives the offsets."""

    def __init__(self, workloads, precision=32, h_mode=0, leaf_size=0):
        import torch
        self.lib = load()
        ws = list(workloads)
        self.d = ws[0].T.shape[1] - 1
        self.din = ws[0].V.shape[1]
        self.n = int(sum(w.V.shape[0] for w in ws))
        self.m = int(sum(w.T.shape[0] for w in ws))
        self.precision = precision
        self.dtype = torch.float32 if precision == 32 else torch.float64
        meshes = (Mesh * len(ws))()
        opts = (Options * len(ws))()
        keep = []
        npin = 0
        for i, w in enumerate(ws):
            ms, k1 = _mesh_struct(w.V, w.T)
            op, k2 = _options_struct(self.d, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision, h_mode, 1,
                                     leaf_size)
            meshes[i] = ms
            opts[i] = op
            keep += [k1, k2]
            npin += len(w.pinned_idx) if len(w.pinned_idx) else 1
        h = C.c_void_p()
        _check(self.lib.ffd_batch_create(meshes, opts, len(ws), C.byref(h)))
        self.h = h
        self.n_pinned = npin
        self.n_meshes = len(ws)
        self.device = torch.device("cuda", torch.cuda.current_device())

    def layout(self):
        vo = np.empty(self.n_meshes + 1, dtype=np.int64)
        eo = np.empty(self.n_meshes + 1, dtype=np.int64)
        _check(self.lib.ffd_batch_layout(self.h, vo.ctypes.data_as(C.POINTER(C.c_int64)),
                                         eo.ctypes.data_as(C.POINTER(C.c_int64))))
        return vo, eo
