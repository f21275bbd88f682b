"""Replayed HIP graphs of the iteration (ffd_iterate_graph) against direct
launches (ffd_iterate): bitwise equal states and history records after every
group of replays, with direct iterations, synchronisations and schedule
changes between the groups."""
import sys

import numpy as np
import pytest

from paper_2107_05200_amd import meshgen as mg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _state(s):
    import torch
    st = {k: v.cpu().numpy() for k, v in s.get_state().items()}
    torch.cuda.synchronize()
    return st


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("case", ["cube_fp32", "height_field_fp64", "batch_fp32"])
def test_graph_replays_match_direct_launches(gpu_lib, case, tmp_path):
    import torch
    from paper_2107_05200_amd.binding import BatchSolver, Solver
    if case == "batch_fp32":
        ws = mg.batched_charts(n_charts=5, seed_c=3, m_lo=200.0, m_hi=2000.0)
        x0 = np.concatenate([w.x0 for w in ws])
        mk = lambda: BatchSolver(ws, precision=32)
    else:
        w = mg.twisted_cube(7) if case == "cube_fp32" else mg.height_field_uv()
        prec = 32 if case == "cube_fp32" else 64
        x0 = w.x0
        mk = lambda: Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=prec)
    say(f"case: graph replay {case}")
    a, b = mk(), mk()
    a.init(x0)
    b.init(x0)
    # groups of replays with direct work and synchronisations in between
    for n_graph, n_direct in ((6, 0), (5, 1), (8, 3), (2, 0), (7, 2)):
        a.iterate(n_graph)
        b.iterate(n_graph, graph=True)
        torch.cuda.synchronize()
        _same(_state(a), _state(b))
        assert np.array_equal(a.history(), b.history(), equal_nan=True)
        if n_direct:
            a.iterate(n_direct)
            b.iterate(n_direct)
    # a schedule change re-captures the graph
    cache = str(tmp_path / "tune.txt")
    a.autotune(cache)
    b.autotune(cache)
    a.iterate(9)
    b.iterate(9, graph=True)
    _same(_state(a), _state(b))
    assert np.array_equal(a.history(), b.history(), equal_nan=True)
    assert a.iteration() == b.iteration()


def test_graph_recaptured_when_history_grows(gpu_lib):
    """The first replays write into the initial history buffer; a call that
    needs a larger one re-captures the graph against the new buffer."""
    import torch
    from paper_2107_05200_amd.binding import Solver
    w = mg.height_field_uv()
    say("case: graph replay across a history reallocation")
    a = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32)
    b = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32)
    a.init(w.x0)
    b.init(w.x0)
    a.iterate(100)
    b.iterate(100, graph=True)
    a.iterate(16350)
    b.iterate(16350, graph=True)
    torch.cuda.synchronize()
    _same(_state(a), _state(b))
    ha, hb = a.history(), b.history()
    assert ha.shape == hb.shape == (16450, hb.shape[1])
    assert np.array_equal(ha, hb, equal_nan=True)


def _with_streams(line, groups, top):
    """the same cached choice with another stream count and top level"""
    f = line.split()
    f[4], f[5] = str(groups), str(top)
    return " ".join(f) + "\n"


@pytest.mark.parametrize("case", ["cube", "batch"])
def test_solve_streams_are_invisible(gpu_lib, case, tmp_path):
    """Spreading the subtrees below a top level over several streams changes
    only the launch order: states and history are bitwise those of one
    stream, for direct launches and for replayed graphs."""
    import torch
    from paper_2107_05200_amd.binding import BatchSolver, Solver
    if case == "batch":
        ws = mg.batched_charts(n_charts=7, seed_c=5, m_lo=200.0, m_hi=3000.0)
        x0 = np.concatenate([w.x0 for w in ws])
        mk = lambda: BatchSolver(ws, precision=32)
    else:
        w = mg.twisted_cube(9)
        x0 = w.x0
        mk = lambda: Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32)
    say(f"case: solve streams {case}")
    base = str(tmp_path / "tune0.txt")
    s0 = mk()
    s0.init(x0)
    s0.autotune(base)
    line = open(base).read().strip().splitlines()[-1]
    nlev = int(line.split()[3])
    ref = None
    for groups, top in ((1, nlev), (2, nlev - 1), (3, max(1, nlev - 3)), (4, max(1, nlev - 2))):
        c = str(tmp_path / f"tune_{groups}_{top}.txt")
        open(c, "w").write(_with_streams(line, groups, top))
        for graph in (False, True):
            s = mk()
            s.init(x0)
            ch = s.autotune(c)
            assert ch["solve_streams"] == groups and ch["solve_top_level"] == (top if groups > 1 else nlev)
            s.iterate(11, graph=graph)
            x = s.solve(torch.ones((s.info()["n_free"], s.d), dtype=torch.float64, device="cuda"))
            st = _state(s)
            st["solve"] = x.cpu().numpy()
            st["hist"] = s.history()
            if ref is None:
                ref = st
            else:
                _same(ref, st)


def _forced(line, fwd, bwd):
    """the cached choice with every level's (mode, outputs, chunk, waves, deferred) replaced"""
    f = line.split()
    nlev = int(f[3])
    head = f[:6]
    return " ".join(head + list(map(str, fwd)) * nlev + list(map(str, bwd)) * nlev) + "\n"


@pytest.mark.parametrize("fwd,bwd", [((0, 64, 256, 4, 1), (0, 64, 256, 4, 0)),
                                     ((0, 32, 256, 8, 0), (0, 16, 256, 16, 0)),
                                     ((0, 16, 512, 4, 1), (1, 32, 0, 4, 0)),
                                     ((0, 64, 256, 4, 1), (0, 64, 256, 4, 1)),
                                     ((0, 32, 256, 8, 0), (0, 16, 256, 16, 1))])
def test_forced_split_schedules(gpu_lib, fwd, bwd, tmp_path):
    """Every level split (forward partials added right away or by the backward
    pass): the solve matches SciPy's sparse LU and twelve iterations match
    the default schedule to rounding."""
    import torch
    import scipy.sparse.linalg as spla
    from paper_2107_05200_amd.binding import Solver
    import oracle as O
    w = mg.twisted_cube(9)
    say(f"case: forced schedule fwd {fwd} bwd {bwd}")
    base = str(tmp_path / "t0.txt")
    a = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=64)
    a.init(w.x0)
    a.autotune(base)
    line = open(base).read().strip().splitlines()[-1]
    c = str(tmp_path / "t1.txt")
    open(c, "w").write(_forced(line, fwd, bwd))
    b = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=64)
    b.init(w.x0)
    b.autotune(c)
    # the solve against SciPy's sparse LU of the oracle's L_FF, in the
    # library's internal vertex order
    order = b.vertex_order()
    nF = w.n - len(w.pinned_idx)
    B, wt = O.element_geometry(w.V, w.T)
    L = O.global_matrix(O.gradient_operator(B, w.T, w.n), w.rho * wt, w.d)
    LFF = L[order[:nF]][:, order[:nF]].tocsc()
    rng = np.random.default_rng(0)
    rhs = rng.normal(size=(nF, w.d))
    x = b.solve(torch.tensor(rhs, device="cuda")).cpu().numpy()
    ref = spla.splu(LFF).solve(rhs)
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    say(f"  solve rel err {err:.2e}")
    assert err < 1e-10
    a2 = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=64)
    a2.init(w.x0)
    a2.iterate(12)
    b.iterate(12)
    sa, sb = _state(a2), _state(b)
    for k in sa:
        nrm = np.linalg.norm(np.nan_to_num(sa[k]))
        assert np.linalg.norm(np.nan_to_num(sa[k]) - np.nan_to_num(sb[k])) <= 1e-10 * max(nrm, 1e-300), k


@pytest.mark.parametrize("case", ["cube", "batch"])
def test_deferred_backward_reductions_are_invisible(gpu_lib, case, tmp_path):
    """Backward split levels that leave their chunk partials to the next
    backward launch (which reads the pending rows from them and writes the
    rows) give bitwise the states, history and solves of the same split
    schedule reduced after every level: one stream and several, direct
    launches and replayed graphs."""
    import torch
    from paper_2107_05200_amd.binding import BatchSolver, Solver
    if case == "batch":
        ws = mg.batched_charts(n_charts=7, seed_c=5, m_lo=200.0, m_hi=3000.0)
        x0 = np.concatenate([w.x0 for w in ws])
        mk = lambda: BatchSolver(ws, precision=32)
    else:
        w = mg.twisted_cube(9)
        x0 = w.x0
        mk = lambda: Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32)
    say(f"case: deferred backward reductions {case}")
    base = str(tmp_path / "tune0.txt")
    s0 = mk()
    s0.init(x0)
    s0.autotune(base)
    line0 = open(base).read().strip().splitlines()[-1]
    nlev = int(line0.split()[3])
    ref = None
    for defer in (0, 1):
        line = _forced(line0, (0, 64, 256, 4, 1), (0, 32, 256, 4, defer)).strip()
        for groups, top in ((1, nlev), (2, nlev - 1), (3, max(1, nlev - 3))):
            c = str(tmp_path / f"tune_{defer}_{groups}_{top}.txt")
            open(c, "w").write(_with_streams(line, groups, top))
            for graph in (False, True):
                s = mk()
                s.init(x0)
                s.autotune(c)
                s.iterate(11, graph=graph)
                x = s.solve(torch.ones((s.info()["n_free"], s.d), dtype=torch.float64, device="cuda"))
                st = _state(s)
                st["solve"] = x.cpu().numpy()
                st["hist"] = s.history()
                if ref is None:
                    ref = st
                else:
                    _same(ref, st)


@pytest.mark.parametrize("case", ["adjoint_disk", "constrained_cube"])
def test_deferred_backward_reductions_in_adjoint_and_constraints(gpu_lib, case, tmp_path):
    """The adjoint's solves and the constrained W-step run the same backward
    launches: with every split backward level deferred, the gradients (disk,
    float64) and the constrained iterations (cube, float32) are bitwise those
    of the same split schedule reduced after every level."""
    import torch
    from paper_2107_05200_amd.binding import Solver
    if case == "adjoint_disk":
        w = mg.disk_deformation(R=24)
        mk = lambda: Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=64)
        x0 = w.V
    else:
        w = mg.twisted_cube(8)
        rng = np.random.default_rng(3)
        v = rng.choice(np.setdiff1d(np.arange(w.n), w.pinned_idx), size=6, replace=False)
        A = np.zeros((2, w.n))
        A[0, v[:3]] = [1.0, -0.5, -0.5]
        A[1, v[3:]] = 1.0 / 3.0
        c = np.stack([np.zeros(3), w.V[v[3:]].mean(axis=0) + 0.01])
        mk = lambda: Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32, constraints=(A, c))
        x0 = w.x0
    say(f"case: deferred backward reductions, {case}")
    base = str(tmp_path / "tune0.txt")
    s0 = mk()
    s0.init(x0)
    s0.autotune(base)
    line0 = open(base).read().strip().splitlines()[-1]
    out = []
    for defer in (0, 1):
        c_path = str(tmp_path / f"tune_{defer}.txt")
        open(c_path, "w").write(_forced(line0, (0, 64, 256, 4, 1), (0, 16, 256, 4, defer)))
        s = mk()
        s.init(x0)
        s.autotune(c_path)
        if case == "adjoint_disk":
            s.init(x0).adjoint_forward(12, 4)
            pb, vb = s.adjoint_backward(energy_loss=True)
            torch.cuda.synchronize()
            out.append({"pins_bar": pb.cpu().numpy(), "V_bar": vb.cpu().numpy()})
        else:
            s.iterate(9)
            st = _state(s)
            st["hist"] = s.history()
            out.append(st)
    _same(out[0], out[1])
