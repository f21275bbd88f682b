"""General linear constraints A W = c on the device (ffd_create_constrained)
against the oracle's KKT W-step.

Float64: 1e-9 relative on the map over free-running iterations and A W = c
to 1e-10; float32 element steps: 1e-5.  Pins written as constraint rows give
the pinned solver's iterations; graph replay is bitwise; new right-hand
sides, rescaling events and the error paths are covered."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2107_05200_amd import meshgen as mg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def relational_rows(n, d, seed, k=3, exclude=()):
    """k groups of three rows: a vertex at a fixed affine combination of two
    others, a fixed difference of two vertices, the centroid of three."""
    rng = np.random.default_rng(seed)
    pool = np.setdiff1d(np.arange(n), np.asarray(exclude, dtype=np.int64))
    v = rng.choice(pool, size=7 * k, replace=False)
    rows, cs = [], []
    for i in range(k):
        a, b, c_ = v[7 * i:7 * i + 3]
        t = rng.uniform(0.2, 0.8)
        row = np.zeros(n)
        row[a], row[b], row[c_] = 1.0, -t, -(1 - t)
        rows.append(row)
        cs.append(rng.normal(size=d) * 0.05)
        row = np.zeros(n)
        row[v[7 * i + 3]], row[v[7 * i + 4]] = 1.0, -1.0
        rows.append(row)
        cs.append(rng.normal(size=d) * 0.2)
        row = np.zeros(n)
        row[v[7 * i + 4:7 * i + 7]] = 1.0 / 3.0
        rows.append(row)
        cs.append(rng.normal(size=d) * 0.3 + 0.5)
    return np.array(rows), np.array(cs)


def _pair(w, prec, A, c, pins=True, h_mode=0):
    from paper_2107_05200_amd.binding import Solver
    pi, pp = (w.pinned_idx, w.pinned_pos) if pins else ([], None)
    g = Solver(w.V, w.T, w.energy, w.rho, pi, pp, precision=prec, h_mode=h_mode, constraints=(A, c))
    r = O.OracleSolver(w.V, w.T, w.energy, w.rho, pi, pp, h_mode=h_mode, constraints=(A, c))
    g.init(w.x0)
    r.init(w.x0)
    return g, r


CASES = {
    "height_field_pins_fp64": (lambda: mg.height_field_uv(), 64, True, 3, 1e-9),
    "disk_no_pins_fp64": (lambda: mg.disk_deformation(R=12), 64, False, 2, 1e-9),
    "cube6_pins_fp64": (lambda: mg.twisted_cube(6), 64, True, 3, 1e-9),
    "cube6_pins_fp32": (lambda: mg.twisted_cube(6), 32, True, 3, 1e-5),
    "sphere_cap_sg_fp32": (lambda: mg.sphere_cap_uv(R=12), 32, True, 2, 1e-5),
}


@pytest.mark.parametrize("name", list(CASES))
def test_constrained_iterations_match_oracle(gpu_lib, name):
    import torch
    mk, prec, pins, k, tol = CASES[name]
    w = mk()
    A, c = relational_rows(w.n, w.d, seed=len(name), k=k, exclude=w.pinned_idx)
    say(f"case: constrained {name} n={w.n} rows={A.shape[0]} pins={pins}")
    g, r = _pair(w, prec, A, c, pins=pins)
    worst = worst_c = 0.0
    for it in range(3):
        g.iterate(10)
        r.iterate(10)
        st = g.get_state()
        torch.cuda.synchronize()
        x = host(st["map"])
        worst = max(worst, rel(x, r.x))
        worst_c = max(worst_c, np.max(np.abs(A @ x - c)))
    say(f"  worst rel err map {worst:.2e}, worst |A W - c| {worst_c:.2e}")
    assert worst < tol
    assert worst_c < 1e-10
    h, hr = g.history(), r.history.array()
    assert np.allclose(h[:, 0], hr[:, 0], rtol=100 * tol, atol=1e-12)


def test_pins_as_rows_match_pinned_solver(gpu_lib):
    """Pins eliminated from the factor and the same pins written as rows of a
    constraint system (no pinned vertex) run the same iterations."""
    import torch
    from paper_2107_05200_amd.binding import Solver
    w = mg.height_field_uv()
    say("case: pins as constraint rows (height field fp64)")
    a = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=64)
    A = np.zeros((len(w.pinned_idx), w.n))
    A[np.arange(len(w.pinned_idx)), w.pinned_idx] = 1.0
    b = Solver(w.V, w.T, w.energy, w.rho, [], None, precision=64, constraints=(A, w.pinned_pos))
    a.init(w.x0).iterate(40)
    b.init(w.x0).iterate(40)
    sa, sb = a.get_state(), b.get_state()
    torch.cuda.synchronize()
    e = rel(host(sb["map"]), host(sa["map"]))
    say(f"  rel diff {e:.2e}")
    assert e < 1e-10


def test_graph_replay_and_new_rhs(gpu_lib):
    """Replayed graphs give the direct launches' iterations bit for bit, and
    a new right-hand side mid-run follows the oracle."""
    import torch
    from paper_2107_05200_amd.binding import Solver
    w = mg.twisted_cube(6)
    A, c = relational_rows(w.n, 3, seed=21, k=2, exclude=w.pinned_idx)
    say("case: constrained graph replay and new right-hand sides (cube6 fp64)")
    g1 = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=64, constraints=(A, c))
    g2 = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=64, constraints=(A, c))
    g1.init(w.x0).iterate(12)
    g2.init(w.x0).iterate(12, graph=True)
    s1, s2 = g1.get_state(), g2.get_state()
    torch.cuda.synchronize()
    for k in ("map", "U", "P", "Lam"):
        assert torch.equal(s1[k], s2[k]), k
    r = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, constraints=(A, c))
    r.init(w.x0)
    r.iterate(12)
    c2 = c + 0.1
    g2.set_constraint_rhs(c2)
    r.set_constraint_rhs(c2)
    g2.iterate(8, graph=True)
    r.iterate(8)
    x = host(g2.get_state()["map"])
    torch.cuda.synchronize()
    e = rel(x, r.x)
    say(f"  after the new right-hand side: rel err {e:.2e}, |A W - c2| {np.max(np.abs(A @ x - c2)):.2e}")
    assert e < 1e-9 and np.max(np.abs(A @ x - c2)) < 1e-10


def test_rescaling_with_constraints(gpu_lib):
    """Rescaling events refactorise L + gamma A^T A and rebuild Z and S^{-1}:
    the iterations after two events still follow the oracle."""
    import torch
    w = mg.height_field_uv()
    A, c = relational_rows(w.n, 2, seed=33, k=2, exclude=w.pinned_idx)
    say("case: rescaling with constraints (height field fp64)")
    g, r = _pair(w, 64, A, c)
    for n_before in (4, 3):
        g.iterate(n_before)
        r.iterate(n_before)
        g.rescale(5.0)
        r.rescale(5.0)
    g.iterate(10)
    r.iterate(10)
    x = host(g.get_state()["map"])
    torch.cuda.synchronize()
    e = rel(x, r.x)
    say(f"  rel err {e:.2e}")
    assert e < 1e-9 and np.max(np.abs(A @ x - c)) < 1e-10


def test_constraint_errors(gpu_lib):
    from paper_2107_05200_amd.binding import FFDError, Solver
    w = mg.height_field_uv()
    A, c = relational_rows(w.n, 2, seed=2, k=1, exclude=w.pinned_idx)

    def make(A_, c_, pins=True):
        pi, pp = (w.pinned_idx, w.pinned_pos) if pins else ([], None)
        return Solver(w.V, w.T, w.energy, w.rho, pi, pp, precision=64, constraints=(A_, c_))

    with pytest.raises(FFDError):
        make(np.vstack([A, A[:1]]), np.vstack([c, c[:1]]))  # dependent rows
    only_pins = np.zeros((1, w.n))
    only_pins[0, w.pinned_idx] = 1.0
    with pytest.raises(FFDError):
        make(np.vstack([A, only_pins]), np.vstack([c, [[0.0, 0.0]]]))  # a row on pinned vertices only
    diff = np.zeros((1, w.n))
    diff[0, [3, 9]] = [1.0, -1.0]
    with pytest.raises(FFDError):
        make(diff, [[0.1, 0.0]], pins=False)  # the translation stays free
    with pytest.raises(FFDError):
        big = np.zeros((1025, w.n))
        big[np.arange(1025), np.arange(1025) % w.n] = 1.0
        make(big, np.zeros((1025, 2)), pins=False)
    g = make(A, c)
    g.init(w.x0)
    with pytest.raises(FFDError):
        g.adjoint_forward(3)
    g.iterate(2)
    assert g.iteration() == 2
