"""Degenerate inputs of the iteration on the device against the oracle
(float64, 1e-9 relative on the map and W_el): a single triangle and a single
tetrahedron with one free vertex, a mesh whose every vertex is fixed (no
W-step unknowns), a fixed vertex that no element uses, and flipped
elements in the initial map of a tiny mesh."""
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
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _run_both(V, T, energy, pins, pos, x0, iters=15, prec=64):
    import torch
    from paper_2107_05200_amd.binding import Solver
    g = Solver(V, T, energy, 10.0, pins, pos, precision=prec)
    g.init(x0).iterate(iters)
    st = g.get_state()
    torch.cuda.synchronize()
    r = O.OracleSolver(V, T, energy, 10.0, pins, pos)
    r.init(x0)
    r.iterate(iters)
    ex = rel(st["map"].cpu().numpy(), r.x)
    ew = rel(st["Wel"].cpu().numpy(), r.wel())
    h, hr = g.history(), r.history.array()
    return ex, ew, h, hr


@pytest.mark.parametrize("energy", [mg.SYMMETRIC_DIRICHLET, mg.SYMMETRIC_GRADIENT])
def test_single_triangle_and_tetrahedron(gpu_lib, energy):
    V2 = np.array([[0.0, 0.0], [1.0, 0.0], [0.2, 0.9]])
    T2 = np.array([[0, 1, 2]], dtype=np.int32)
    x2 = np.array([[0.0, 0.0], [1.3, 0.1], [0.5, -0.4]])  # flipped at the start
    V3 = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.1, 0.2, 0.8]])
    T3 = np.array([[0, 1, 2, 3]], dtype=np.int32)
    x3 = V3 * np.array([1.2, 0.9, 1.0]) + np.array([0.0, 0.0, 0.3]) * (np.arange(4) == 3)[:, None]
    for V, T, x0, pins in ((V2, T2, x2, [0, 1]), (V3, T3, x3, [0, 1, 2])):
        say(f"case: single element d={T.shape[1] - 1} energy={energy}")
        ex, ew, h, hr = _run_both(V, T, energy, np.array(pins, dtype=np.int32), x0[pins], x0)
        say(f"  map {ex:.2e} Wel {ew:.2e}")
        assert ex < 1e-9 and ew < 1e-9
        assert np.allclose(h[:, 0], hr[:, 0], rtol=1e-8, atol=1e-14)


def test_every_vertex_fixed(gpu_lib):
    """No free vertex: the W-step returns the fixed positions and the local
    steps still run."""
    w = mg.height_field_uv(grid=6)
    pins = np.arange(w.n, dtype=np.int32)
    rng = np.random.default_rng(1)
    pos = w.V[:, :2] * 1.1 + rng.normal(0.0, 0.01, size=(w.n, 2))
    say(f"case: every vertex fixed, n={w.n}")
    ex, ew, h, hr = _run_both(w.V, w.T, w.energy, pins, pos, pos)
    say(f"  map {ex:.2e} Wel {ew:.2e}")
    assert ex < 1e-12 and ew < 1e-9


def test_fixed_vertex_outside_the_mesh(gpu_lib):
    """A fixed vertex that no element uses changes nothing else."""
    w = mg.height_field_uv(grid=8)
    V = np.vstack([w.V, [[5.0, 5.0, 0.0]]])
    pins = np.append(w.pinned_idx, w.n).astype(np.int32)
    pos = np.vstack([w.pinned_pos, [[5.0, 5.0]]])
    x0 = np.vstack([w.x0, [[5.0, 5.0]]])
    say("case: fixed vertex outside the mesh")
    ex, ew, h, hr = _run_both(V, w.T, w.energy, pins, pos, x0)
    say(f"  map {ex:.2e} Wel {ew:.2e}")
    assert ex < 1e-9 and ew < 1e-9
