"""Tutte initial maps on the device (ffd_tutte_map) against the oracle.

The device factorises the edge Laplacian of Tutte's energy with the W-step's
host factorisation and solves it with the W-step's solve kernels (float64):
1e-10 relative to the oracle's sparse LU solution at oracle sizes; at the
sphere cap's full size (501,126 triangles) the residual of the oracle's
Laplacian at the device map, Tutte's theorem (no flipped triangle) and an
ADMM run started from it."""
import sys
import time

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


def _orient2(W, T):
    e1 = W[T[:, 1]] - W[T[:, 0]]
    e2 = W[T[:, 2]] - W[T[:, 0]]
    return e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]


def _twisted_boundary(V, idx, twist_deg=45.0):
    """The cube's boundary vertices rotated about the vertical axis through the
    centre by twist_deg * z (a target surface for a volume map)."""
    P = V[idx]
    a = np.deg2rad(twist_deg) * P[:, 2]
    x, y = P[:, 0] - 0.5, P[:, 1] - 0.5
    return np.stack([0.5 + np.cos(a) * x - np.sin(a) * y, 0.5 + np.sin(a) * x + np.cos(a) * y, P[:, 2]], axis=1)


CASES = {
    "height_field_circle": lambda: (lambda w: (w.V, w.T) + mg.circle_boundary(w.V, w.T))(mg.height_field_uv()),
    "sphere_cap_R40_circle": lambda: (lambda w: (w.V, w.T) + mg.circle_boundary(w.V, w.T))(mg.sphere_cap_uv(R=40)),
    "disk_R30_circle": lambda: (lambda w: (w.V, w.T) + mg.circle_boundary(w.V, w.T))(mg.disk_deformation(R=30)),
    "cube10_twisted_surface": lambda: (lambda V, T: (V, T, mg.boundary_vertices(T),
                                                     _twisted_boundary(V, mg.boundary_vertices(T))))(
        *mg.kuhn_cube(10)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_tutte_map_matches_oracle(gpu_lib, name):
    import torch
    from paper_2107_05200_amd.binding import tutte_map
    V, T, idx, pos = CASES[name]()
    say(f"case: Tutte map {name} n={V.shape[0]} m={T.shape[0]} fixed={len(idx)}")
    W = tutte_map(V, T, idx, pos)
    torch.cuda.synchronize()
    W = W.cpu().numpy()
    ref = O.tutte.tutte_map(V, T, idx, pos)
    e = rel(W, ref)
    say(f"  rel err vs oracle {e:.2e}")
    assert e < 1e-10
    assert np.array_equal(W[idx], pos)
    if T.shape[1] == 3:
        assert _orient2(W, T).min() > 0


def test_tutte_map_sphere_cap_full_size(gpu_lib):
    """The sphere cap at its full size (R = 289): residual of the oracle's
    Laplacian below 1e-10, no flipped triangle, then 500 iterations of the
    symmetric gradient ADMM from it end flip-free with a finite energy."""
    import torch
    import scipy.sparse  # noqa: F401
    from paper_2107_05200_amd.binding import Solver, tutte_map
    w = mg.sphere_cap_uv()
    idx, pos = mg.circle_boundary(w.V, w.T)
    say(f"case: Tutte map sphere cap R=289 m={w.m} fixed={len(idx)}")
    t0 = time.perf_counter()
    Wd = tutte_map(w.V, w.T, idx, pos)
    torch.cuda.synchronize()
    say(f"  ffd_tutte_map {time.perf_counter() - t0:.2f} s (host factor + device solve)")
    W = Wd.cpu().numpy()
    K = O.tutte.tutte_laplacian(w.V, w.T).tocsr()
    free = np.setdiff1d(np.arange(w.n), idx)
    res = K[free] @ W
    scale = np.linalg.norm(K[free][:, idx] @ pos)
    say(f"  relative residual {np.linalg.norm(res) / scale:.2e}")
    assert np.linalg.norm(res) / scale < 1e-10
    assert _orient2(W, w.T).min() > 0
    g = Solver(w.V, w.T, w.energy, w.rho, idx[:1], W[idx[:1]], precision=32)
    g.init(Wd)
    g.iterate(w.iters, graph=True)
    h = g.history()
    say(f"  after {w.iters} iterations: flips {h[-1, 5]:.0f} E_map {h[-1, 3]:.6g} e_prim {h[-1, 0]:.3e}")
    assert h[-1, 5] == 0 and np.isfinite(h[-1, 3])
    assert h[-1, 3] <= h[0, 3]


def test_tutte_map_errors(gpu_lib):
    from paper_2107_05200_amd.binding import FFDError, tutte_map
    w = mg.height_field_uv()
    idx, pos = mg.circle_boundary(w.V, w.T)
    with pytest.raises(FFDError):
        tutte_map(w.V, w.T, idx[:0], pos[:0])  # nothing fixed
    V2 = np.concatenate([w.V, w.V + 5.0])
    T2 = np.concatenate([w.T, w.T + w.n])
    with pytest.raises(FFDError):
        tutte_map(V2, T2, idx, pos)  # the second component has no fixed vertex
    V3 = w.V.copy()
    V3[w.T[0, 1]] = V3[w.T[0, 0]]
    with pytest.raises(FFDError):
        tutte_map(V3, w.T, idx, pos)  # zero-length edge
    bad = pos.copy()
    bad[0, 0] = np.nan
    with pytest.raises(FFDError):
        tutte_map(w.V, w.T, idx, bad)
