"""Pins of the Tutte-initialiser oracle (supplement "Tutte's Energy"), each
against something other than the oracle's own assembly: the edge count of a
disk (Euler), the vanishing first variation of the edge-sum energy, a
general-purpose minimiser, the affine reproduction of centrally symmetric
stencils, and Tutte's theorem (no flipped triangle with a convex boundary)."""
import numpy as np
import pytest
import scipy.optimize as so

import oracle as O
from paper_2107_05200_amd import meshgen as mg

T_ = O.tutte


def _noisy_disk(R=4, seed=3):
    ring, tt, T = mg.hex_disk(R)
    phi = 2.0 * np.pi * tt / np.maximum(6 * ring, 1)
    rng = np.random.default_rng(seed)
    r = ring + np.where(ring < R, rng.uniform(-0.25, 0.25, ring.size), 0.0)
    V = np.stack([r * np.cos(phi), r * np.sin(phi), 0.2 * np.sin(r)], axis=1)
    return V, T


def _orient2(W, T):
    e1 = W[T[:, 1]] - W[T[:, 0]]
    e2 = W[T[:, 2]] - W[T[:, 0]]
    return e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]


def test_edges_of_a_disk_follow_euler():
    for R in (1, 3, 6):
        ring, tt, T = mg.hex_disk(R)
        n, f = ring.size, T.shape[0]
        assert T_.mesh_edges(T).shape[0] == n + f - 1  # V - E + F = 1
    k = 5
    assert T_.mesh_edges(mg.grid_triangles(k)).shape[0] == 3 * k * k + 2 * k


def test_first_variation_of_the_edge_sum_vanishes():
    """At the minimiser the edge-sum energy has no linear term along any
    free-vertex direction: E(W + t D) - E(W - t D) = 0 (to rounding), while
    the quadratic term is positive."""
    V, T = _noisy_disk()
    idx, pos = mg.circle_boundary(V, T)
    W = T_.tutte_map(V, T, idx, pos)
    free = np.setdiff1d(np.arange(V.shape[0]), idx)
    rng = np.random.default_rng(7)
    E0 = T_.tutte_energy(V, T, W)
    for _ in range(4):
        D = np.zeros_like(W)
        D[free] = rng.normal(size=(free.size, 2))
        t = 1e-3
        ep, em = T_.tutte_energy(V, T, W + t * D), T_.tutte_energy(V, T, W - t * D)
        lin = (ep - em) / (2 * t)
        quad = (ep + em - 2 * E0) / (t * t)
        assert abs(lin) < 1e-9 * quad
        assert quad > 0


def test_matches_a_general_minimiser():
    V, T = _noisy_disk(R=3, seed=5)
    idx, pos = mg.circle_boundary(V, T)
    W = T_.tutte_map(V, T, idx, pos)
    free = np.setdiff1d(np.arange(V.shape[0]), idx)

    def f(z):
        X = np.empty((V.shape[0], 2))
        X[idx] = pos
        X[free] = z.reshape(-1, 2)
        return T_.tutte_energy(V, T, X)

    res = so.minimize(f, np.zeros(2 * free.size), method="BFGS", options={"gtol": 1e-11, "maxiter": 5000})
    assert np.max(np.abs(res.x.reshape(-1, 2) - W[free])) < 1e-5
    assert T_.tutte_energy(V, T, W) <= res.fun + 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_symmetric_stencils_reproduce_affine_boundaries(dim):
    """On a regular grid (2D) and a Kuhn cube (3D) every interior vertex's
    edges come in opposite pairs of equal length, so an affine image of the
    boundary extends affinely."""
    rng = np.random.default_rng(11 + dim)
    if dim == 2:
        k = 7
        T = mg.grid_triangles(k)
        i, j = np.meshgrid(np.arange(k + 1), np.arange(k + 1), indexing="xy")
        V = np.stack([i.ravel() / k, j.ravel() / k], axis=1).astype(np.float64)
    else:
        V, T = mg.kuhn_cube(4)
    A = rng.normal(size=(dim, dim))
    c = rng.normal(size=dim)
    idx = mg.boundary_vertices(T)
    W = T_.tutte_map(V, T, idx, V[idx] @ A.T + c)
    assert np.max(np.abs(W - (V @ A.T + c))) < 1e-12


def test_convex_boundary_gives_no_flip():
    """Tutte's theorem on a noisy, curved disk: all triangles keep their
    orientation and the interior stays inside the circle."""
    V, T = _noisy_disk(R=8, seed=9)
    idx, pos = mg.circle_boundary(V, T)
    W = T_.tutte_map(V, T, idx, pos)
    assert _orient2(W, T).min() > 0
    free = np.setdiff1d(np.arange(V.shape[0]), idx)
    assert np.linalg.norm(W[free], axis=1).max() < 1.0


def test_boundary_helpers():
    ring, tt, T = mg.hex_disk(4)
    loop = mg.boundary_loop(T)
    assert sorted(loop.tolist()) == sorted(np.nonzero(ring == 4)[0].tolist())
    assert np.array_equal(np.sort(loop), mg.boundary_vertices(T))
    V, T3 = mg.kuhn_cube(3)
    b = mg.boundary_vertices(T3)
    on = np.any((V == 0.0) | (V == 1.0), axis=1)
    assert np.array_equal(b, np.nonzero(on)[0])
