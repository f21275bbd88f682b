"""FP64 oracle of the Tutte initialiser.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Tutte's energy (supplement "Tutte's Energy"; Table 1, first row) of a map W of
a mesh with rest vertices V is the sum over the mesh edges (i, j), each edge
once, of |W_i - W_j|^2 / |V_i - V_j|.  It is quadratic in W, so with some
vertices held fixed its minimiser is the solution of one sparse linear system;
in 2D with the boundary on a convex curve that minimiser has no flipped
triangle (the cited theorem of Tutte), in 3D it may.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = ["mesh_edges", "tutte_energy", "tutte_laplacian", "tutte_map"]


def mesh_edges(T) -> np.ndarray:
    """The distinct edges (i < j) of the simplices of T: every pair of
    vertices of an element."""
    T = np.asarray(T, dtype=np.int64)
    nc = T.shape[1]
    pairs = [np.sort(T[:, [a, b]], axis=1) for a in range(nc) for b in range(a + 1, nc)]
    return np.unique(np.concatenate(pairs, axis=0), axis=0)


def tutte_energy(V, T, W) -> float:
    """Tutte's energy written out as the edge sum of its definition."""
    V = np.asarray(V, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    E = mesh_edges(T)
    total = 0.0
    for i, j in E:
        total += np.sum((W[i] - W[j]) ** 2) / np.linalg.norm(V[i] - V[j])
    return total


def tutte_laplacian(V, T) -> sp.csr_matrix:
    """The edge Laplacian K with Tutte's energy = trace(W^T K W): weight
    1 / |V_i - V_j| per edge, off-diagonal -weight, diagonal the row sums."""
    V = np.asarray(V, dtype=np.float64)
    E = mesh_edges(T)
    n = V.shape[0]
    wgt = 1.0 / np.linalg.norm(V[E[:, 0]] - V[E[:, 1]], axis=1)
    rows = np.concatenate([E[:, 0], E[:, 1], E[:, 0], E[:, 1]])
    cols = np.concatenate([E[:, 1], E[:, 0], E[:, 0], E[:, 1]])
    vals = np.concatenate([-wgt, -wgt, wgt, wgt])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def tutte_map(V, T, fixed_idx, fixed_pos) -> np.ndarray:
    """The minimiser of Tutte's energy over the free vertices with the vertices
    fixed_idx held at fixed_pos: K_FF W_F = -K_FC W_C (the gradient 2 K W
    vanishes on the free rows)."""
    V = np.asarray(V, dtype=np.float64)
    n = V.shape[0]
    fixed = np.asarray(fixed_idx, dtype=np.int64)
    pos = np.asarray(fixed_pos, dtype=np.float64).reshape(fixed.size, -1)
    free = np.setdiff1d(np.arange(n), fixed)
    K = tutte_laplacian(V, T)
    W = np.empty((n, pos.shape[1]))
    W[fixed] = pos
    rhs = -(K[free][:, fixed] @ pos)
    W[free] = spla.splu(K[free][:, free].tocsc()).solve(np.asarray(rhs))
    return W
