"""Fill-reducing symmetric permutation for the oracle's W-step solve.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The W-step (eq. solvinginw) solves L_FF x = b.  Solving P L_FF P^T y = P b
and setting x = P^T y gives the same x for every permutation P, so a
permutation changes only the cost of the factorisation and the rounding, not
the result.  The oracle orders the free vertices by nested dissection
(George's method) with coordinate bisection: split a vertex set at the median
of its longest coordinate extent, take as separator the vertices of the lower
half that have a neighbour in the upper half (so the two halves are
disconnected once the separator is removed), number the two halves
recursively and the separator last.  SuperLU then factorises the permuted
matrix in that order (no column permutation of its own, no pivoting, which is
stable for the symmetric positive definite L_FF).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = ["nested_dissection", "SymmetricSolve"]


def nested_dissection(A, X, leaf: int = 64) -> np.ndarray:
    """Permutation p (new position -> old index) of the vertices of the
    symmetric sparse matrix A with coordinates X (n, k): halves first, then
    their separator, recursively down to sets of at most `leaf` vertices."""
    A = sp.csr_matrix(A)
    X = np.asarray(X, dtype=np.float64)
    n = A.shape[0]
    side = np.zeros(n, dtype=np.int8)
    order = []
    stack = [("split", np.arange(n))]
    while stack:
        what, idx = stack.pop()
        if what == "emit" or idx.size <= leaf:
            order.append(idx)
            continue
        c = X[idx, int(np.argmax(X[idx].max(axis=0) - X[idx].min(axis=0)))]
        lower = c < np.median(c)
        if not lower.any() or lower.all():
            order.append(idx)
            continue
        lo, hi = idx[lower], idx[~lower]
        side[hi] = 2
        side[lo] = 1
        rows = A[lo]
        owner = np.repeat(np.arange(lo.size), np.diff(rows.indptr))
        touches = np.zeros(lo.size, dtype=bool)
        touches[owner[side[rows.indices] == 2]] = True
        side[idx] = 0
        # processed last-in first-out: lower half, upper half, then the separator
        stack.append(("emit", lo[touches]))
        stack.append(("split", hi))
        stack.append(("split", lo[~touches]))
    p = np.concatenate(order) if order else np.zeros(0, dtype=np.int64)
    assert p.size == n and np.unique(p).size == n
    return p


class SymmetricSolve:
    """x = A^{-1} b for a symmetric positive definite sparse A, factorised once
    in the nested-dissection order of the coordinates X."""

    def __init__(self, A, X):
        A = sp.csc_matrix(A)
        self.p = nested_dissection(A, X)
        Ap = A[self.p][:, self.p].tocsc()
        self.lu = spla.splu(Ap, permc_spec="NATURAL", diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))

    def solve(self, b):
        b = np.asarray(b, dtype=np.float64)
        x = np.empty_like(b)
        x[self.p] = self.lu.solve(b[self.p])
        return x
