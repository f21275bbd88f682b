"""Pins of the oracle's W-step under general linear constraints A W = c
(eq. solvinginw and the W-step text), against things other than its KKT
solve: the elimination of pinned rows (pins written as constraint rows), the
constrained minimiser of the W-step objective found over a null-space basis,
and the KKT conditions."""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
from paper_2107_05200_amd import meshgen as mg


def _state(r, seed=4):
    rng = np.random.default_rng(seed)
    d, m = r.d, r.m
    U = np.linalg.qr(rng.normal(size=(m, d, d)))[0]
    U = U * np.sign(np.linalg.det(U))[:, None, None]
    M = rng.normal(size=(m, d, d)) * 0.3
    P = np.eye(d) + 0.5 * (M + np.transpose(M, (0, 2, 1)))
    Lam = rng.normal(size=(m, d, d)) * 0.1
    return U, P, Lam


def _relational_rows(n, d, rng, k=3):
    """k random relations: a vertex at a fixed affine combination of two
    others, a difference of two vertices, the centroid of a few vertices."""
    rows, cs = [], []
    v = rng.choice(n, size=7 * k, replace=False)
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
        cs.append(rng.normal(size=d))
    return np.array(rows), np.array(cs)


def test_pins_written_as_constraint_rows():
    """Pins eliminated from L and the same pins as rows e_i^T W = p_i of a
    constraint system give the same W-step and the same iterations."""
    w = mg.height_field_uv(grid=10)
    a = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    A = np.zeros((len(w.pinned_idx), w.n))
    A[np.arange(len(w.pinned_idx)), w.pinned_idx] = 1.0
    b = O.OracleSolver(w.V, w.T, w.energy, w.rho, [], None, constraints=(A, w.pinned_pos))
    assert b.pins.size == 0 and not b.auto_pinned
    a.init(w.x0)
    b.init(w.x0)
    U, P, Lam = _state(a)
    assert np.max(np.abs(a.w_step(U, P, Lam) - b.w_step(U, P, Lam))) < 1e-12
    a.iterate(5)
    b.iterate(5)
    assert np.max(np.abs(a.x - b.x)) < 1e-11


def test_constrained_w_step_is_the_constrained_minimiser():
    """The W-step objective sum_i mu_i/2 |(G W)_i - (U_i P_i - Lam_i)|^2,
    minimised over W = W_p + N z with N a basis of the null space of the
    stacked pin and constraint rows (least squares, no KKT system)."""
    w = mg.height_field_uv(grid=9)
    rng = np.random.default_rng(2)
    A, c = _relational_rows(w.n, 2, rng, k=2)
    r = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, constraints=(A, c))
    r.init(w.x0)
    U, P, Lam = _state(r, seed=8)
    x = r.w_step(U, P, Lam)
    # all constraints on the full W: pins as rows, then A
    E = np.zeros((len(w.pinned_idx), w.n))
    E[np.arange(len(w.pinned_idx)), w.pinned_idx] = 1.0
    Cmat = np.vstack([E, A])
    crhs = np.vstack([w.pinned_pos, c])
    Wp = np.linalg.lstsq(Cmat, crhs, rcond=None)[0]
    N = sla.null_space(Cmat)
    G = r.G.toarray()
    target = (U @ P - Lam).reshape(r.m * 2, 2)
    sw = np.sqrt(np.repeat(r.mu, 2))[:, None]
    # minimise |sw * (G (Wp + N z) - target)|^2 column by column
    z = np.linalg.lstsq(sw * (G @ N), sw * (target - G @ Wp), rcond=None)[0]
    W = Wp + N @ z
    assert np.max(np.abs(W - x)) < 1e-9
    assert np.max(np.abs(A @ x - c)) < 1e-12


def test_kkt_conditions_in_3d_without_pins():
    """A tet cube held only by general constraints (no pin, so no vertex is
    fixed by the no-constraint rule): A W = c holds and the gradient of the
    W-step objective lies in the row space of A."""
    w = mg.twisted_cube(3)
    rng = np.random.default_rng(5)
    A, c = _relational_rows(w.n, 3, rng, k=3)
    r = O.OracleSolver(w.V, w.T, w.energy, w.rho, [], None, constraints=(A, c))
    assert r.pins.size == 0 and r.free.size == w.n
    r.init(w.x0)
    U, P, Lam = _state(r, seed=6)
    x = r.w_step(U, P, Lam)
    assert np.max(np.abs(A @ x - c)) < 1e-11
    rhs = np.asarray(r.G.T @ (r.mu[:, None, None] * (U @ P - Lam)).reshape(r.m * 3, 3))
    grad = r.L @ x - rhs
    y = np.linalg.lstsq(A.T, grad, rcond=None)[0]
    assert np.linalg.norm(A.T @ y - grad) < 1e-9 * np.linalg.norm(rhs)
    r.iterate(3)
    assert np.max(np.abs(A @ r.x - c)) < 1e-11


def test_satisfied_constraint_changes_nothing():
    """A constraint the unconstrained W-step already satisfies (written from
    that solution) leaves the W-step as it is."""
    w = mg.height_field_uv(grid=8)
    a = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    a.init(w.x0)
    U, P, Lam = _state(a, seed=3)
    x = a.w_step(U, P, Lam)
    A = np.zeros((1, w.n))
    A[0, [5, 17, 30]] = [0.5, 0.25, 0.25]
    b = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, constraints=(sp.csr_matrix(A), A @ x))
    b.init(w.x0)
    assert np.max(np.abs(b.w_step(U, P, Lam) - x)) < 1e-12
