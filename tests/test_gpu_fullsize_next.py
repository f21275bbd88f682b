"""Full-size checks of rescaling, Tutte maps and general constraints on the
benchmark workload (twisted tet cube, 1,572,864 tets, float32 element
steps).  The oracle cannot run this size end to end: it checks one rescaling
event on sampled elements, the Tutte map through the residual of its edge
Laplacian, and the constrained W-step through its optimality condition on the
rows no constraint touches."""
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


def _host_state(s):
    import torch
    st = {k: v.cpu().numpy().astype(np.float64) for k, v in s.get_state().items()}
    torch.cuda.synchronize()
    return st


def test_fullsize_rescale_event_sampled(gpu_lib):
    """One rescaling event after iteration 4: on 4000 sampled elements the
    factor Lambda_before / Lambda_after is the oracle's rule applied to the
    device state (elements within 1e-3 of a decision boundary are left out),
    and the iterations after the host refactorisation stay finite."""
    from paper_2107_05200_amd.binding import Solver
    w = mg.twisted_cube(64)
    say(f"case: full-size rescaling event {w.name} m={w.m}")
    s = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32)
    s.init(w.x0).iterate(3)
    x3 = _host_state(s)["map"]
    s.iterate(1)
    st4 = _host_state(s)
    t0 = time.perf_counter()
    s.rescale(5.0)
    say(f"  event (device rule + host refactorisation) {time.perf_counter() - t0:.2f} s")
    lam_after = _host_state(s)["Lam"]
    rng = np.random.default_rng(11)
    sel = np.sort(rng.choice(w.m, size=4000, replace=False))
    T = w.T[sel]
    verts, Tl = np.unique(T, return_inverse=True)
    Tl = Tl.reshape(T.shape)
    B, wt = O.element_geometry(w.V[verts], Tl)
    G = O.gradient_operator(B, Tl, len(verts))
    J4 = O.jacobians(G, st4["map"][verts], 3)
    J3 = O.jacobians(G, x3[verts], 3)
    U, P = st4["U"][sel], st4["P"][sel]
    mu = w.rho * wt
    e_prim = np.sqrt(np.sum((J4 - U @ P) ** 2, axis=(1, 2)))
    e_dual = mu * np.sqrt(np.sum((J4 - J3) ** 2, axis=(1, 2)))
    p = np.linalg.eigvalsh(P)
    Bq = np.sqrt(5.0 * (1.0 + O.grad_norm_sq_of_spd_eigs(p, w.energy)))
    floor = 0.5 * O.mu_min(wt, O.lipschitz_f(Bq, 3, w.energy))
    new_mu, sfac = O.rescale_rule(mu, e_prim, e_dual, floor, 5.0)
    up = e_prim / np.maximum(5.0 * e_dual, 1e-300)
    down = e_dual / np.maximum(5.0 * e_prim, 1e-300)
    cand = np.where(e_prim > 5.0 * e_dual, mu * 2.5, np.where(e_dual > 5.0 * e_prim, mu / 2.5, mu))
    clear = (np.abs(up - 1) > 1e-3) & (np.abs(down - 1) > 1e-3) & (np.abs(cand / floor - 1) > 1e-3)
    lb, la = st4["Lam"][sel], lam_after[sel]
    big = np.linalg.norm(lb, axis=(1, 2)) > 1e-20
    use = clear & big
    ratio = np.linalg.norm(lb, axis=(1, 2))[use] / np.linalg.norm(la, axis=(1, 2))[use]
    err = np.max(np.abs(ratio / sfac[use] - 1))
    say(f"  {use.sum()} of {len(sel)} sampled elements compared; factors "
        f"{np.unique(np.round(sfac[use], 3))[:6]}...; worst rel err {err:.2e}")
    assert use.sum() > 3500
    assert err < 1e-5
    s.iterate(6, graph=True)
    h = s.history()
    assert np.all(np.isfinite(h[:, :3]))
    say(f"  six iterations after the event: e_prim {h[-1, 0]:.3e}, E_P {h[-1, 2]:.6g}")


def test_fullsize_tutte_volume(gpu_lib):
    """The cube's 24,578 boundary vertices on a twisted surface: the device
    map zeroes the oracle's edge-Laplacian residual on the interior rows."""
    import torch
    from paper_2107_05200_amd.binding import tutte_map
    V, T = mg.kuhn_cube(64)
    idx = mg.boundary_vertices(T)
    P = V[idx]
    a = np.deg2rad(45.0) * P[:, 2]
    x, y = P[:, 0] - 0.5, P[:, 1] - 0.5
    pos = np.stack([0.5 + np.cos(a) * x - np.sin(a) * y, 0.5 + np.sin(a) * x + np.cos(a) * y, P[:, 2]], axis=1)
    say(f"case: full-size Tutte volume map, {T.shape[0]} tets, {len(idx)} fixed vertices")
    t0 = time.perf_counter()
    Wd = tutte_map(V, T, idx, pos)
    torch.cuda.synchronize()
    say(f"  ffd_tutte_map {time.perf_counter() - t0:.2f} s")
    W = Wd.cpu().numpy()
    K = O.tutte.tutte_laplacian(V, T).tocsr()
    free = np.setdiff1d(np.arange(V.shape[0]), idx)
    res = np.linalg.norm(K[free] @ W) / np.linalg.norm(K[free][:, idx] @ pos)
    say(f"  relative residual {res:.2e}")
    assert res < 1e-10
    assert np.array_equal(W[idx], pos)


def test_fullsize_constrained_w_step(gpu_lib):
    """60 relational constraint rows on the cube: after 12 replayed
    iterations A W = c holds to 1e-9, and the W-step of the last iteration
    meets the KKT conditions: the gradient L W - G^T r (r from the previous
    state, recomputed in float64 from the float32 state, hence the 1e-5
    tolerance) vanishes on every free row no constraint touches and lies in
    the row space of A on the touched ones."""
    from paper_2107_05200_amd.binding import Solver
    w = mg.twisted_cube(64)
    rng = np.random.default_rng(60)
    v = rng.choice(np.setdiff1d(np.arange(w.n), w.pinned_idx), size=140, replace=False)
    A = np.zeros((60, w.n))
    c = np.zeros((60, 3))
    for i in range(20):
        A[3 * i, v[7 * i:7 * i + 3]] = [1.0, -0.5, -0.5]
        A[3 * i + 1, v[7 * i + 3:7 * i + 5]] = [1.0, -1.0]
        c[3 * i + 1] = w.V[v[7 * i + 3]] - w.V[v[7 * i + 4]]
        A[3 * i + 2, v[7 * i + 4:7 * i + 7]] = 1.0 / 3.0
        c[3 * i + 2] = w.V[v[7 * i + 4:7 * i + 7]].mean(axis=0) + 0.01
    say(f"case: full-size constrained W-step, {A.shape[0]} rows")
    s = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32, constraints=(A, c))
    s.init(w.x0).iterate(11, graph=True)
    prev = _host_state(s)
    s.iterate(1)
    cur = _host_state(s)
    x = cur["map"]
    viol = np.max(np.abs(A @ x - c))
    say(f"  |A W - c| = {viol:.2e}")
    assert viol < 1e-9
    B, wt = O.element_geometry(w.V, w.T)
    G = O.gradient_operator(B, w.T, w.n)
    mu = w.rho * wt
    L = O.global_matrix(G, mu, 3)
    r = mu[:, None, None] * (prev["U"] @ prev["P"] - prev["Lam"])
    f = np.asarray(G.T @ r.reshape(w.m * 3, 3))
    res = np.asarray(L @ x) - f
    touched = np.zeros(w.n, dtype=bool)
    touched[np.nonzero(A)[1]] = True
    touched[w.pinned_idx] = True
    rows = ~touched
    fn = np.linalg.norm(f[rows])
    rel_res = np.linalg.norm(res[rows]) / fn
    cols = np.unique(np.nonzero(A)[1])
    lam = np.linalg.lstsq(A[:, cols].T, res[cols], rcond=None)[0]
    span_res = np.linalg.norm(A[:, cols].T @ lam - res[cols]) / fn
    say(f"  gradient on {rows.sum()} untouched free rows {rel_res:.2e}; on the {cols.size} constrained "
        f"vertices {np.linalg.norm(res[cols]) / fn:.2e}, outside the row space of A {span_res:.2e}")
    assert rel_res < 1e-5
    assert span_res < 1e-5
    h = s.history()
    assert np.all(np.isfinite(h[:, :3]))
