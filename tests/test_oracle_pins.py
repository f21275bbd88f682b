"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics,
independent of the oracle's own code paths (brute-force searches, independent
textbook routines, closed forms, invariants).  CPU only."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from paper_2107_05200_amd import meshgen as mg


def rng(seed=0):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------------------
# scalar roots
# ----------------------------------------------------------------------------

def _fs(p, energy):
    # per-eigenvalue defining function on S+: SD 1/2(p^2 + p^-2), SG 1/2 p^2 - log p
    return 0.5 * (p * p + 1.0 / (p * p)) if energy == O.SD else 0.5 * p * p - np.log(p)


def _brute_min(q, w, mu, energy):
    """Minimise phi(p) = w f(p) + mu/2 (p - q)^2 over p > 0 by a log grid and a
    golden-section refinement in log p (no use of the stationarity equation)."""
    # mu/2 (p-q)^2 without its constant mu q^2/2, so that large |q| does not
    # swamp the resolution of the search
    phi = lambda p: w * _fs(p, energy) + 0.5 * mu * p * p - mu * q * p
    grid = np.exp(np.linspace(math.log(1e-6), math.log(1e4), 200001))
    k = int(np.argmin(phi(grid)))
    a = math.log(grid[max(k - 2, 0)])
    b = math.log(grid[min(k + 2, grid.size - 1)])
    g = (math.sqrt(5) - 1) / 2
    c, d = b - g * (b - a), a + g * (b - a)
    for _ in range(200):
        if phi(math.exp(c)) < phi(math.exp(d)):
            b = d
        else:
            a = c
        c, d = b - g * (b - a), a + g * (b - a)
    return math.exp(0.5 * (a + b))


@pytest.mark.parametrize("energy", [O.SD, O.SG])
def test_pin1_root_matches_brute_force_minimisation(energy):
    r = rng(1)
    qs = np.concatenate([r.uniform(-30, 30, 20), [-1e3, -5.0, -1e-3, 0.0, 1e-3, 1.0, 3.0, 1e3]])
    for q in qs:
        ratio = 10 ** r.uniform(-3, 3)  # w / mu in [1e-3, 1e3]
        w, mu = ratio, 1.0
        p_ref = _brute_min(q, w, mu, energy)
        p = (O.root_sd if energy == O.SD else O.root_sg)(np.array([q]), w, mu)[0]
        # the objective is flat at its minimum: a direct search resolves p to ~sqrt(eps)
        assert abs(p - p_ref) <= 2e-7 * p_ref, (q, w, mu, p, p_ref)


@pytest.mark.parametrize("energy", [O.SD, O.SG])
def test_pin2_root_polynomial_residual(energy):
    r = rng(2)
    q = np.concatenate([r.uniform(-1e3, 1e3, 500), r.uniform(-2, 2, 500)])
    w = 10 ** r.uniform(-3, 3, q.size)
    mu = np.ones_like(q)
    if energy == O.SG:
        p = O.root_sg(q, w, mu)
        terms = np.abs((w + mu) * p * p) + np.abs(mu * q * p) + w
        res = (w + mu) * p * p - mu * q * p - w          # supplement eq. peqfsgpluggedin
        assert np.all(np.abs(res) <= 4e-15 * terms)
    else:
        p = O.root_sd(q, w, mu)
        terms = np.abs((w + mu) * p ** 4) + np.abs(mu * q * p ** 3) + w
        res = (w + mu) * p ** 4 - mu * q * p ** 3 - w    # supplement eq. peqfsdpluggedin
        assert np.all(np.abs(res) <= 1e-14 * terms)
    assert np.all(p > 0)


@pytest.mark.parametrize("energy", [O.SD, O.SG])
def test_root_special_values(energy):
    # q = 1 (the identity) is the root for every w, mu; the SG quadratic formula
    # written out independently for a few values
    w = np.array([1e-3, 0.1, 1.0, 7.0, 1e3])
    f = O.root_sd if energy == O.SD else O.root_sg
    assert np.allclose(f(np.ones(5), w, 1.0), 1.0, rtol=1e-15, atol=0)
    if energy == O.SG:
        from decimal import Decimal, getcontext
        getcontext().prec = 50
        for q in [-3.0, 0.5, 4.0]:
            for ww in w:
                Q, W = Decimal(q), Decimal(float(ww))
                exact = float((Q + (Q * Q + 4 * W * (W + 1)).sqrt()) / (2 * (W + 1)))
                assert abs(f(np.array([q]), ww, 1.0)[0] - exact) <= 1e-14 * exact


# ----------------------------------------------------------------------------
# matrix P-step and U-step
# ----------------------------------------------------------------------------

def _direct_pstep(S, w, mu, energy):
    """Minimise w f(P) + mu/2 |P - S|^2 over P = L L^T with a general optimizer."""
    d = S.shape[0]
    il = np.tril_indices(d)

    def obj(v):
        Lm = np.zeros((d, d))
        Lm[il] = v
        P = Lm @ Lm.T
        det = np.linalg.det(P)
        if det <= 0:
            return 1e30
        if energy == O.SD:
            f = 0.5 * (np.sum(P * P) + np.sum(np.linalg.inv(P) ** 2))
        else:
            f = 0.5 * np.sum(P * P) - math.log(det)
        return w * f + 0.5 * mu * np.sum((P - S) ** 2)

    v0 = np.eye(d)[il]
    res = minimize(obj, v0, method="BFGS", options={"gtol": 1e-12, "maxiter": 10000})
    res = minimize(obj, res.x, method="Nelder-Mead",
                   options={"xatol": 1e-12, "fatol": 1e-16, "maxiter": 40000})
    Lm = np.zeros((d, d))
    Lm[il] = res.x
    return Lm @ Lm.T


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("energy", [O.SD, O.SG])
def test_pin3_matrix_pstep(d, energy):
    r = rng(3 + d)
    for trial in range(4):
        A = r.normal(size=(d, d))
        S = 0.5 * (A + A.T) + (1.5 if trial % 2 == 0 else 0.0) * np.eye(d)
        w, mu = 1.0, 10 ** r.uniform(-1, 1)
        P, p = O.p_step(S[None], np.array([w]), np.array([mu]), energy)
        P = P[0]
        P_ref = _direct_pstep(S, w, mu, energy)
        assert np.allclose(P, P.T, atol=1e-14)
        assert np.all(np.linalg.eigvalsh(P) > 0)
        assert np.linalg.norm(P - P_ref) <= 1e-5 * max(1.0, np.linalg.norm(P_ref))
        # stationarity w grad f(P) + mu P = mu S  (eq. rootfindinginp)
        Pi = np.linalg.inv(P)
        grad = P - Pi @ Pi @ Pi if energy == O.SD else P - Pi
        assert np.linalg.norm(w * grad + mu * P - mu * S) <= 1e-12 * max(1.0, mu * np.linalg.norm(S))


def test_pin4_rot2_brute_force_angle():
    r = rng(4)
    Q = r.normal(size=(50, 2, 2))
    U = O.rot2(Q, np.tile(np.eye(2), (50, 1, 1)))
    phis = np.linspace(0, 2 * np.pi, 720001)
    for i in range(50):
        val = np.cos(phis) * (Q[i, 0, 0] + Q[i, 1, 1]) + np.sin(phis) * (Q[i, 1, 0] - Q[i, 0, 1])
        k = int(np.argmax(val))
        a, b = phis[k] - 1e-5, phis[k] + 1e-5
        f = lambda t: -(np.cos(t) * (Q[i, 0, 0] + Q[i, 1, 1]) + np.sin(t) * (Q[i, 1, 0] - Q[i, 0, 1]))
        g = (math.sqrt(5) - 1) / 2
        for _ in range(100):
            c, d = b - g * (b - a), a + g * (b - a)
            if f(c) < f(d):
                b = d
            else:
                a = c
        phi = 0.5 * (a + b)
        phi_or = math.atan2(U[i, 1, 0], U[i, 0, 0])
        dphi = (phi_or - phi + np.pi) % (2 * np.pi) - np.pi
        assert abs(dphi) < 1e-7
        assert abs(np.linalg.det(U[i]) - 1) < 1e-14


def _quat_rot(qv):
    w, x, y, z = qv
    return np.array([
        [w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z]])


def _horn(Q):
    """Rotation maximising tr(R^T Q) as the top eigenvector of the symmetric 4x4
    matrix of the quadratic form q -> tr(R(q)^T Q) (Horn / Davenport); built by
    polarisation, no SVD."""
    f = lambda qv: np.sum(_quat_rot(qv) * Q)
    E = np.eye(4)
    N = np.empty((4, 4))
    for a in range(4):
        for b in range(4):
            N[a, b] = 0.25 * (f(E[a] + E[b]) - f(E[a] - E[b]))
    ev, V = np.linalg.eigh(N)
    return _quat_rot(V[:, -1]), ev


def test_pin5_rot3_against_quaternion_method():
    r = rng(5)
    Q = r.normal(size=(200, 3, 3))
    # orthogonal inputs of both signs of det: det = -1 gives a tie (a circle of optima)
    Q[:50] = np.linalg.qr(r.normal(size=(50, 3, 3)))[0]
    Q[:25, :, 2] *= -1.0
    U = O.rot3(Q)
    checked = 0
    for i in range(Q.shape[0]):
        R, ev = _horn(Q[i])
        assert abs(np.linalg.det(U[i]) - 1) < 1e-12
        # the optimal value is the top eigenvalue of the quaternion form, ties or not
        assert abs(np.sum(U[i] * Q[i]) - ev[-1]) < 1e-10 * max(1.0, abs(ev[-1]))
        H = U[i].T @ Q[i]
        assert np.allclose(H, H.T, atol=1e-10)  # U^T Q symmetric at the optimum
        if ev[-1] - ev[-2] > 1e-6 * max(1.0, abs(ev[-1])):  # unique optimum
            assert np.abs(U[i] - R).max() < 1e-9
            checked += 1
    assert checked > 160


# ----------------------------------------------------------------------------
# discretisation
# ----------------------------------------------------------------------------

def test_pin7_D_exactness_and_weights():
    r = rng(7)
    # planar triangles (d_in = d = 2) and tets: affine maps reproduced exactly
    w2 = mg.hex_disk(6)
    ring, tt, T = w2
    phi = 2 * np.pi * tt / np.maximum(6 * ring, 1)
    V = np.stack([ring * np.cos(phi), ring * np.sin(phi)], 1) / 6.0
    V = V + r.normal(scale=0.01, size=V.shape)
    for (VV, TT) in [(V, T), mg.kuhn_cube(3)]:
        d = TT.shape[1] - 1
        B, w = O.element_geometry(VV, TT)
        G = O.gradient_operator(B, TT, VV.shape[0])
        A = r.normal(size=(d, d))
        t = r.normal(size=d)
        J = O.jacobians(G, VV @ A + t, d)
        assert np.abs(J - A).max() < 1e-11
        assert np.abs(G @ np.ones(VV.shape[0])).max() < 1e-11
        e = VV[TT[:, 1:]] - VV[TT[:, [0]]]
        if d == 2:
            area = 0.5 * np.abs(e[:, 0, 0] * e[:, 1, 1] - e[:, 0, 1] * e[:, 1, 0])
        else:
            area = np.abs(np.einsum("mi,mi->m", e[:, 0], np.cross(e[:, 1], e[:, 2]))) / 6.0
        assert np.allclose(w, area, rtol=1e-13)
    # intrinsic gradient on a surface: a flat mesh tilted in 3D, mapped to its
    # own in-plane coordinates, has rotation Jacobians; areas are 1/2|e1 x e2|
    wk = mg.height_field_uv(grid=6)
    R3 = np.linalg.qr(r.normal(size=(3, 3)))[0]
    flat = np.concatenate([wk.V[:, :2], np.zeros((wk.n, 1))], 1)
    B, w = O.element_geometry(flat @ R3.T, wk.T)
    G = O.gradient_operator(B, wk.T, wk.n)
    J = O.jacobians(G, wk.V[:, :2], 2)
    assert np.abs(np.einsum("mji,mjk->mik", J, J) - np.eye(2)).max() < 1e-12
    assert np.abs(np.linalg.det(J) - 1).max() < 1e-12
    e = wk.V[wk.T[:, 1:]] - wk.V[wk.T[:, [0]]]
    _, w3 = O.element_geometry(wk.V, wk.T)
    assert np.allclose(w3, 0.5 * np.linalg.norm(np.cross(e[:, 0], e[:, 1]), axis=1), rtol=1e-13)


def _cot(a, b, c):
    u, v = b - a, c - a
    return np.dot(u, v) / abs(u[0] * v[1] - u[1] * v[0])


def test_pin8_global_matrix_is_scaled_cotangent_laplacian():
    r = rng(8)
    ring, tt, T = mg.hex_disk(4)
    phi = 2 * np.pi * tt / np.maximum(6 * ring, 1)
    V = np.stack([ring * np.cos(phi), ring * np.sin(phi)], 1) / 4.0 + r.normal(scale=0.02, size=(ring.size, 2))
    rho = 10.0
    B, w = O.element_geometry(V, T)
    L = O.global_matrix(O.gradient_operator(B, T, V.shape[0]), rho * w, 2).toarray()
    assert np.abs(L - L.T).max() < 1e-12
    assert np.abs(L.sum(1)).max() < 1e-11
    C = np.zeros_like(L)
    for t in T:
        for k in range(3):
            i, j, o = t[k], t[(k + 1) % 3], t[(k + 2) % 3]
            c = _cot(V[o], V[i], V[j])  # angle opposite edge (i, j)
            C[i, j] += -0.5 * rho * c
            C[j, i] += -0.5 * rho * c
    off = ~np.eye(L.shape[0], dtype=bool)
    assert np.abs(L[off] - C[off]).max() < 1e-11
    # 3D: the stiffness matrix annihilates affine functions at interior vertices
    V3, T3 = mg.kuhn_cube(4)
    V3 = V3 + r.normal(scale=0.01, size=V3.shape)
    B3, w3 = O.element_geometry(V3, T3)
    L3 = O.global_matrix(O.gradient_operator(B3, T3, V3.shape[0]), rho * w3, 3)
    interior = np.all((mg.kuhn_cube(4)[0] > 0) & (mg.kuhn_cube(4)[0] < 1), axis=1)
    aff = V3 @ r.normal(size=(3, 3)) + 1.0
    assert np.abs((L3 @ aff)[interior]).max() < 1e-10


# ----------------------------------------------------------------------------
# W-step, init and the iteration
# ----------------------------------------------------------------------------

def _random_state(s, r, scale=0.3):
    d = s.d
    U = O.rotation_step(np.eye(d) + scale * r.normal(size=(s.m, d, d)), np.tile(np.eye(d), (s.m, 1, 1)))
    A = r.normal(size=(s.m, d, d)) * scale
    P = np.eye(d) + 0.5 * (A + np.transpose(A, (0, 2, 1)))
    P = np.einsum("mij,mkj->mik", P, P)  # SPD
    Lam = scale * r.normal(size=(s.m, d, d))
    return U, P, Lam


def test_pin9_wstep_is_weighted_least_squares():
    r = rng(9)
    wk = mg.height_field_uv(grid=7)
    s = O.OracleSolver(wk.V, wk.T, wk.energy, wk.rho, wk.pinned_idx, wk.pinned_pos)
    s.init(wk.x0)
    U, P, Lam = _random_state(s, r)
    x = s.w_step(U, P, Lam)
    # independent: dense weighted least squares over the free vertices
    Y = U @ P - Lam
    G = s.G.toarray()
    sw = np.sqrt(np.repeat(s.mu, s.d))
    free = s.free
    Gf, Gc = G[:, free], G[:, s.pins]
    rhs = (Y.reshape(-1, s.d) - Gc @ s.pin_pos) * sw[:, None]
    xf = np.linalg.lstsq(Gf * sw[:, None], rhs, rcond=None)[0]
    assert np.abs(x[free] - xf).max() < 1e-10
    assert np.allclose(x[s.pins], s.pin_pos)
    # normal equations residual
    b = (s.G.T @ (s.mu[:, None, None] * Y).reshape(-1, s.d))[free] - s.L_FC @ s.pin_pos
    res = s.L_FF @ x[free] - b
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("energy", [O.SD, O.SG])
def test_polar_init_rules(energy):
    r = rng(10)
    for d in (2, 3):
        J = r.normal(size=(300, d, d))
        U, P, flipped = O.polar_init(J, energy)
        eps = O.init_epsilon(energy)
        assert np.allclose(np.linalg.det(U), 1.0, atol=1e-12)
        assert np.array_equal(flipped, np.linalg.det(J) <= 0)
        ev = np.linalg.eigvalsh(P)
        assert np.all(ev >= eps * (1 - 1e-12))
        ok = ~flipped & (np.linalg.svd(J, compute_uv=False).min(axis=1) > eps)
        assert np.abs(U[ok] @ P[ok] - J[ok]).max() < 1e-12
        assert np.allclose(P[flipped], eps * np.eye(d), atol=1e-15)
    assert math.isclose(O.init_epsilon(O.SG), 2.0 ** -13)
    assert math.isclose(O.init_epsilon(O.SD), 2.0 ** -6.5)


@pytest.mark.parametrize("energy", [O.SD, O.SG])
def test_pin6_identity_fixed_point(energy):
    for wk in (mg.flat_grid(6, energy=energy), mg.twisted_cube(3, twist_deg=0.0, lift=0.0, energy=energy)):
        s = O.OracleSolver(wk.V, wk.T, energy, wk.rho, wk.pinned_idx, wk.pinned_pos)
        s.init(wk.x0)
        s.iterate(3)
        d = s.d
        assert np.abs(s.x - wk.V).max() < 1e-13
        assert np.abs(s.U - np.eye(d)).max() < 1e-13
        assert np.abs(s.P - np.eye(d)).max() < 1e-13
        assert np.abs(s.Lam).max() < 1e-13
        E = s.history.col("E_P")[-1] / s.w.sum()
        # f_SD(I) = d (with the paper's 1/2), i.e. 4 per triangle and 6 per tet
        # without it; f_SG(I) = d/2
        if energy == O.SD:
            assert abs(2 * E - 2 * d) < 1e-12 and abs(E - d) < 1e-12
        else:
            assert abs(E - d / 2) < 1e-12


def _phi(s, x, U, P, Lam):
    J = O.jacobians(s.G, x, s.d)
    p = np.linalg.eigvalsh(P)
    R = J - U @ P + Lam
    return np.sum(s.w * O.energy_of_spd_eigs(p, s.energy)
                  + 0.5 * s.mu * (np.sum(R * R, axis=(1, 2)) - np.sum(Lam * Lam, axis=(1, 2))))


@pytest.mark.parametrize("energy", [O.SD, O.SG])
@pytest.mark.parametrize("dims", [2, 3])
def test_algorithm1_substeps_by_brute_force(energy, dims):
    """One oracle iteration from a random state on a tiny mesh; each sub-step is
    checked as the argmin Algorithm 1 says it is, by independent searches."""
    r = rng(11)
    wk = mg.height_field_uv(grid=3, energy=energy) if dims == 2 else \
        mg.twisted_cube(1, energy=energy)
    s = O.OracleSolver(wk.V, wk.T, energy, wk.rho, wk.pinned_idx, wk.pinned_pos)
    s.init(wk.x0)
    U0, P0, L0 = _random_state(s, r)
    s.set_state(wk.x0, U0, P0, L0)
    s.iterate(1)
    x1, U1, P1, L1 = s.x, s.U, s.P, s.Lam
    # W: minimiser of Phi(., U0, P0, L0) -- gradient wrt free coordinates vanishes
    h = 1e-6
    for v in s.free[:4]:
        for k in range(s.d):
            xp, xm = x1.copy(), x1.copy()
            xp[v, k] += h
            xm[v, k] -= h
            g = (_phi(s, xp, U0, P0, L0) - _phi(s, xm, U0, P0, L0)) / (2 * h)
            assert abs(g) < 1e-6 * max(1.0, s.mu.max())
    J1 = O.jacobians(s.G, x1, s.d)
    # U: minimiser of the per-element term over rotations (with P0, L0, h = 0)
    for i in range(s.m):
        target = J1[i] + L0[i]
        f = lambda Rm: np.sum((target - Rm @ P0[i]) ** 2)
        if s.d == 2:
            best = min(f(np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]]))
                       for t in np.linspace(0, 2 * np.pi, 20001))
        else:
            qs = r.normal(size=(20000, 4))
            qs /= np.linalg.norm(qs, axis=1)[:, None]
            best = min(f(_quat_rot(q)) for q in qs)
        assert f(U1[i]) <= best + 1e-9
    # P: minimiser of w f(P) + mu/2 |J1 - U1 P + L0|^2 (eq. optimizinginp)
    for i in range(min(s.m, 3)):
        S = 0.5 * (U1[i].T @ (J1[i] + L0[i]) + (J1[i] + L0[i]).T @ U1[i])
        Pr = _direct_pstep(S, s.w[i], s.mu[i], energy)
        assert np.linalg.norm(P1[i] - Pr) <= 1e-5 * np.linalg.norm(Pr)
    # Lambda: eq. lambdaupdate
    assert np.abs(L1 - (L0 + J1 - U1 @ P1)).max() < 1e-13


def test_pin10_step_identities_and_flip_free_UP():
    wk = mg.height_field_uv(grid=12)
    s = O.OracleSolver(wk.V, wk.T, wk.energy, wk.rho, wk.pinned_idx, wk.pinned_pos)
    s.init(wk.x0)
    for _ in range(15):
        L_old = s.Lam.copy()
        x_old = s.x.copy()
        s.iterate(1)
        e_prim = s.history.col("e_prim")[-1]
        assert abs(np.linalg.norm(s.Lam - L_old) - e_prim) <= 1e-12 * max(1.0, e_prim)
        assert np.all(np.linalg.det(s.U @ s.P) > 0)
        # e_dual of eq. primaldualerror and E_P = sum w f(P) from their definitions
        dJ = O.jacobians(s.G, s.x - x_old, s.d)
        e_dual = math.sqrt(np.sum(s.mu[:, None, None] ** 2 * dJ ** 2))
        assert abs(s.history.col("e_dual")[-1] - e_dual) <= 1e-12 * e_dual
        E_P = np.sum(s.w * O.energy_density(s.P, s.energy))
        assert abs(s.history.col("E_P")[-1] - E_P) <= 1e-12 * E_P


@pytest.mark.parametrize("energy", [O.SD, O.SG])
def test_pin11_kkt(energy):
    wk = mg.height_field_uv(grid=5, sigma=0.01, energy=energy)
    s = O.OracleSolver(wk.V, wk.T, energy, wk.rho, wk.pinned_idx, wk.pinned_pos)
    s.init(wk.x0)
    for it in range(3000):
        s.iterate(1)
        if it < 5 or it % 500 == 0:
            # first KKT line, symmetric part: exact after every P-step
            p, Qs = np.linalg.eigh(s.P)
            g = p - p ** -3 if energy == O.SD else p - 1 / p
            gradf = np.einsum("mij,mj,mkj->mik", Qs, g, Qs)
            UL = np.transpose(s.U, (0, 2, 1)) @ s.Lam
            symUL = 0.5 * (UL + np.transpose(UL, (0, 2, 1)))
            assert np.abs(s.w[:, None, None] * gradf - s.mu[:, None, None] * symUL).max() < 1e-12
    UL = np.transpose(s.U, (0, 2, 1)) @ s.Lam
    skew = 0.5 * (UL - np.transpose(UL, (0, 2, 1)))
    assert np.abs(skew).max() < 1e-6
    assert s.history.col("e_prim")[-1] < 1e-6
    # second KKT line (eq. kkt): mu Lam P^T lies in the normal cone of SO(d) at U,
    # i.e. U^T Lam P^T is symmetric.  Reading: the "argmin" restatement of that
    # line is a stationarity condition; at many elements U is its maximiser.
    ULP = np.transpose(s.U, (0, 2, 1)) @ s.Lam @ np.transpose(s.P, (0, 2, 1))
    assert np.abs(ULP - np.transpose(ULP, (0, 2, 1))).max() < 1e-6
    # third line: J = U P
    J = O.jacobians(s.G, s.x, s.d)
    assert np.abs(J - s.U @ s.P).max() < 1e-6


def test_pin12_rotation_equivariance():
    r = rng(12)
    wk = mg.height_field_uv(grid=10)
    a = 0.7
    R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
    s1 = O.OracleSolver(wk.V, wk.T, wk.energy, wk.rho, wk.pinned_idx, wk.pinned_pos)
    s2 = O.OracleSolver(wk.V, wk.T, wk.energy, wk.rho, wk.pinned_idx, wk.pinned_pos @ R.T)
    s1.init(wk.x0)
    s2.init(wk.x0 @ R.T)
    s1.iterate(20)
    s2.iterate(20)
    assert np.abs(s2.x - s1.x @ R.T).max() < 1e-10
    assert np.abs(np.linalg.eigvalsh(s2.P) - np.linalg.eigvalsh(s1.P)).max() < 1e-10
    h1, h2 = s1.history.array(), s2.history.array()
    assert np.allclose(h1[:, :5], h2[:, :5], rtol=1e-9, atol=1e-12)
    # moving the source rigidly leaves the map unchanged
    R3 = np.linalg.qr(r.normal(size=(3, 3)))[0]
    s3 = O.OracleSolver(wk.V @ R3.T + 0.3, wk.T, wk.energy, wk.rho, wk.pinned_idx, wk.pinned_pos)
    s3.init(wk.x0)
    s3.iterate(20)
    assert np.abs(s3.x - s1.x).max() < 1e-10


def test_pin13_residual_decrease_on_height_field():
    wk = mg.height_field_uv()  # 32 x 32 grid, sigma 0.02, SD, rho 10
    s = O.OracleSolver(wk.V, wk.T, wk.energy, wk.rho, wk.pinned_idx, wk.pinned_pos)
    s.init(wk.x0)
    s.iterate(200)
    ep, ed = s.history.col("e_prim"), s.history.col("e_dual")
    assert ep[-1] <= 0.1 * ep[0] and ed[-1] <= 0.1 * ed[0]
    win_p = [ep[i:i + 10].min() for i in range(0, 200, 10)]
    win_d = [ed[i:i + 10].min() for i in range(0, 200, 10)]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(win_p, win_p[1:]))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(win_d, win_d[1:]))
    assert s.history.col("flips")[-1] == 0
    assert math.isfinite(s.history.col("E_map")[-1])


# ---------------------------------------------------------------------------
# penalty rescaling (Section "Implementation", "Rescaling mu_i and Lambda")
# ---------------------------------------------------------------------------

def test_lipschitz_constants_of_the_lemma():
    """C^L and C^LG solve their polynomials, equal 1 at B = 0, behave like 1/B
    and B^(-1/3) for large B, and satisfy the lemma's C^L <= C^LG <= 1."""
    B = np.concatenate([[0.0], np.logspace(-3, 3, 400)])
    cl, clg = O.c_l(B), O.c_lg(B)
    assert np.all(cl > 0) and np.all(clg > 0)
    assert np.max(np.abs(cl * cl + B * cl - 1.0)) < 1e-13
    assert np.max(np.abs(clg ** 4 + B * clg ** 3 - 1.0)) < 1e-13
    assert cl[0] == 1.0 and abs(clg[0] - 1.0) < 1e-15
    assert np.all(cl <= clg + 1e-15) and np.all(clg <= 1.0)
    big = B > 500
    assert np.allclose(cl[big] * B[big], 1.0, rtol=1e-4)
    assert np.allclose(clg[big] * B[big] ** (1 / 3), 1.0, rtol=1e-2)


def test_mu_min_is_the_boundary_of_the_proposition():
    """mu_min(w, F) is the positive root of mu^2 + w mu - 4 w^2 F^2 = 0 (the
    proposition's inequality with gamma = 1, epsilon = 0, solved for mu), and
    F^2 is capped at eps_m^(-1/4)."""
    rng = np.random.default_rng(4)
    w = 10 ** rng.uniform(-6, 0, 300)
    F = 10 ** rng.uniform(0, 1.9, 300)
    mu = O.mu_min(w, F)
    assert np.all(mu > 0)
    assert np.max(np.abs(mu * mu + w * mu - 4 * w * w * F * F) / (4 * w * w * F * F)) < 1e-12
    Fsd = O.lipschitz_f(np.array([1e6]), 3, O.SD)
    assert abs(Fsd[0] ** 2 - O.EPS_M ** -0.25) <= 1e-9 * O.EPS_M ** -0.25
    assert abs(O.lipschitz_f(np.array([0.0]), 2, O.SG)[0] - (1 + math.sqrt(2))) < 1e-15


def test_rescale_rule_cases():
    mu = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 0.3])
    ep = np.array([6.0, 1.0, 5.0, 1.0, 1.0, 1.0])
    ed = np.array([1.0, 6.0, 1.0, 5.0, 1.0, 6.0])
    floor = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.2])
    new, s = O.rescale_rule(mu, ep, ed, floor, 5.0)
    assert np.allclose(new, [2.5, 0.4, 1.0, 1.0, 1.0, 0.2])
    assert np.allclose(s, new / mu)


def test_rescale_schedule_reading():
    ks = O.rescale_schedule(400)
    assert ks[:5] == [1, 2, 3, 4, 5]
    assert np.diff(ks[4:]).tolist() == [38, 57, 85, 128]


def test_rescale_keeps_the_unscaled_dual_and_refactors():
    """A rescaling event changes mu_i by 5/2 or 2/5 (or not, or up to the
    floor) and the scaled dual Lambda_i in the opposite direction, so the
    unscaled dual mu_i Lambda_i is unchanged; the new L_FF factor solves the
    new W-step exactly."""
    w = mg.height_field_uv()
    r = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    r.init(w.x0)
    r.iterate(3)
    Y0 = r.mu[:, None, None] * r.Lam
    mu0 = r.mu.copy()
    r.rescale(5.0)
    ratio = r.mu / mu0
    assert np.all(np.isclose(ratio, 2.5) | np.isclose(ratio, 0.4) | np.isclose(ratio, 1.0) | (ratio > 0.4))
    assert np.any(ratio != 1.0)
    assert np.allclose(r.mu[:, None, None] * r.Lam, Y0, rtol=1e-14, atol=1e-300)
    x = r.w_step(r.U, r.P, r.Lam)
    rr = r.mu[:, None, None] * (r.U @ r.P - r.Lam)
    rhs = np.asarray(r.G.T @ rr.reshape(r.m * r.d, r.d))[r.free] - r.L_FC @ r.pin_pos
    res = np.linalg.norm(r.L_FF @ x[r.free] - rhs) / np.linalg.norm(rhs)
    assert res < 1e-12


def test_constants_the_paper_prints():
    """tests/golden/paper_constants.txt transcribes the method's constants as
    the paper prints them (each with its passage); the oracle uses exactly
    these: machine epsilon of float64, the termination pair, the rescaling
    factor and F^2 cap, the initialisation epsilons and the eigenvalue floor."""
    import inspect
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")
    vals = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            name, expr, _ = [f.strip() for f in line.split("|")]
            vals[name] = float(eval(expr, {"__builtins__": {}}, {"eps_m": np.finfo(np.float64).eps}))
    assert O.EPS_M == np.finfo(np.float64).eps
    run = inspect.signature(O.OracleSolver.run).parameters
    assert run["eps_abs"].default == vals["eps_abs"] and run["eps_rel"].default == vals["eps_rel"]
    assert run["rho_r"].default == vals["rescale_rho"]
    assert inspect.signature(O.OracleSolver.rescale).parameters["rho_r"].default == vals["rescale_rho"]
    # F^2 cap: a huge B saturates F at the cap
    F = O.lipschitz_f(np.array([1e30]), 3, O.SD)[0]
    assert F * F == pytest.approx(vals["lipschitz_F2_cap"], rel=1e-15)
    F = O.lipschitz_f(np.array([1e30]), 2, O.SG)[0]
    assert F * F == pytest.approx(vals["lipschitz_F2_cap"], rel=1e-15)
    assert O.init_epsilon(O.SG) == pytest.approx(vals["init_eps_sg"], rel=1e-15)
    assert O.init_epsilon(O.SD) == pytest.approx(vals["init_eps_sd"], rel=1e-15)
    # the P-step floor: a nearly singular S gives eigenvalues raised to sqrt(eps_m)
    S = np.diag([-1e3, -1e3, -1e3])[None]
    P, p = O.p_step(S, np.array([1.0]), np.array([1e6]), O.SG)
    assert np.min(p) >= vals["p_eig_floor"] * (1 - 1e-15)


def test_diagnostic_proxies_closed_forms():
    """The two proxies of the figure with the UV-mapping bounds.
    max |grad f(P)|: eigenvalues p - p^-3 (SD) and p - 1/p (SG), so 0 at the
    identity and 15/8 (SD), 3/2 (SG) at P = diag(2, 1, 1).  Lambda ratio:
    with U = I a symmetric step gives exactly 1 (U L^T U = L), an
    antisymmetric one +inf (the denominator vanishes; up to rounding when the
    states themselves are symmetric), no step 0; the ratio
    is unchanged when the step and both states are rotated by one rotation R
    applied as U -> R U R^T, L -> R L R^T."""
    p = np.array([[2.0, 1.0, 1.0]])
    assert math.sqrt(O.grad_norm_sq_of_spd_eigs(p, O.SD)[0]) == pytest.approx(15 / 8, rel=1e-15)
    assert math.sqrt(O.grad_norm_sq_of_spd_eigs(p, O.SG)[0]) == pytest.approx(3 / 2, rel=1e-15)
    w = mg.flat_grid(6)
    r = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    r.init(w.x0)
    r.iterate(2)
    assert np.all(r.history.col("max_grad_f") < 1e-12)
    rng = np.random.default_rng(3)
    I = np.broadcast_to(np.eye(3), (4, 3, 3))
    L0 = rng.normal(size=(4, 3, 3))
    S = rng.normal(size=(4, 3, 3))
    S = S + np.transpose(S, (0, 2, 1))
    A = rng.normal(size=(4, 3, 3))
    A = A - np.transpose(A, (0, 2, 1))
    L0s = L0 + np.transpose(L0, (0, 2, 1))
    assert np.allclose(O.lambda_ratio(I, L0s, I, L0s + S), 1.0, rtol=1e-14)
    assert np.all(O.lambda_ratio(I, L0s, I, L0s + A) > 1e12)  # 0 up to rounding in the denominator
    assert np.all(np.isinf(O.lambda_ratio(I[:1], np.zeros((1, 3, 3)), I[:1], A[:1])))
    assert np.all(O.lambda_ratio(I, L0, I, L0) == 0.0)
    U0 = np.linalg.qr(rng.normal(size=(4, 3, 3)))[0]
    U1 = np.linalg.qr(rng.normal(size=(4, 3, 3)))[0]
    L1 = L0 + rng.normal(size=(4, 3, 3))
    R = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    rot = lambda X: R @ X @ R.T
    assert np.allclose(O.lambda_ratio(rot(U0), rot(L0), rot(U1), rot(L1)), O.lambda_ratio(U0, L0, U1, L1), rtol=1e-12)


# ----------------------------------------------------------------------------
# Algorithm 2: energies, Phi, thresholds, stop rule, rescaling direction,
# flipped initialisation
# ----------------------------------------------------------------------------

def _rand_rot(r, d, n):
    Q = np.linalg.qr(r.normal(size=(n, d, d)))[0]
    Q[np.linalg.det(Q) < 0, :, 0] *= -1.0
    return Q


def test_energy_density_closed_forms():
    """f at matrices whose values follow by hand from Table 1's definitions
    (SD: 1/2(|X|^2 + |X^-1|^2), SG: 1/2|X|^2 - log det X), for X = R1 S R2
    with rotations R1, R2 (f depends on the singular values only), a shear
    with det 1 and |X|^2 = |X^-1|^2 = 3, and +inf for det X <= 0."""
    r = rng(21)
    for d, S, sd, sg in ((2, [2.0, 1.0], 3.125, 2.5 - math.log(2.0)),
                         (3, [2.0, 1.0, 1.0], 4.125, 3.0 - math.log(2.0)),
                         (3, [0.5, 2.0, 3.0], 0.5 * (13.25 + 4.0 + 0.25 + 1 / 9), 0.5 * 13.25 - math.log(3.0))):
        X = _rand_rot(r, d, 8) @ np.diag(S) @ _rand_rot(r, d, 8)
        assert np.allclose(O.energy_density(X, O.SD), sd, rtol=1e-13)
        assert np.allclose(O.energy_density(X, O.SG), sg, rtol=1e-13)
        Xf = X.copy()
        Xf[:, :, 0] *= -1.0
        assert np.all(np.isinf(O.energy_density(Xf, O.SD))) and np.all(np.isinf(O.energy_density(Xf, O.SG)))
    shear = np.array([[[1.0, 1.0], [0.0, 1.0]]])
    assert O.energy_density(shear, O.SD)[0] == pytest.approx(3.0, rel=1e-15)
    assert O.energy_density(shear, O.SG)[0] == pytest.approx(1.5, rel=1e-15)
    # the eigenvalue form used for E_P agrees with the matrix form on S+
    P = np.diag([0.5, 2.0, 3.0])[None]
    for e in (O.SD, O.SG):
        assert O.energy_of_spd_eigs(np.array([[0.5, 2.0, 3.0]]), e)[0] == pytest.approx(
            O.energy_density(P, e)[0], rel=1e-15)


@pytest.mark.parametrize("energy", [O.SD, O.SG])
def test_history_phi_is_the_augmented_lagrangian(energy):
    """Field Phi of each history record equals eq. augmentedlagrangian
    evaluated at the state the iteration produced, (W^k, U^k, P^k, Lambda^k),
    with f(P) in its matrix form."""
    w = mg.height_field_uv(grid=10, energy=energy)
    s = O.OracleSolver(w.V, w.T, energy, w.rho, w.pinned_idx, w.pinned_pos)
    s.init(w.x0)
    for _ in range(12):
        s.iterate(1)
        J = O.jacobians(s.G, s.x, s.d)
        R = J - s.U @ s.P + s.Lam
        phi = np.sum(s.w * O.energy_density(s.P, energy)
                     + 0.5 * s.mu * (np.sum(R * R, axis=(1, 2)) - np.sum(s.Lam * s.Lam, axis=(1, 2))))
        assert s.history.col("Phi")[-1] == pytest.approx(phi, rel=1e-12)


def test_thresholds_use_sqrt_dm():
    """eq. primaldualthresholds: eps_abs sqrt(d m).  The 32x32 chart has
    d m = 2 * 1922 = 3844 = 62^2; the flat 8x8 grid d m = 2 * 98 = 196 = 14^2
    and, at its identity fixed point (J = P = I, Lambda = 0), |G W| = |P| =
    sqrt(d m) = 14 and |G^T Lambda| = 0."""
    w = mg.height_field_uv()
    s = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    s.init(w.x0)
    s.iterate(2)
    assert s.thresholds(1.0, 0.0) == pytest.approx((62.0, 62.0), rel=1e-15)
    f = mg.flat_grid(8)
    t = O.OracleSolver(f.V, f.T, f.energy, f.rho, f.pinned_idx, f.pinned_pos)
    t.init(f.x0)
    t.iterate(1)
    assert t.thresholds(1.0, 0.0) == pytest.approx((14.0, 14.0), rel=1e-15)
    prim, dual = t.thresholds(0.0, 1.0)
    assert prim == pytest.approx(14.0, rel=1e-13) and abs(dual) < 1e-12


@pytest.mark.parametrize("check_every,flip_free", [(1, True), (7, True), (1, False)])
def test_run_stop_iteration_by_hand(check_every, flip_free):
    """Without rescaling, Algorithm 2 stops at the first check iteration whose
    record meets both inequalities of eq. primaldualthresholds (and, with
    flip_free, has no flipped element): the rule applied by hand to the
    history of a plain run, with sqrt(d m) = 62 on the 32x32 chart."""
    w = mg.height_field_uv()
    a = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    a.init(w.x0)
    done, conv, nres = a.run(400, check_every=check_every, eps_abs=1e-6, eps_rel=1e-5,
                             flip_free=flip_free, rescale=False)
    b = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    b.init(w.x0)
    b.iterate(400)
    H = b.history.array()
    prim = H[:, 0] < 1e-6 * 62.0 + 1e-5 * np.maximum(H[:, 7], H[:, 8])
    dual = H[:, 1] < 1e-6 * 62.0 + 1e-5 * H[:, 9]
    ok = prim & dual & ((H[:, 5] == 0) | (not flip_free))
    ks = np.arange(1, 401)
    hit = ks[ok & (ks % check_every == 0)]
    assert conv and nres == 0 and hit.size > 0 and done == hit[0]
    # the two inequalities are met at different iterations, so swapping
    # "and" for "or" or dropping one would move the stop
    assert np.any(prim[:done - 1] != dual[:done - 1])


def test_run_takes_the_test_on_rescaling_iterations():
    """Algorithm 2 evaluates the termination condition after the rescaling
    block of the same iteration.  From the identity fixed point of the flat
    grid (both residuals 0 at every iteration) the run must stop at
    iteration 1, which is also the first rescaling event."""
    f = mg.flat_grid(8)
    t = O.OracleSolver(f.V, f.T, f.energy, f.rho, f.pinned_idx, f.pinned_pos)
    t.init(f.x0)
    assert t.run(20, check_every=1, rescale=True) == (1, True, 1)


def _rescale_state(rho, dims):
    w = mg.height_field_uv(grid=12, rho=rho) if dims == 2 else mg.twisted_cube(3, rho=rho)
    s = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    s.init(w.x0)
    s.iterate(4)
    return s


@pytest.mark.parametrize("dims", [2, 3])
def test_rescale_direction_by_construction(dims):
    """The rescaling passage: e_prim_i > 5 e_dual_i multiplies mu_i by 5/2 and
    divides Lambda_i by 5/2; e_dual_i > 5 e_prim_i divides mu_i by 5/2 and
    multiplies Lambda_i by it.  States are built so that every element is on
    one side: W^k = W^{k-1} gives e_dual_i = 0 < e_prim_i (all up);
    U_i P_i = J_i (the polar factors of J_i) gives e_prim_i ~ 0 < e_dual_i
    (all down).  rho = 1000 keeps mu_i far above the floor.  After a uniform
    factor s the post-event test values scale as e_dual * s and
    |G^T Lambda| / s."""
    s = _rescale_state(1000.0, dims)
    x, xp, U, P, L = s.x.copy(), s.x_prev.copy(), s.U.copy(), s.P.copy(), s.Lam.copy()
    mu0 = s.mu.copy()
    # all up: no change of the map in the last iteration
    s.set_state(x, U, P, L, x_prev=x)
    J = O.jacobians(s.G, x, s.d)
    assert np.all(np.sqrt(np.sum((J - U @ P) ** 2, axis=(1, 2))) > 0)
    v0 = s.termination_values()
    s.rescale(5.0)
    assert np.allclose(s.mu, 2.5 * mu0, rtol=1e-15)
    assert np.allclose(s.Lam, L / 2.5, rtol=1e-15, atol=0)
    v1 = s.termination_values()
    assert v1["norm_GtLam"] == pytest.approx(v0["norm_GtLam"] / 2.5, rel=1e-13)
    assert v1["e_prim"] == v0["e_prim"] and v1["e_dual"] == 0.0
    # all down: U P = J per element, the map moved in the last iteration
    assert np.all(np.linalg.det(J) > 0)
    R1, S, R2t = np.linalg.svd(J)
    Up, Pp = R1 @ R2t, np.transpose(R2t, (0, 2, 1)) @ (S[:, :, None] * R2t)
    t = _rescale_state(1000.0, dims)
    t.set_state(x, Up, Pp, L, x_prev=xp)
    v0 = t.termination_values()
    assert v0["e_prim"] < 1e-12 and v0["e_dual"] > 1e-3
    t.rescale(5.0)
    assert np.allclose(t.mu, mu0 / 2.5, rtol=1e-15)
    assert np.allclose(t.Lam, L * 2.5, rtol=1e-15, atol=0)
    v1 = t.termination_values()
    assert v1["e_dual"] == pytest.approx(v0["e_dual"] / 2.5, rel=1e-13)
    assert v1["norm_GtLam"] == pytest.approx(v0["norm_GtLam"] * 2.5, rel=1e-13)


def test_flipped_init_is_the_closest_rotation():
    """For a flipped J0 (det <= 0) the reading of the initialisation passage
    gives U0 = the rotation maximising tr(U^T J0) over SO(d) (the closest
    rotation): checked by a brute-force angle search in 2D and by Horn's
    quaternion method in 3D (no SVD); P0 = eps I."""
    r = rng(22)
    J = r.normal(size=(400, 2, 2))
    J = J[np.linalg.det(J) < 0][:60]
    U, P, flipped = O.polar_init(J, O.SD)
    assert np.all(flipped)
    phis = np.linspace(0, 2 * np.pi, 400001)
    for i in range(J.shape[0]):
        val = np.cos(phis) * (J[i, 0, 0] + J[i, 1, 1]) + np.sin(phis) * (J[i, 1, 0] - J[i, 0, 1])
        phi = phis[int(np.argmax(val))]
        Ub = np.array([[math.cos(phi), -math.sin(phi)], [math.sin(phi), math.cos(phi)]])
        assert np.abs(U[i] - Ub).max() < 1e-4
    J = r.normal(size=(400, 3, 3))
    J = J[np.linalg.det(J) < 0][:80]
    U, P, flipped = O.polar_init(J, O.SG)
    assert np.all(flipped)
    for i in range(J.shape[0]):
        Rh, ev = _horn(J[i])
        assert ev[-1] - ev[-2] > 1e-6
        assert np.abs(U[i] - Rh).max() < 1e-9
        assert np.sum(U[i] * J[i]) == pytest.approx(ev[-1], rel=1e-12)
    assert np.allclose(P, O.init_epsilon(O.SG) * np.eye(3), atol=1e-15)


def test_union_of_problems_stops_when_every_problem_passes():
    """A mesh made of two independent charts, declared as two problems, stops
    at the first check where both charts meet eq. primaldualthresholds with
    their own m (sqrt(2 * 98) = 14 and sqrt(2 * 1058) = 46): the later of the
    stops found by hand from each chart's own history."""
    ws = [mg.height_field_uv(grid=8), mg.height_field_uv(grid=24, seed_c=7)]
    oks = []
    for w, root in zip(ws, (14.0, 46.0)):
        r = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
        r.init(w.x0)
        r.iterate(300)
        H = r.history.array()
        oks.append((H[:, 0] < 1e-6 * root + 1e-5 * np.maximum(H[:, 7], H[:, 8]))
                   & (H[:, 1] < 1e-6 * root + 1e-5 * H[:, 9]) & (H[:, 5] == 0))
    ks = np.arange(1, 301)
    both = ks[oks[0] & oks[1] & (ks % 5 == 0)][0]
    assert ks[oks[0] & (ks % 5 == 0)][0] != ks[oks[1] & (ks % 5 == 0)][0]
    voff = np.cumsum([0] + [w.n for w in ws])
    eoff = np.cumsum([0] + [w.m for w in ws])
    u = O.OracleSolver(np.vstack([w.V for w in ws]), np.vstack([w.T + voff[i] for i, w in enumerate(ws)]),
                       ws[0].energy, ws[0].rho, np.concatenate([w.pinned_idx + voff[i] for i, w in enumerate(ws)]),
                       np.vstack([w.pinned_pos for w in ws])).set_problems(eoff, voff)
    u.init(np.vstack([w.x0 for w in ws]))
    assert u.run(300, check_every=5, rescale=False) == (both, True, 0)


def test_nested_dissection_order_is_a_separator_order():
    """The oracle's W-step permutation is a permutation of the free vertices,
    the permuted solve returns the same x as SciPy's sparse solve of the
    unpermuted system, and the dissection order cuts the factor's fill
    against the natural order."""
    import scipy.sparse.linalg as spla
    from oracle import ordering
    w = mg.twisted_cube(6)
    s = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    A = s.L_FF.tocsr()
    X = w.V[s.free]
    p = ordering.nested_dissection(A, X, leaf=16)
    assert np.array_equal(np.sort(p), np.arange(A.shape[0]))
    b = rng(31).normal(size=(A.shape[0], 3))
    x = ordering.SymmetricSolve(A, X).solve(b)
    assert np.linalg.norm(x - spla.spsolve(A.tocsc(), b)) <= 1e-12 * np.linalg.norm(x)
    # an ordering by dissection has a lower-triangular factor much sparser than the natural one
    lu_nd = spla.splu(A[p][:, p].tocsc(), permc_spec="NATURAL", diag_pivot_thresh=0.0,
                      options=dict(SymmetricMode=True))
    lu_nat = spla.splu(A.tocsc(), permc_spec="NATURAL", diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
    assert lu_nd.L.nnz < 0.7 * lu_nat.L.nnz
