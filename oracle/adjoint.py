"""Forward-mode tangent (JVP) of K ADMM iterations -- oracle of the adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Differentiated function (deformation setting, d_in == d): the rest vertices V
(which fix the element frames B_i, the weights w_i and mu_i = rho w_i, and the
initial map W^0 = V) and the pinned targets x_C go in; the loss
L = sum_i w_i f(P_i^K) after K iterations of Algorithm 1 (h = 0) comes out.
Because W^0 = V, J^0 = G(V) V is the identity for every V, so U^0 = P^0 = I and
Lambda^0 = 0 carry no tangent.

Each step's tangent follows from differentiating the step as the paper
defines it:
 * W-step (eq. solvinginw): the normal equations (G^T M (G x - Y))_F = 0 with
   Y = U P - Lambda; implicit differentiation gives
   L_FF dx_F = (dG^T M res + G^T dM res + G^T M (dY - dG x - G dx_C))_F,
   res = Y - G x.
 * U-step (eq. optimizationinudecoupled): U = rot(Q); with H = U^T Q
   symmetric, dU = U [w]_x where (tr H I - H) w = vee(U^T dQ - dQ^T U) (3D);
   in 2D U = z/|z| gives d(phi) = (z_re dz_im - z_im dz_re)/|z|^2.
 * P-step (eqs. optimizinginp / rootfindinginp): P = V diag(p(q)) V^T is a
   spectral function of S; dP = V (Gamma o (V^T dS V)) V^T with divided
   differences Gamma_ab = (p_a - p_b)/(q_a - q_b) and Gamma_aa = p'(q_a) =
   mu / (mu + w f_s''(p_a)) (implicit function theorem on the scalar root).
 * Lambda-step (eq. lambdaupdate): linear.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from . import admm as A

__all__ = ["skew_vec", "hat", "rot_tangent", "spectral_tangent", "fpp", "run_jvp", "loss_only"]


def hat(w):
    """[w]_x for w (m, 3)."""
    Z = np.zeros(w.shape[:-1] + (3, 3))
    Z[..., 0, 1] = -w[..., 2]
    Z[..., 0, 2] = w[..., 1]
    Z[..., 1, 0] = w[..., 2]
    Z[..., 1, 2] = -w[..., 0]
    Z[..., 2, 0] = -w[..., 1]
    Z[..., 2, 1] = w[..., 0]
    return Z


def skew_vec(X):
    """vee(X) = (X_21, X_02, X_10) of a (skew) 3x3 matrix."""
    return np.stack([X[..., 2, 1], X[..., 0, 2], X[..., 1, 0]], axis=-1)


def rot_tangent(U, Q, dQ):
    """Tangent of U = rot(Q) (closest rotation)."""
    d = Q.shape[1]
    if d == 2:
        zr = Q[:, 0, 0] + Q[:, 1, 1]
        zi = Q[:, 1, 0] - Q[:, 0, 1]
        dzr = dQ[:, 0, 0] + dQ[:, 1, 1]
        dzi = dQ[:, 1, 0] - dQ[:, 0, 1]
        n2 = zr * zr + zi * zi
        dphi = np.where(n2 > 0, (zr * dzi - zi * dzr) / np.where(n2 > 0, n2, 1.0), 0.0)
        Jm = np.array([[0.0, -1.0], [1.0, 0.0]])
        return (U @ Jm) * dphi[:, None, None]
    H = np.transpose(U, (0, 2, 1)) @ Q
    H = 0.5 * (H + np.transpose(H, (0, 2, 1)))
    K = np.trace(H, axis1=1, axis2=2)[:, None, None] * np.eye(3) - H
    X = np.transpose(U, (0, 2, 1)) @ dQ
    rhs = skew_vec(X - np.transpose(X, (0, 2, 1)))
    w = np.linalg.solve(K, rhs[..., None])[..., 0]
    return U @ hat(w)


def fpp(p, energy):
    """f_s''(p): SD 1 + 3 p^-4, SG 1 + p^-2."""
    return 1.0 + 3.0 / p ** 4 if energy == A.SD else 1.0 + 1.0 / (p * p)


def spectral_tangent(S, dS, w, mu, energy):
    """P = F(S) of the P-step and its tangent dP (divided differences; the
    eigenvalues raised to the floor get a zero derivative)."""
    q, Vs = np.linalg.eigh(S)
    ww, mm = w[:, None], mu[:, None]
    p = A.root_sg(q, ww, mm) if energy == A.SG else A.root_sd(q, ww, mm)
    floor = math.sqrt(A.EPS_M)
    small = (np.prod(p, axis=1) < floor) | (np.sum(p, axis=1) < floor)
    clamped = small[:, None] & (p < floor)
    p = np.where(small[:, None], np.maximum(p, floor), p)
    dp = np.where(clamped, 0.0, mm / (mm + ww * fpp(p, energy)))
    d = S.shape[1]
    G = np.empty(S.shape)
    for a in range(d):
        for b in range(d):
            if a == b:
                G[:, a, a] = dp[:, a]
            else:
                dq = q[:, a] - q[:, b]
                scale = np.maximum(np.abs(q[:, a]) + np.abs(q[:, b]), 1e-300)
                near = np.abs(dq) <= 1e-8 * scale
                G[:, a, b] = np.where(near, 0.5 * (dp[:, a] + dp[:, b]),
                                      (p[:, a] - p[:, b]) / np.where(near, 1.0, dq))
    Vt = np.transpose(Vs, (0, 2, 1))
    dP = Vs @ (G * (Vt @ dS @ Vs)) @ Vt
    P = np.einsum("mij,mj,mkj->mik", Vs, p, Vs)
    return P, dP, p


def _setup(V, T, rho):
    B, w = A.element_geometry(V, T)
    return B, w, rho * w


def run_jvp(V, T, energy, rho, pinned_idx, pins, K, dV, dpins, factor=None):
    """Loss L = sum_i w_i f(P_i^K) and its directional derivative along
    (dV, dpins), with W^0 = V.  Returns (L, dL).

    factor(L_FF) -> object with .solve(b) factorises the free-vertex block;
    the default is SciPy's sparse LU.  Two factorisations agree in exact
    arithmetic, so the spread of their results measures how strongly the K
    iterations amplify rounding."""
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    n, d = V.shape
    if T.shape[1] - 1 != d:
        raise ValueError("the tangent oracle covers d_in == d")
    pins = np.asarray(pins, dtype=np.float64).reshape(-1, d)
    dpins = np.asarray(dpins, dtype=np.float64).reshape(-1, d)
    dV = np.asarray(dV, dtype=np.float64).reshape(n, d)
    pidx = np.asarray(pinned_idx, dtype=np.int64)
    free = np.setdiff1d(np.arange(n), pidx)
    B, w, mu = _setup(V, T, rho)
    dDm = np.transpose(dV[T[:, 1:]] - dV[T[:, [0]]], (0, 2, 1))  # columns are edge tangents
    dB = -B @ np.transpose(dDm, (0, 2, 1)) @ B
    dw = w * np.einsum("mij,mij->m", B, dDm)
    dmu = rho * dw
    G = A.gradient_operator(B, T, n)
    dG = A.gradient_operator(dB, T, n)
    L = A.global_matrix(G, mu, d)
    lu = (factor or spla.splu)(L[free][:, free].tocsc())
    Mrep = np.repeat(mu, d)
    dMrep = np.repeat(dmu, d)
    # initial state W^0 = V: J^0 = I, so U^0 = P^0 = I, Lambda^0 = 0, no tangent
    J0 = A.jacobians(G, V, d)
    if np.abs(J0 - np.eye(d)).max() > 1e-9:
        raise ValueError("W^0 must be the identity map of V")
    m = T.shape[0]
    U = np.tile(np.eye(d), (m, 1, 1))
    P = U.copy()
    Lam = np.zeros_like(U)
    dU = np.zeros_like(U)
    dP = np.zeros_like(U)
    dLam = np.zeros_like(U)
    for _ in range(K):
        Y = U @ P - Lam
        dY = dU @ P + U @ dP - dLam
        # W-step
        x = np.zeros((n, d))
        x[pidx] = pins
        rhs = np.asarray(G.T @ (Mrep[:, None] * (Y.reshape(m * d, d) - np.asarray(G @ x))))
        x[free] = lu.solve(rhs[free])
        Gx = np.asarray(G @ x)
        res = Y.reshape(m * d, d) - Gx
        dxC = np.zeros((n, d))
        dxC[pidx] = dpins
        t = (np.asarray(dG.T @ (Mrep[:, None] * res)) + np.asarray(G.T @ (dMrep[:, None] * res))
             + np.asarray(G.T @ (Mrep[:, None] * (dY.reshape(m * d, d) - np.asarray(dG @ x)
                                                  - np.asarray(G @ dxC)))))
        dx = dxC.copy()
        dx[free] = lu.solve(t[free])
        J = Gx.reshape(m, d, d)
        dJ = (np.asarray(dG @ x) + np.asarray(G @ dx)).reshape(m, d, d)
        # U-step
        Am = J + Lam
        dA = dJ + dLam
        Q = Am @ P
        dQ = dA @ P + Am @ dP
        U1 = A.rotation_step(Q, U)
        dU1 = rot_tangent(U1, Q, dQ)
        # P-step
        M1 = np.transpose(U1, (0, 2, 1)) @ Am
        dM1 = np.transpose(dU1, (0, 2, 1)) @ Am + np.transpose(U1, (0, 2, 1)) @ dA
        S = 0.5 * (M1 + np.transpose(M1, (0, 2, 1)))
        dS = 0.5 * (dM1 + np.transpose(dM1, (0, 2, 1)))
        P1, dP1, p = spectral_tangent(S, dS, w, mu, energy)
        # Lambda-step
        Lam1 = Lam + J - U1 @ P1
        dLam1 = dLam + dJ - dU1 @ P1 - U1 @ dP1
        U, P, Lam, dU, dP, dLam = U1, P1, Lam1, dU1, dP1, dLam1
    # loss and its tangent: f spectral, grad f(P) = V diag(f_s'(p)) V^T
    q, Vs = np.linalg.eigh(P)
    fP = A.energy_of_spd_eigs(q, energy)
    g = q - q ** -3 if energy == A.SD else q - 1.0 / q
    gradf = np.einsum("mij,mj,mkj->mik", Vs, g, Vs)
    loss = float(np.sum(w * fP))
    dloss = float(np.sum(dw * fP) + np.sum(w * np.einsum("mij,mij->m", gradf, dP)))
    return loss, dloss


def loss_only(V, T, energy, rho, pinned_idx, pins, K):
    """The same loss through the plain oracle solver (W^0 = V)."""
    s = A.OracleSolver(V, T, energy, rho, pinned_idx, pins)
    s.init(V)
    s.iterate(K)
    return float(s.history.col("E_P")[-1])
