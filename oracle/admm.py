"""FP64 oracle: discretisation, sub-steps and driver of the flip-free ADMM.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function cites
the passage of the paper it follows.  Readings of passages that are silent or
ambiguous are marked "Reading:".

Conventions (paper, Def. "Piecewise constant Jacobian" and supplement
"Computing the Jacobian Map"): J_i = (G W)_i is d x d with column k equal to
the gradient of output coordinate k on element i.  Element arrays are
(m, d, d) float64.  mu_i = rho * w_i until a rescaling event (OracleSolver.rescale).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .ordering import SymmetricSolve

__all__ = [
    "EPS_M", "SD", "SG", "element_geometry", "gradient_operator", "global_matrix",
    "jacobians", "energy_density", "energy_of_spd_eigs", "grad_norm_sq_of_spd_eigs",
    "root_sg", "root_sd", "rot2", "rot3", "rotation_step", "p_step", "polar_init",
    "init_epsilon", "OracleSolver", "History", "HIST_FIELDS",
    "c_l", "c_lg", "lipschitz_f", "mu_min", "rescale_rule", "rescale_schedule", "lambda_ratio",
]

# Reading: the machine epsilon of the supplement is taken as the float64 one
# for every precision of the GPU path (so both sides clamp at the same values).
EPS_M = 2.0 ** -52
SD = 0  # symmetric Dirichlet, f(X) = 1/2 (|X|^2 + |X^-1|^2)      (Table 1; app. "Symmetric Dirichlet")
SG = 1  # symmetric gradient,  f(X) = 1/2 |X|^2 - log det X      (Table 1; Def. "Symmetric gradient energy")


# ----------------------------------------------------------------------------
# discretisation
# ----------------------------------------------------------------------------

def element_geometry(V: np.ndarray, T: np.ndarray):
    """Per-element B_i = Dm_i^{-T} and weights w_i.

    Supplement "Computing the Jacobian Map": the Jacobian is the piecewise
    linear finite-element gradient; column k of J_i is the gradient of output
    coordinate k.  For a triangle in 3D the gradient is intrinsic (taken in the
    triangle's own plane); for d_in == d it is the coordinate gradient.

    Dm_i has the source edge vectors v_j - v_0 (j = 1..d) as columns, in the
    element's frame; the gradient g of a linear function with increments
    Delta_j along those edges satisfies Dm^T g = Delta, so J_i = Dm^{-T} E_i with
    E_i[j-1, k] = x_{T_ij}[k] - x_{T_i0}[k].  w_i is the area / volume
    (Section "Preliminaries").
    Reading: the intrinsic frame is e1 = normalize(v1 - v0), e2 = n x e1 with
    n the triangle normal (any frame gives the same map, see the rotation
    invariance of f).
    """
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T, dtype=np.int64)
    d = T.shape[1] - 1
    din = V.shape[1]
    E = V[T[:, 1:]] - V[T[:, [0]]]  # (m, d, din): row j = edge j
    if din == d:
        Dm = np.transpose(E, (0, 2, 1))
    elif d == 2 and din == 3:
        e1 = E[:, 0] / np.linalg.norm(E[:, 0], axis=1)[:, None]
        nrm = np.cross(E[:, 0], E[:, 1])
        nrm = nrm / np.linalg.norm(nrm, axis=1)[:, None]
        e2 = np.cross(nrm, e1)
        Dm = np.empty((T.shape[0], 2, 2))
        for j in range(2):
            Dm[:, 0, j] = np.einsum("mk,mk->m", E[:, j], e1)
            Dm[:, 1, j] = np.einsum("mk,mk->m", E[:, j], e2)
    else:
        raise ValueError("unsupported (d, d_in)")
    det = np.linalg.det(Dm)
    w = np.abs(det) / math.factorial(d)
    if not np.all(np.isfinite(w)) or np.any(w <= 1e-300):
        raise ValueError("degenerate element")
    B = np.transpose(np.linalg.inv(Dm), (0, 2, 1))
    return B, w


def gradient_operator(B: np.ndarray, T: np.ndarray, n: int) -> sp.csr_matrix:
    """G as a sparse (m*d) x n matrix: row (i, a) holds C_i[a, c] at column T_ic,
    with C_i[:, 1:] = B_i and C_i[:, 0] = -sum of the others, so that
    (G X)[i*d + a, k] = J_i[a, k] (Def. "Piecewise constant Jacobian")."""
    m, d, _ = B.shape
    C = np.empty((m, d, d + 1))
    C[:, :, 1:] = B
    C[:, :, 0] = -B.sum(axis=2)
    rows = np.repeat(np.arange(m * d), d + 1)
    cols = np.repeat(np.asarray(T, dtype=np.int64), d, axis=0).ravel()
    return sp.csr_matrix((C.ravel(), (rows, cols)), shape=(m * d, n))


def global_matrix(G: sp.csr_matrix, mu: np.ndarray, d: int) -> sp.csr_matrix:
    """L = G^T M G with M = diag(mu) repeated per Jacobian row (eq. solvinginw)."""
    M = sp.diags(np.repeat(mu, d))
    return (G.T @ M @ G).tocsr()


def jacobians(G: sp.csr_matrix, X: np.ndarray, d: int) -> np.ndarray:
    """J = G X reshaped to (m, d, d_o)."""
    return np.asarray(G @ X).reshape(-1, d, X.shape[1])


# ----------------------------------------------------------------------------
# energies
# ----------------------------------------------------------------------------

def energy_density(X: np.ndarray, energy: int) -> np.ndarray:
    """f(X) per matrix, +inf where det X <= 0 (eq. genericdeformationenergy's
    indicator).  SD: 1/2(|X|^2 + |X^-1|^2); SG: 1/2 |X|^2 - log det X."""
    det = np.linalg.det(X)
    out = np.full(X.shape[0], np.inf)
    ok = det > 0
    Xo = X[ok]
    if energy == SD:
        inv = np.linalg.inv(Xo)
        out[ok] = 0.5 * (np.sum(Xo * Xo, axis=(1, 2)) + np.sum(inv * inv, axis=(1, 2)))
    else:
        out[ok] = 0.5 * np.sum(Xo * Xo, axis=(1, 2)) - np.log(det[ok])
    return out


def energy_of_spd_eigs(p: np.ndarray, energy: int) -> np.ndarray:
    """f(P) for symmetric positive definite P with eigenvalues p (m, d)."""
    if energy == SD:
        return 0.5 * np.sum(p * p + 1.0 / (p * p), axis=1)
    return 0.5 * np.sum(p * p, axis=1) - np.sum(np.log(p), axis=1)


def grad_norm_sq_of_spd_eigs(p: np.ndarray, energy: int) -> np.ndarray:
    """|grad f(P)|^2 on S+: eigenvalues p - p^-3 (SD, eq. symmetricdirichletdefininggrad)
    or p - p^-1 (SG, eq. symmetricgradientdefininggrad)."""
    g = p - p ** -3 if energy == SD else p - 1.0 / p
    return np.sum(g * g, axis=1)


# ----------------------------------------------------------------------------
# P-step: scalar roots (supplement "Solving the Optimization in P")
# ----------------------------------------------------------------------------

def root_sg(q, w, mu):
    """Positive root of (w+mu) p^2 - mu q p - w = 0 (eq. peqfsgpluggedin per
    eigenvalue), i.e. the quadratic formula of eq. solvesgwithquadraticformula;
    for q < 0 the algebraically equal conjugate form avoids cancellation."""
    q = np.asarray(q, dtype=np.float64)
    w = np.broadcast_to(np.asarray(w, dtype=np.float64), q.shape)
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), q.shape)
    disc = np.sqrt((mu * q) ** 2 + 4.0 * w * (w + mu))
    pos = (mu * q + disc) / (2.0 * (w + mu))
    with np.errstate(divide="ignore", invalid="ignore"):
        neg = 2.0 * w / (disc - mu * q)
    return np.where(q >= 0, pos, neg)


def _h_sd(p, q, w, mu):
    # (w+mu) p - w p^-3 - mu q: the quartic of eq. peqfsdpluggedin divided by p^3
    return (w + mu) * p - w / (p * p * p) - mu * q


def root_sd(q, w, mu, iters: int = 100):
    """Unique positive root of (w+mu) p^4 - mu q p^3 - w = 0 (eq. peqfsdpluggedin
    per eigenvalue) by bisection, then one Newton step.

    h(p) = (w+mu) p - w p^-3 - mu q is strictly increasing on (0, inf), so the
    root is unique.  Bracket: for q >= 0, lo = max((w/(w+mu))^(1/4), mu q/(w+mu));
    for q < 0, lo = min((w/(2(w+mu)))^(1/4), (w/(2 mu |q|))^(1/3)); in both
    cases h(lo) <= 0 and hi = max(1, (w + mu q)/(w+mu)) has h(hi) >= 0."""
    q = np.asarray(q, dtype=np.float64)
    w = np.broadcast_to(np.asarray(w, dtype=np.float64), q.shape)
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), q.shape)
    lo_pos = np.maximum((w / (w + mu)) ** 0.25, mu * q / (w + mu))
    with np.errstate(divide="ignore"):
        lo_neg = np.minimum((w / (2.0 * (w + mu))) ** 0.25,
                            (w / (2.0 * mu * np.maximum(-q, 1e-300))) ** (1.0 / 3.0))
    lo = np.where(q >= 0, lo_pos, lo_neg)
    hi = np.maximum(1.0, (w + mu * q) / (w + mu))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        neg = _h_sd(mid, q, w, mu) <= 0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    p = 0.5 * (lo + hi)
    dh = (w + mu) + 3.0 * w / p ** 4
    pn = p - _h_sd(p, q, w, mu) / dh
    better = np.abs(_h_sd(pn, q, w, mu)) < np.abs(_h_sd(p, q, w, mu))
    return np.where(better & (pn > 0), pn, p)


def p_step(S: np.ndarray, w: np.ndarray, mu: np.ndarray, energy: int):
    """argmin over SPD P of w f(P) + mu/2 |P - S|^2 for symmetric S (eqs.
    optimizinginp / rootfindinginp): f is spectral and convex on S+, so P shares
    S's eigenvectors and each eigenvalue solves the scalar root problem
    (supplement "Solving the Optimization in P").  If det P or tr P falls below
    sqrt(eps_m), the eigenvalues are raised to at least sqrt(eps_m) (supplement,
    last paragraph of that subsection).  Returns (P, eigenvalues p)."""
    q, Qs = np.linalg.eigh(S)
    ww = w[:, None]
    mm = mu[:, None]
    p = root_sg(q, ww, mm) if energy == SG else root_sd(q, ww, mm)
    floor = math.sqrt(EPS_M)
    small = (np.prod(p, axis=1) < floor) | (np.sum(p, axis=1) < floor)
    p = np.where(small[:, None], np.maximum(p, floor), p)
    P = np.einsum("mij,mj,mkj->mik", Qs, p, Qs)
    return P, p


# ----------------------------------------------------------------------------
# U-step: Procrustes (supplement "Solving the Optimization in U")
# ----------------------------------------------------------------------------

def rot2(Q: np.ndarray, U_prev: np.ndarray) -> np.ndarray:
    """d = 2 (eq. twodprocrustes): maximise U(phi) . Q = cos(phi)(Q00+Q11) +
    sin(phi)(Q10-Q01); U is the unit complex number z/|z|, z = (Q00+Q11) +
    i (Q10-Q01).  Reading: where z = 0 every rotation is optimal and the previous
    rotation is kept."""
    c = Q[:, 0, 0] + Q[:, 1, 1]
    s = Q[:, 1, 0] - Q[:, 0, 1]
    nz = np.hypot(c, s)
    U = U_prev.copy()
    ok = nz > 0
    c = c[ok] / nz[ok]
    s = s[ok] / nz[ok]
    U[ok, 0, 0] = c
    U[ok, 0, 1] = -s
    U[ok, 1, 0] = s
    U[ok, 1, 1] = c
    return U


def rot3(Q: np.ndarray) -> np.ndarray:
    """d = 3: closest rotation via the SVD Q = R1 S R2^T (supplement, d = 3):
    U = R1 diag(1, 1, det(R1 R2^T)) R2^T."""
    R1, _, R2t = np.linalg.svd(Q)
    s = np.sign(np.linalg.det(R1 @ R2t))
    s[s == 0] = 1.0
    D = np.ones((Q.shape[0], 3))
    D[:, 2] = s
    return np.einsum("mij,mj,mjk->mik", R1, D, R2t)


def rotation_step(Q: np.ndarray, U_prev: np.ndarray) -> np.ndarray:
    """argmin over SO(d) of |U - Q|^2 (eq. optimizationinudecoupled)."""
    return rot2(Q, U_prev) if Q.shape[1] == 2 else rot3(Q)


# ----------------------------------------------------------------------------
# initialisation (Section "Implementation", "Initializing U, P, Lambda")
# ----------------------------------------------------------------------------

def init_epsilon(energy: int) -> float:
    """eps = eps_m^(1/4) for the symmetric gradient energy, eps_m^(1/8) for the
    symmetric Dirichlet energy (eq. polardecompositionapplied and the text after)."""
    return EPS_M ** 0.25 if energy == SG else EPS_M ** 0.125


def polar_init(J0: np.ndarray, energy: int):
    """U0, P0 from the SVD J0 = R1 S R2^T (eqs. initialpolardecomposition,
    polardecompositionapplied): U0 = R1 R2^T, P0 = R2 S R2^T; singular values
    below eps are raised to eps.  Reading: an element is flipped when det J0 <= 0;
    then U0 = R1 diag(1, .., det(R1 R2^T)) R2^T (the last column of R1 negated,
    singular values sorted descending) and S = eps I."""
    d = J0.shape[1]
    eps = init_epsilon(energy)
    R1, sig, R2t = np.linalg.svd(J0)
    flipped = np.linalg.det(J0) <= 0
    s = np.sign(np.linalg.det(R1 @ R2t))
    s[s == 0] = 1.0
    D = np.ones((J0.shape[0], d))
    D[:, -1] = s
    U = np.einsum("mij,mj,mjk->mik", R1, D, R2t)
    sig = np.maximum(sig, eps)
    sig[flipped] = eps
    P = np.einsum("mji,mj,mjk->mik", R2t, sig, R2t)
    return U, P, flipped


# ----------------------------------------------------------------------------
# driver (Algorithm 1 with the fixed penalties of Algorithm 2's loop)
# ----------------------------------------------------------------------------

HIST_FIELDS = ("e_prim", "e_dual", "E_P", "E_map", "Phi", "flips", "nonfinite",
               "norm_GW", "norm_P", "norm_GtLam", "max_grad_f", "max_lambda_ratio")


def lambda_ratio(U0, L0, U1, L1):
    """Per element, the ratio the paper plots as a proxy for gamma^(1/2) of
    Condition "lambdabound" (caption of the figure with the UV-mapping
    bounds): |L1 - L0| / |1/2 (L1 - L0 + U1 L1^T U1 - U0 L0^T U0)| for
    consecutive iterates.  Reading: the figure scales Lambda by mu_i so that
    iterates compare across rescalings; within one iteration mu_i is the same
    on both sides and cancels, and after a rescaling event the stored scaled
    dual is already divided by the event's factor.  A zero denominator gives
    +inf when the numerator is positive and 0 when it is zero."""
    tr = lambda X: np.transpose(X, (0, 2, 1))
    num = np.sqrt(np.sum((L1 - L0) ** 2, axis=(1, 2)))
    den = 0.5 * np.sqrt(np.sum((L1 - L0 + U1 @ tr(L1) @ U1 - U0 @ tr(L0) @ U0) ** 2, axis=(1, 2)))
    with np.errstate(divide="ignore", invalid="ignore"):
        r = num / den
    return np.where(den > 0, r, np.where(num > 0, np.inf, 0.0))


@dataclass
class History:
    rows: list = field(default_factory=list)

    def array(self) -> np.ndarray:
        return np.asarray(self.rows, dtype=np.float64).reshape(-1, len(HIST_FIELDS))

    def col(self, name: str) -> np.ndarray:
        return self.array()[:, HIST_FIELDS.index(name)]


# ----------------------------------------------------------------------------
# penalty rescaling (Section "Implementation", "Rescaling mu_i and Lambda";
# Lemma "local Lipschitz constant" and Prop. "Sufficient decrease")
# ----------------------------------------------------------------------------

def c_l(B):
    """C^L of the Lipschitz lemma, (-B + sqrt(4 + B^2)) / 2: the positive root
    of x^2 + B x - 1 = 0, evaluated as 2 / (B + sqrt(4 + B^2)) (the same
    number without the cancellation of the printed form at large B)."""
    B = np.asarray(B, dtype=np.float64)
    return 2.0 / (B + np.sqrt(4.0 + B * B))


def c_lg(B, iters: int = 200):
    """C^LG of the Lipschitz lemma: the positive root of x^4 + B x^3 - 1 = 0
    (bisection on [0, 1]: the polynomial is -1 at 0 and B >= 0 at 1)."""
    B = np.asarray(B, dtype=np.float64)
    lo, hi = np.zeros_like(B), np.ones_like(B)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        neg = mid ** 4 + B * mid ** 3 - 1.0 < 0.0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    return 0.5 * (lo + hi)


def lipschitz_f(B, d: int, energy: int):
    """F_i of the Lipschitz lemma (SG: 1 + sqrt(d) / C^L^2, SD: 1 + 3 sqrt(d) /
    C^LG^4), with F_i^2 capped at eps_m^(-1/4) as the rescaling passage does."""
    F = 1.0 + math.sqrt(d) / c_l(B) ** 2 if energy == SG else 1.0 + 3.0 * math.sqrt(d) / c_lg(B) ** 4
    return np.minimum(F, math.sqrt(EPS_M ** -0.25))


def mu_min(w, F):
    """The penalty bound of Prop. "Sufficient decrease" with gamma = 1 and
    epsilon = 0: 1/2 (-w + sqrt(w^2 + 16 w^2 F^2))."""
    w = np.asarray(w, dtype=np.float64)
    return 0.5 * (-w + np.sqrt(w * w + 16.0 * w * w * F * F))


def rescale_rule(mu, e_prim, e_dual, floor, rho_r: float = 5.0):
    """One rescaling event per element: e_prim > rho_r e_dual multiplies mu by
    rho_r / 2 (and divides the scaled dual Lambda by it); e_dual > rho_r e_prim
    divides mu by rho_r / 2 (multiplies Lambda); mu never goes below floor
    (half the bound of Prop. "Sufficient decrease").  Returns (new mu, the
    factor s with Lambda_new = Lambda / s, s = mu_new / mu)."""
    mu = np.asarray(mu, dtype=np.float64)
    up = e_prim > rho_r * e_dual
    down = e_dual > rho_r * e_prim
    new = np.where(up, mu * (0.5 * rho_r), np.where(down, mu / (0.5 * rho_r), mu))
    new = np.maximum(new, floor)
    return new, new / mu


def rescale_schedule(max_iter: int):
    """Iterations after which Algorithm 2 rescales: five directly after the
    initialisation (after iterations 1..5), then every 5 (3/2)^p iterations
    with p the number of past events (rounded half up)."""
    ks, k, p = [], 0, 0
    while True:
        k = k + 1 if p < 5 else k + int(math.floor(5.0 * 1.5 ** p + 0.5))
        if k > max_iter:
            return ks
        ks.append(k)
        p += 1


class OracleSolver:
    """Plain FP64 reference of the per-iteration ADMM loop.

    State after iteration k: x (n, d) map W^k, U, P, Lam (m, d, d).
    mu_i = rho w_i (fixed).  h_mode 0: h_i = 0; h_mode 1: h_i = 4 w_i^2 B_i^2 / mu_i
    with B_i = sqrt(5 (1 + |grad f(P_i^{k-1})|^2)) (Prop. "Sufficient decrease",
    gamma = 1, epsilon = 0, and the B_i of Section "Implementation").
    """

    def __init__(self, V, T, energy: int, rho: float, pinned_idx, pinned_pos, h_mode: int = 0,
                 constraints=None):
        self.V = np.asarray(V, dtype=np.float64)
        self.T = np.asarray(T, dtype=np.int64)
        self.n = self.V.shape[0]
        self.m = self.T.shape[0]
        self.d = self.T.shape[1] - 1
        self.energy = int(energy)
        self.rho = float(rho)
        self.h_mode = int(h_mode)
        self.B, self.w = element_geometry(self.V, self.T)
        self.mu = self.rho * self.w
        self.G = gradient_operator(self.B, self.T, self.n)
        self.L = global_matrix(self.G, self.mu, self.d)
        pins = np.asarray(pinned_idx if pinned_idx is not None else [], dtype=np.int64)
        # general linear constraints A W = c (eq. solvinginw): A is (rows, n),
        # c is (rows, d); the pins are the constraints that fix a vertex
        self.A = None if constraints is None else sp.csr_matrix(constraints[0], dtype=np.float64)
        self.c = None if constraints is None else \
            np.asarray(constraints[1], dtype=np.float64).reshape(self.A.shape[0], self.d)
        if pins.size == 0 and self.A is None:
            pins = np.array([0], dtype=np.int64)  # no constraints: fix the first vertex (W-step text)
            self.auto_pinned = True
        else:
            self.auto_pinned = False
        self.pins = pins
        self.pin_pos = None if (self.auto_pinned or pinned_pos is None) else \
            np.asarray(pinned_pos, dtype=np.float64).reshape(-1, self.d)
        if pins.size == 0:
            self.pin_pos = np.zeros((0, self.d))
        self.free = np.setdiff1d(np.arange(self.n), pins)
        self.L_FF = self.L[self.free][:, self.free].tocsc()
        self.L_FC = self.L[self.free][:, pins].tocsr()
        self._lu = None  # factorised at the first W-step (once: mu is fixed)
        self.problems = None  # one problem: the whole mesh (set_problems)
        self.k = 0
        self.history = History()

    # -- state ---------------------------------------------------------------
    def init(self, x0):
        """Polar initialisation of U, P from the caller's W^0 as given; Lambda0 = 0
        (Algorithm 2, first lines).  Reading: the constraints are imposed by the
        W-step (eq. solvinginw), not on W^0 -- a deformation starts from the
        identity map with the handles still at rest (caption of the 3D
        deformation figure).  Without given pin positions they are taken from W^0."""
        x0 = np.asarray(x0, dtype=np.float64).reshape(self.n, self.d).copy()
        if self.pin_pos is None:
            self.pin_pos = x0[self.pins].copy()
        self.x = x0
        self.x_prev = x0.copy()
        J0 = jacobians(self.G, self.x, self.d)
        self.U, self.P, self.init_flipped = polar_init(J0, self.energy)
        self.Lam = np.zeros_like(self.U)
        self.k = 0
        self.history = History()
        self.h = np.zeros(self.m)
        if self.h_mode == 1:
            self.h = self._prox_h(self.P)

    def set_state(self, x, U, P, Lam, k=0, x_prev=None):
        self.x = np.array(x, dtype=np.float64).reshape(self.n, self.d)
        self.x_prev = self.x.copy() if x_prev is None else np.array(x_prev, dtype=np.float64)
        self.U = np.array(U, dtype=np.float64)
        self.P = np.array(P, dtype=np.float64)
        self.Lam = np.array(Lam, dtype=np.float64)
        self.k = k
        if self.pin_pos is None:
            self.pin_pos = self.x[self.pins].copy()
        self.h = self._prox_h(self.P) if self.h_mode == 1 else np.zeros(self.m)

    def set_pins(self, pos):
        self.pin_pos = np.asarray(pos, dtype=np.float64).reshape(-1, self.d).copy()

    def _prox_h(self, P):
        p = np.linalg.eigvalsh(P)
        Bsq = 5.0 * (1.0 + grad_norm_sq_of_spd_eigs(p, self.energy))
        return 4.0 * self.w ** 2 * Bsq / self.mu

    def rescale(self, rho_r: float = 5.0):
        """One rescaling event after the last iteration (Section
        "Implementation", "Rescaling mu_i and Lambda"): per element e_prim_i =
        |J_i - U_i P_i|, e_dual_i = mu_i |J_i - J_i^prev| of that iteration,
        B_i = sqrt(5 (1 + |grad f(P_i)|^2)), the floor 1/2 mu_min(w_i, F_i);
        then L = G^T M G is assembled and factorised again."""
        J = jacobians(self.G, self.x, self.d)
        J_prev = jacobians(self.G, self.x_prev, self.d)
        e_prim = np.sqrt(np.sum((J - self.U @ self.P) ** 2, axis=(1, 2)))
        e_dual = self.mu * np.sqrt(np.sum((J - J_prev) ** 2, axis=(1, 2)))
        p = np.linalg.eigvalsh(self.P)
        B = np.sqrt(5.0 * (1.0 + grad_norm_sq_of_spd_eigs(p, self.energy)))
        floor = 0.5 * mu_min(self.w, lipschitz_f(B, self.d, self.energy))
        self.mu, s = rescale_rule(self.mu, e_prim, e_dual, floor, rho_r)
        self.Lam = self.Lam / s[:, None, None]
        self.L = global_matrix(self.G, self.mu, self.d)
        self.L_FF = self.L[self.free][:, self.free].tocsc()
        self.L_FC = self.L[self.free][:, self.pins].tocsr()
        self._lu = None
        if self.h_mode == 1:
            self.h = self._prox_h(self.P)
        return self

    def run(self, max_iter: int, check_every: int = 1, eps_abs: float = 1e-6, eps_rel: float = 1e-5,
            flip_free: bool = True, rescale: bool = True, rho_r: float = 5.0):
        """Algorithm 2 (the paper's implementation of Algorithm 1): iterate;
        after the iterations of rescale_schedule rescale mu and Lambda; then, in
        the same iteration and after any rescaling (the order of Algorithm 2's
        loop body), take the termination test at every check_every-th
        iteration: eq. primaldualthresholds plus the flip-free condition, on
        the state as it stands (termination_values).  Returns (iterations run,
        converged, rescaling events)."""
        events = set(rescale_schedule(max_iter)) if rescale else set()
        nres = 0
        for k in range(1, max_iter + 1):
            self.iterate(1)
            if k in events:
                self.rescale(rho_r)
                nres += 1
            if k % check_every == 0 and self.termination_test(eps_abs, eps_rel, flip_free):
                return k, True, nres
        return max_iter, False, nres

    def set_problems(self, element_offsets, vertex_offsets):
        """Declare the mesh a union of independent problems (a batch): problem
        c owns elements [element_offsets[c], element_offsets[c+1]) and vertices
        [vertex_offsets[c], vertex_offsets[c+1]).  The termination test is
        then taken per problem (each with its own m), and passes when it
        passes for every problem."""
        self.problems = list(zip(element_offsets[:-1], element_offsets[1:], vertex_offsets[:-1], vertex_offsets[1:]))
        return self

    def termination_values(self, problem=None):
        """The quantities of Algorithm 2's termination test for the current
        state (W^k, U^k, P^k, Lambda^k) with the current penalties mu: e_prim
        and e_dual of eq. primaldualerror, |G W^k|, |P^k| and |G^T Lambda^k| of
        eq. primaldualthresholds, the number of elements with det J <= 0, and
        m; over the whole mesh or over problem (e0, e1, v0, v1) (its elements
        and its vertex rows).  Reading: after a rescaling event of the same
        iteration, e_dual uses the new mu_i and |G^T Lambda| the rescaled
        Lambda (e_prim, |G W|, |P| and the flips do not depend on mu or
        Lambda); otherwise these are the values of the iteration's history
        record."""
        e0, e1, v0, v1 = problem if problem is not None else (0, self.m, 0, self.n)
        J = jacobians(self.G, self.x, self.d)[e0:e1]
        J_prev = jacobians(self.G, self.x_prev, self.d)[e0:e1]
        UP = (self.U @ self.P)[e0:e1]
        GtLam = np.asarray(self.G.T @ self.Lam.reshape(self.m * self.d, self.d))[v0:v1]
        mu = self.mu[e0:e1]
        return {"e_prim": math.sqrt(np.sum((J - UP) ** 2)),
                "e_dual": math.sqrt(np.sum(mu[:, None, None] ** 2 * (J - J_prev) ** 2)),
                "norm_GW": math.sqrt(np.sum(J * J)), "norm_P": math.sqrt(np.sum(self.P[e0:e1] ** 2)),
                "norm_GtLam": math.sqrt(np.sum(GtLam ** 2)),
                "flips": int(np.sum(np.linalg.det(J) <= 0)), "m": e1 - e0}

    def thresholds(self, eps_abs=1e-6, eps_rel=1e-5, problem=None):
        """Primal / dual thresholds of eq. primaldualthresholds for the current
        state: eps_abs sqrt(d m) + eps_rel max(|G W|, |P|) and eps_abs sqrt(d m)
        + eps_rel |G^T Lambda| (sqrt(d m) as printed; m of the problem)."""
        v = self.termination_values(problem)
        base = eps_abs * math.sqrt(self.d * v["m"])
        return base + eps_rel * max(v["norm_GW"], v["norm_P"]), base + eps_rel * v["norm_GtLam"]

    def termination_test(self, eps_abs=1e-6, eps_rel=1e-5, flip_free=True):
        """Algorithm 2's termination condition: both residuals below their
        thresholds and, with flip_free, no element with det J <= 0; for a
        union of problems, for each of them."""
        for pr in (self.problems if self.problems else [None]):
            v = self.termination_values(pr)
            prim, dual = self.thresholds(eps_abs, eps_rel, pr)
            if not (v["e_prim"] < prim and v["e_dual"] < dual and (not flip_free or v["flips"] == 0)):
                return False
        return True

    # -- sub-steps -----------------------------------------------------------
    def w_step(self, U, P, Lam):
        """argmin over W with the pins of Phi (eq. solvinginw): L W = G^T r with
        r_i = mu_i (U_i P_i - Lam_i); pinned rows eliminated.  With general
        constraints A W = c the minimiser solves the KKT system
        [L_FF A_F^T; A_F 0] [W_F; Y] = [b; c - A_C W_C] (sparse LU, which
        takes the indefinite matrix as it is)."""
        r = self.mu[:, None, None] * (U @ P - Lam)
        rhs = np.asarray(self.G.T @ r.reshape(self.m * self.d, self.d))
        b = rhs[self.free] - self.L_FC @ self.pin_pos
        x = np.empty((self.n, self.d))
        x[self.pins] = self.pin_pos
        if self.free.size == 0:  # every vertex fixed: the W-step is the constraint itself
            return x
        if self.A is None:
            if self._lu is None:  # SPD: nested-dissection order (oracle/ordering.py), then SuperLU
                self._lu = SymmetricSolve(self.L_FF, self.V[self.free])
            x[self.free] = self._lu.solve(b)
            return x
        AF = self.A[:, self.free]
        cF = self.c - self.A[:, self.pins] @ self.pin_pos
        if self._lu is None:
            self._lu = spla.splu(sp.bmat([[self.L_FF, AF.T], [AF, None]]).tocsc())
        x[self.free] = self._lu.solve(np.vstack([b, cF]))[:self.free.size]
        return x

    def set_constraint_rhs(self, c):
        """New right-hand sides c of the constraints A W = c."""
        self.c = np.asarray(c, dtype=np.float64).reshape(self.A.shape[0], self.d)

    def iterate(self, n_iter: int = 1):
        """Algorithm 1: W, then U (with P^{k-1}, Lam^{k-1}), then P (with U^k,
        Lam^{k-1}), then Lam; diagnostics of eq. primaldualerror afterwards."""
        for _ in range(n_iter):
            self.local_steps(self.w_step(self.U, self.P, self.Lam))
        return self

    def local_steps(self, x_new):
        """The element-wise part of one iteration given W^k = x_new: U-step,
        P-step, Lambda-step and the diagnostics; advances the state."""
        J = jacobians(self.G, x_new, self.d)
        J_prev = jacobians(self.G, self.x, self.d)
        A = J + self.Lam
        Q = A @ self.P + (self.h / self.mu)[:, None, None] * self.U
        U = rotation_step(Q, self.U)
        At = np.transpose(U, (0, 2, 1)) @ A
        S = 0.5 * (At + np.transpose(At, (0, 2, 1)))
        P, p = p_step(S, self.w, self.mu, self.energy)
        UP = U @ P
        Lam = self.Lam + J - UP
        ratio = float(np.max(lambda_ratio(self.U, self.Lam, U, Lam)))
        self.x_prev, self.x = self.x, x_new
        self.U, self.P, self.Lam = U, P, Lam
        self.k += 1
        self.history.rows.append(self._diagnostics(J, J_prev, UP, p) + [ratio])
        if self.h_mode == 1:
            self.h = self._prox_h(self.P)
        return self

    def _diagnostics(self, J, J_prev, UP, p):
        """e_prim, e_dual (eq. primaldualerror), E_P = sum w f(P), E_map = sum w f(J)
        (+inf with any det J <= 0), Phi (eq. augmentedlagrangian at the new
        iterate), flip count, non-finite count, the norms used by the
        thresholds of eq. primaldualthresholds, and max_i |grad f(P_i)| (the
        proxy for the B_i of Condition "gradf" in the figure with the UV-mapping
        bounds)."""
        mu, w = self.mu, self.w
        e_prim = math.sqrt(np.sum((J - UP) ** 2))
        e_dual = math.sqrt(np.sum(mu[:, None, None] ** 2 * (J - J_prev) ** 2))
        fP = energy_of_spd_eigs(p, self.energy)
        E_P = float(np.sum(w * fP))
        detJ = np.linalg.det(J)
        flips = int(np.sum(detJ <= 0))
        E_map = float(np.sum(w * energy_density(J, self.energy))) if flips == 0 else math.inf
        R = J - UP + self.Lam
        Phi = float(np.sum(w * fP + 0.5 * mu * (np.sum(R * R, axis=(1, 2))
                                                  - np.sum(self.Lam ** 2, axis=(1, 2)))))
        nonfinite = int(np.sum(~np.isfinite(self.Lam).all(axis=(1, 2))))
        GtLam = np.asarray(self.G.T @ self.Lam.reshape(self.m * self.d, self.d))
        gmax = math.sqrt(float(np.max(grad_norm_sq_of_spd_eigs(p, self.energy))))
        return [e_prim, e_dual, E_P, E_map, Phi, flips, nonfinite,
                math.sqrt(np.sum(J * J)), math.sqrt(np.sum(self.P ** 2)),
                math.sqrt(np.sum(GtLam ** 2)), gmax]

    def wel(self):
        """Per-element U_i P_i (the flip-free Jacobian estimate)."""
        return self.U @ self.P
