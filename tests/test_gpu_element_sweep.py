"""Per-element device checks of the P-step root and the U-step rotation over
the ranges the oracle's pins cover, through ffd_set_state on handles whose
every vertex is fixed at the origin (so J = 0 and the local step sees A = J +
Lambda = the Lambda that was set, exactly; with P^{k-1} = I the U-step input
is Q = A).

* Root sweep (the per-eigenvalue root of the supplement, "Solving the
  Optimization in P"; eqs. peqfsgpluggedin / peqfsdpluggedin): A = diag(2e3,
  [2e3,] q) with q over +-[1e-3, 1e3] per element, so U = I and S = A; each
  rho = mu / w in {1e-3 .. 1e3} on its own handle; the device's P against the
  oracle's P-step of the same S (with its eigenvalue floor), element by
  element: |p - p*| <= 1e-6 p* in float32, 1e-12 p* in float64.
* Rotation ties (supplement, "Solving the Optimization in U"): Q with a
  repeated smallest singular value and det Q < 0, rank-one Q and Q = 0, where
  the closest rotation is not unique: the device's U and the oracle's are
  compared through the objective tr(U^T Q) (within 1e-6 |Q|) and counted;
  det U = 1 always; unique cases also entry by entry."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2107_05200_amd import meshgen as mg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pinned_at_origin(d, energy, rho, prec):
    from paper_2107_05200_amd.binding import Solver
    w = mg.flat_grid(12, energy=energy) if d == 2 else mg.twisted_cube(4, twist_deg=0.0, lift=0.0, energy=energy)
    pins = np.arange(w.n, dtype=np.int32)
    g = Solver(w.V, w.T, energy, rho, pins, np.zeros((w.n, d)), precision=prec)
    return w, g


def _one_step(g, w, d, Lam, prec):
    import torch
    npd = np.float32 if prec == 32 else np.float64
    eye = np.broadcast_to(np.eye(d), (w.m, d, d)).astype(npd)
    g.set_state(np.zeros((w.n, d)), eye, eye, Lam.astype(npd), 0)
    g.iterate(1)
    st = g.get_state()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in st.items()}


def _sweep_values(m):
    mags = 10.0 ** np.linspace(-3.0, 3.0, (m + 1) // 2)
    q = np.concatenate([mags, -mags])[:m]
    return q


@pytest.mark.parametrize("prec", [32, 64])
@pytest.mark.parametrize("energy", [mg.SYMMETRIC_DIRICHLET, mg.SYMMETRIC_GRADIENT])
@pytest.mark.parametrize("d", [2, 3])
def test_root_sweep_matches_oracle(gpu_lib, d, energy, prec):
    worst_all = 0.0
    for rho in (1e-3, 1e-2, 1e-1, 1.0, 10.0, 1e2, 1e3):
        w, g = _pinned_at_origin(d, energy, rho, prec)
        q = _sweep_values(w.m)
        npd = np.float32 if prec == 32 else np.float64
        diag = np.full((w.m, d), 2e3)
        diag[:, -1] = q
        diag = diag.astype(npd).astype(np.float64)  # the values the device holds
        Lam = np.zeros((w.m, d, d))
        Lam[:, np.arange(d), np.arange(d)] = diag
        st = _one_step(g, w, d, Lam, prec)
        g.close()
        wt = O.element_geometry(w.V, w.T)[1]
        Pr, p = O.p_step(Lam, wt, rho * wt, energy)
        assert np.abs(st["U"] - np.eye(d)).max() < 1e-6
        pd = st["P"][:, np.arange(d), np.arange(d)]
        pr = Pr[:, np.arange(d), np.arange(d)]
        off = np.abs(st["P"] - pd[:, :, None] * np.eye(d)).max()
        err = np.abs(pd - pr) / pr
        k = int(np.argmax(err[:, -1]))
        say(f"  d={d} energy={energy} fp{prec} rho={rho:g}: worst |p - p*|/p* {err.max():.2e} "
            f"(q={diag[k, -1]:.4g}, p*={pr[k, -1]:.4g}); off-diagonal {off:.1e}")
        worst_all = max(worst_all, float(err.max()))
        assert err.max() <= (1e-6 if prec == 32 else 1e-12)
        assert off <= 1e-12 * max(1.0, float(np.abs(pr).max()))
    say(f"case: root sweep d={d} energy={energy} fp{prec}: worst {worst_all:.2e}")


def _tie_cases(rng, n):
    """Q = R1 S R2^T: (a) S = (s1, s2, s2) with det(R1 R2^T) = -1 (the smallest
    singular value repeated and det Q < 0: a circle of optimal rotations),
    (b) rank one, (c) zero, (d) generic (unique optimum)."""
    def rot(k):
        R = np.linalg.qr(rng.normal(size=(k, 3, 3)))[0]
        R[np.linalg.det(R) < 0, :, 0] *= -1.0
        return R
    k = n // 4
    out, kind = [], []
    R1, R2 = rot(k), rot(k)
    s = rng.uniform(0.5, 3.0, size=(k, 1))
    S = np.concatenate([s + rng.uniform(0.5, 2.0, size=(k, 1)), s, s], axis=1)
    F = np.diag([1.0, 1.0, -1.0])
    out.append(R1 @ (S[:, :, None] * np.eye(3)) @ F @ np.transpose(R2, (0, 2, 1)))
    kind += ["repeated smallest, det < 0"] * k
    R1, R2 = rot(k), rot(k)
    S = np.zeros((k, 3))
    S[:, 0] = rng.uniform(0.5, 3.0, size=k)
    out.append(R1 @ (S[:, :, None] * np.eye(3)) @ np.transpose(R2, (0, 2, 1)))
    kind += ["rank one"] * k
    out.append(np.zeros((k, 3, 3)))
    kind += ["zero"] * k
    rest = n - 3 * k
    out.append(rng.normal(size=(rest, 3, 3)))
    kind += ["generic"] * rest
    return np.concatenate(out), np.array(kind)


@pytest.mark.parametrize("prec", [32, 64])
def test_rotation_ties_through_the_objective(gpu_lib, prec):
    rng = np.random.default_rng(41)
    w, g = _pinned_at_origin(3, mg.SYMMETRIC_DIRICHLET, 10.0, prec)
    Q, kind = _tie_cases(rng, w.m)
    npd = np.float32 if prec == 32 else np.float64
    Q = Q.astype(npd).astype(np.float64)
    st = _one_step(g, w, 3, Q, prec)
    g.close()
    Ud = st["U"]
    Ur = O.rot3(Q)
    obj_d = np.sum(Ud * Q, axis=(1, 2))
    obj_r = np.sum(Ur * Q, axis=(1, 2))
    scale = np.maximum(np.linalg.norm(Q, axis=(1, 2)), 1.0)
    gap = np.abs(obj_d - obj_r) / scale
    tol = 1e-6 if prec == 32 else 1e-12
    for kd in np.unique(kind):
        sel = kind == kd
        differ = int(np.sum(np.abs(Ud[sel] - Ur[sel]).max(axis=(1, 2)) > 1e-3))
        say(f"  fp{prec} {kd}: {sel.sum()} elements, objective gap max {gap[sel].max():.2e}, "
            f"rotations differing from the oracle's {differ}")
    assert np.all(gap <= tol)
    assert np.abs(np.linalg.det(Ud) - 1.0).max() < (1e-5 if prec == 32 else 1e-12)
    gen = kind == "generic"
    assert np.abs(Ud[gen] - Ur[gen]).max() < (1e-4 if prec == 32 else 1e-10)
