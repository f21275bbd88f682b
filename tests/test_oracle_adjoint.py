"""Pins of the tangent (JVP) oracle: float64 central differences of the plain
oracle, the Taylor remainder slope, and the step tangents one by one.  CPU only."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import adjoint as AD
from paper_2107_05200_amd import meshgen as mg


def _dirs(w, rng):
    dV = rng.normal(size=w.V.shape)
    dp = rng.normal(size=w.pinned_pos.shape)
    nrm = math.sqrt((dV ** 2).sum() + (dp ** 2).sum())
    return dV / nrm, dp / nrm


def _loss(w, V, pins, K, energy):
    return AD.loss_only(V, w.T, energy, w.rho, w.pinned_idx, pins, K)


@pytest.mark.parametrize("energy", [O.SD, O.SG])
@pytest.mark.parametrize("case", ["disk", "cube"])
def test_jvp_matches_central_differences(energy, case):
    w = mg.disk_deformation(R=6) if case == "disk" else mg.twisted_cube(2, twist_deg=20.0, lift=0.1)
    K = 10 if case == "disk" else 6
    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(4):
        dV, dp = _dirs(w, rng)
        L, dL = AD.run_jvp(w.V, w.T, energy, w.rho, w.pinned_idx, w.pinned_pos, K, dV, dp)
        assert abs(L - _loss(w, w.V, w.pinned_pos, K, energy)) <= 1e-12 * abs(L)
        fd = (_loss(w, w.V + h * dV, w.pinned_pos + h * dp, K, energy)
              - _loss(w, w.V - h * dV, w.pinned_pos - h * dp, K, energy)) / (2 * h)
        assert abs(dL - fd) <= 1e-6 * max(abs(fd), 1e-3), (dL, fd)


def test_taylor_remainder_slope_two():
    w = mg.disk_deformation(R=5)
    K = 8
    rng = np.random.default_rng(5)
    dV, dp = _dirs(w, rng)
    L0, dL = AD.run_jvp(w.V, w.T, O.SD, w.rho, w.pinned_idx, w.pinned_pos, K, dV, dp)
    hs = [2e-2, 1e-2, 5e-3]
    r = [abs(_loss(w, w.V + h * dV, w.pinned_pos + h * dp, K, O.SD) - L0 - h * dL) for h in hs]
    slopes = [math.log(r[i] / r[i + 1]) / math.log(hs[i] / hs[i + 1]) for i in range(2)]
    assert all(1.7 < s < 2.3 for s in slopes), slopes


def test_rotation_and_spectral_tangents_by_differences():
    rng = np.random.default_rng(3)
    h = 1e-6
    for d in (2, 3):
        Q = rng.normal(size=(40, d, d)) + 2 * np.eye(d)
        dQ = rng.normal(size=(40, d, d))
        U = O.rotation_step(Q, np.tile(np.eye(d), (40, 1, 1)))
        dU = AD.rot_tangent(U, Q, dQ)
        fd = (O.rotation_step(Q + h * dQ, U) - O.rotation_step(Q - h * dQ, U)) / (2 * h)
        assert np.abs(dU - fd).max() < 1e-7
        A_ = rng.normal(size=(40, d, d))
        S = 0.5 * (A_ + np.transpose(A_, (0, 2, 1))) + np.eye(d)
        B_ = rng.normal(size=(40, d, d))
        dS = 0.5 * (B_ + np.transpose(B_, (0, 2, 1)))
        wv = np.full(40, 0.3)
        mu = 10 * wv
        for energy in (O.SD, O.SG):
            P, dP, _ = AD.spectral_tangent(S, dS, wv, mu, energy)
            Pp, _ = O.p_step(S + h * dS, wv, mu, energy)
            Pm, _ = O.p_step(S - h * dS, wv, mu, energy)
            assert np.abs(dP - (Pp - Pm) / (2 * h)).max() < 1e-7
            assert np.abs(P - O.p_step(S, wv, mu, energy)[0]).max() < 1e-12
