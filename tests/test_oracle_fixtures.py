"""What the oracle's full-size runs (tests/golden/oracle_*.txt, written by the
scripts beside them from the oracle alone) record, checked against what the
method promises at convergence: the primal residual of eq. primaldualerror
falls by orders of magnitude and both thresholds of eq.
primaldualthresholds hold at the paper's pair (1e-6, 1e-5); the final map has
no flipped element (the sphere cap's initial map has hundreds); the energy
of the map, the energy of P and the augmented
Lagrangian of eq. augmentedlagrangian agree once J = U P; |G W| = |P|.  CPU
only, no oracle run: the files are read."""
import math
import os
import sys

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import make_fullsize_fixtures as fixtures  # noqa: E402

# history fields
E_PRIM, E_DUAL, E_P, E_MAP, PHI, FLIPS, NONFINITE, NORM_GW, NORM_P, NORM_GTLAM = range(10)
# (d, m) of the two workloads
SIZES = {"twisted_cube_64": (3, 1572864), "sphere_cap_uv_289": (2, 501126)}


@pytest.mark.parametrize("name", sorted(fixtures.WORKLOADS))
def test_fullsize_run_converges_flip_free(name):
    fx = fixtures.read(name)
    H = fx["hist"]
    _, iters, _ = fixtures.WORKLOADS[name]
    assert H.shape == (iters, 12)
    assert np.all(H[:, NONFINITE] == 0)
    last = H[-1]
    # flip-free at the end, with a finite energy of the map equal to E_P
    assert last[FLIPS] == 0 and math.isfinite(last[E_MAP])
    assert abs(last[E_MAP] - last[E_P]) <= 1e-6 * last[E_P]
    assert abs(last[PHI] - last[E_P]) <= 1e-6 * last[E_P]
    assert abs(last[NORM_GW] - last[NORM_P]) <= 1e-6 * last[NORM_P]
    # the primal residual falls by more than five orders of magnitude
    assert last[E_PRIM] < 1e-5 * H[0, E_PRIM]
    # the termination test of Algorithm 2 holds at the end (paper's pair)
    d, m = SIZES[name]
    base = 1e-6 * math.sqrt(d * m)
    assert last[E_PRIM] < base + 1e-5 * max(last[NORM_GW], last[NORM_P])
    assert last[E_DUAL] < base + 1e-5 * last[NORM_GTLAM]


def test_sphere_cap_starts_flipped():
    """The sphere cap's initial map flips elements (its noise is drawn so);
    the run removes every flip."""
    H = fixtures.read("sphere_cap_uv_289")["hist"]
    assert H[0, FLIPS] > 100 and not math.isfinite(H[0, E_MAP])
    first_free = int(np.argmax(H[:, FLIPS] == 0))
    assert first_free > 0 and np.all(H[first_free:, FLIPS] == 0)


@pytest.mark.parametrize("name", sorted(fixtures.WORKLOADS))
def test_fullsize_samples_are_consistent(name):
    """The sampled map rows, W_el = U P and Lambda at every sampled iteration
    are finite; W_el has a positive determinant (a rotation times an SPD
    matrix) and its symmetric factor is SPD."""
    fx = fixtures.read(name)
    for k in fx["iters"]:
        assert np.all(np.isfinite(fx["map"][k])) and np.all(np.isfinite(fx["lam"][k]))
        W = fx["wel"][k]
        assert np.all(np.linalg.det(W) > 0)
        P = np.array([np.linalg.cholesky(w.T @ w) for w in W])  # P^2 = W^T W is SPD
        assert np.all(np.isfinite(P))
