"""Write the oracle's fixture for the adjoint check at K = 100 on the full disk.

Calls only the oracle (``oracle/``) and the seeded workload generator; no
value comes from the GPU library.  Workload: the 99,846-triangle disk
deformation, loss sum_i w_i f(P_i^K) after K = 100 iterations from W^0 = V.
For each of 20 seeded unit directions (``meshgen.unit_tangents``, seed 21)
over (rest vertices, pinned targets) the oracle's forward-mode tangent is
taken twice, with two factorisations of L_FF that agree in exact arithmetic:
SciPy's sparse LU (column ordering COLAMD) and a Cholesky-pivoted LU under the
oracle's own nested-dissection order.  The two differ only by rounding, so
their spread is the precision to which the K-step derivative is determined
at all.  The file also records, along the oracle's trajectory, how close the
iteration comes to its two non-smooth branches: the 2D rotation step's
z = 0 (min over iterations and elements of |z| / |Q|_F) and the P-step's
eigenvalue floor (min over iterations and elements of min(p1 p2, p1 + p2)
divided by the floor).

Usage (from the repository root; about 15 minutes on 6 cores):
    python tests/golden/make_adjoint_k100_fixture.py
"""
from __future__ import annotations

import math
import os
import sys
import time
from multiprocessing import Pool

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import adjoint as AD  # noqa: E402
from oracle import ordering  # noqa: E402
from paper_2107_05200_amd import meshgen as mg  # noqa: E402

K = 100
N_DIR = 20
DIR_SEED = 21
PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_disk_adjoint_k100.txt")


def _one(j):
    w = mg.disk_deformation()
    dV, dp = mg.unit_tangents(w, N_DIR, DIR_SEED)[j]
    free = np.setdiff1d(np.arange(w.n), w.pinned_idx)
    t0 = time.perf_counter()
    L1, d1 = AD.run_jvp(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, K, dV, dp)
    L2, d2 = AD.run_jvp(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, K, dV, dp,
                        factor=lambda A: ordering.SymmetricSolve(A, w.V[free]))
    print(f"direction {j}: L {L1:.15g} dL {d1:.12g} / {d2:.12g} ({time.perf_counter() - t0:.0f} s)", flush=True)
    return j, L1, d1, L2, d2


def _branch_margins():
    w = mg.disk_deformation()
    s = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    s.init(w.V)
    floor = math.sqrt(O.EPS_M)
    zmin, fmin = np.inf, np.inf
    for _ in range(K):
        x = s.w_step(s.U, s.P, s.Lam)
        J = O.jacobians(s.G, x, 2)
        Q = (J + s.Lam) @ s.P
        z = np.hypot(Q[:, 0, 0] + Q[:, 1, 1], Q[:, 1, 0] - Q[:, 0, 1])
        zmin = min(zmin, float(np.min(z / np.linalg.norm(Q, axis=(1, 2)))))
        s.local_steps(x)
        p = np.linalg.eigvalsh(s.P)
        fmin = min(fmin, float(np.min(np.minimum(p[:, 0] * p[:, 1], p[:, 0] + p[:, 1]))) / floor)
    print(f"branch margins: |z|/|Q| >= {zmin:.4g}, floor margin >= {fmin:.4g}", flush=True)
    return zmin, fmin


def main():
    with Pool(6) as pool:
        margins = pool.apply_async(_branch_margins)
        rows = sorted(pool.map(_one, range(N_DIR)))
        zmin, fmin = margins.get()
    w = mg.disk_deformation()
    with open(PATH, "w") as f:
        f.write(f"# disk_deformation R=129 (m={w.m}), loss sum_i w_i f(P_i^K) after K={K} iterations from "
                f"W^0 = V, float64 oracle tangent\n")
        f.write(f"# directions: meshgen.unit_tangents(w, {N_DIR}, seed_c={DIR_SEED}) over (V, pinned targets)\n")
        f.write("# written by tests/golden/make_adjoint_k100_fixture.py (oracle only)\n")
        f.write(f"min_z_ratio {zmin:.17g}\n")
        f.write(f"min_floor_margin {fmin:.17g}\n")
        f.write("# j loss_lu dloss_lu loss_nd dloss_nd\n")
        for j, L1, d1, L2, d2 in rows:
            f.write(f"{j} {L1:.17g} {d1:.17g} {L2:.17g} {d2:.17g}\n")


def load(path=PATH):
    """(min_z_ratio, min_floor_margin, rows (N_DIR, 5): j, L_lu, dL_lu, L_nd, dL_nd)."""
    meta, rows = {}, []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0].startswith("min_"):
                meta[parts[0]] = float(parts[1])
            else:
                rows.append([float(v) for v in parts])
    return meta["min_z_ratio"], meta["min_floor_margin"], np.array(rows)


if __name__ == "__main__":
    main()
