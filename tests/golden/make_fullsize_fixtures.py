"""Write the oracle's fixtures for the two full-size free-running workloads.

Calls only the oracle (``oracle/``) and the seeded workload generator; no
value comes from the GPU library.  For each workload the oracle runs its
configured number of iterations from the workload's initial map and the file
records:
  * every history record (the twelve fields of the oracle's History),
  * the map at a seeded sample of vertices and W_el = U P and Lambda at a
    seeded sample of elements (caller's numbering), after the iterations
    listed in SAMPLE_ITERS,
  * the oracle's own timings on the machine that wrote the file (context).

Usage (from the repository root, about an hour for the tet cube on one core):
    python tests/golden/make_fullsize_fixtures.py twisted_cube_64 sphere_cap_uv_289
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2107_05200_amd import meshgen as mg  # noqa: E402

WORKLOADS = {
    # name: (generator, iterations, sampled iterations)
    "twisted_cube_64": (lambda: mg.twisted_cube(64), 300, (1, 10, 100, 300)),
    "sphere_cap_uv_289": (lambda: mg.sphere_cap_uv(), 500, (1, 10, 100, 500)),
}
N_SAMPLE = 128
SAMPLE_SEED = [210705200, 90]


def samples(w):
    rng = np.random.default_rng(SAMPLE_SEED)
    vs = np.sort(rng.choice(w.n, N_SAMPLE, replace=False))
    es = np.sort(rng.choice(w.m, N_SAMPLE, replace=False))
    return vs, es


def path_for(name):
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_{name}.txt")


def write(name):
    gen, iters, at = WORKLOADS[name]
    w = gen()
    vs, es = samples(w)
    t0 = time.perf_counter()
    r = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    r.init(w.x0)
    r.iterate(1)  # the first W-step factorises L_FF
    t1 = time.perf_counter()
    rows = {}
    t_loop = 0.0
    for k in range(1, iters + 1):
        if k > 1:
            ta = time.perf_counter()
            r.iterate(1)
            t_loop += time.perf_counter() - ta
        if k in at:
            rows[k] = (r.x[vs].copy(), (r.U @ r.P)[es].copy(), r.Lam[es].copy())
        if k % 10 == 0:
            print(f"{name}: iteration {k}, E_P {r.history.col('E_P')[-1]:.10g}", flush=True)
    H = r.history.array()
    with open(path_for(name), "w") as f:
        f.write(f"# oracle fixture: {w.name}, n={w.n}, m={w.m}, energy={w.energy}, rho={w.rho}, "
                f"{iters} iterations from the workload's initial map (float64 oracle)\n")
        f.write("# written by tests/golden/make_fullsize_fixtures.py (calls oracle/ only)\n")
        f.write(f"# oracle timings on the writing machine: first iteration with the factorisation "
                f"{t1 - t0:.1f} s, then {t_loop / max(iters - 1, 1):.3f} s per iteration (one thread)\n")
        f.write(f"# samples: {N_SAMPLE} vertices and {N_SAMPLE} elements drawn by default_rng({SAMPLE_SEED})\n")
        f.write("# hist k e_prim e_dual E_P E_map Phi flips nonfinite norm_GW norm_P norm_GtLam max_grad_f "
                "max_lambda_ratio\n")
        for k in range(H.shape[0]):
            f.write("hist %d %s\n" % (k + 1, " ".join("%.17g" % v for v in H[k])))
        f.write("# map k vertex coordinates / wel k element row-major UP / lam k element row-major Lambda\n")
        for k in sorted(rows):
            X, Wl, L = rows[k]
            for i, v in enumerate(vs):
                f.write("map %d %d %s\n" % (k, v, " ".join("%.17g" % t for t in X[i])))
            for i, e in enumerate(es):
                f.write("wel %d %d %s\n" % (k, e, " ".join("%.17g" % t for t in Wl[i].ravel())))
                f.write("lam %d %d %s\n" % (k, e, " ".join("%.17g" % t for t in L[i].ravel())))
    print(f"{name}: wrote {path_for(name)}", flush=True)


def read(name):
    """The fixture as arrays: hist (iters, 12), and per sampled iteration k
    dicts map[k] (N, d), wel[k] (N, d, d), lam[k] (N, d, d), with the sampled
    vertex and element indices."""
    hist, maps, wels, lams, vidx, eidx = [], {}, {}, {}, {}, {}
    for line in open(path_for(name)):
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        if t[0] == "hist":
            hist.append([float(v) for v in t[2:]])
            continue
        k, i = int(t[1]), int(t[2])
        vals = [float(v) for v in t[3:]]
        if t[0] == "map":
            maps.setdefault(k, []).append(vals)
            vidx.setdefault(k, []).append(i)
        elif t[0] == "wel":
            wels.setdefault(k, []).append(vals)
            eidx.setdefault(k, []).append(i)
        else:
            lams.setdefault(k, []).append(vals)
    d = len(next(iter(maps.values()))[0])
    out = {"hist": np.array(hist), "iters": sorted(maps)}
    out["map"] = {k: np.array(v) for k, v in maps.items()}
    out["wel"] = {k: np.array(v).reshape(-1, d, d) for k, v in wels.items()}
    out["lam"] = {k: np.array(v).reshape(-1, d, d) for k, v in lams.items()}
    out["vidx"] = np.array(vidx[out["iters"][0]])
    out["eidx"] = np.array(eidx[out["iters"][0]])
    return out


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(WORKLOADS):
        write(nm)
