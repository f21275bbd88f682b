"""Free-running parity at the full sizes of the benchmark workloads against
the oracle's fixtures (tests/golden/oracle_*.txt, written by
tests/golden/make_fullsize_fixtures.py from the oracle alone): the twisted tet
cube (1,572,864 tets, 300 iterations) and the sphere cap (501,126 triangles,
500 iterations), with float64 and float32 element steps, in the launch
configuration the benchmark times (autotuned, replayed graphs).

Compared at the fixture's sampled iterations: the map at 128 sampled vertices
and W_el = U P and Lambda at 128 sampled elements (relative Frobenius error
over the samples, and the largest per-row relative error), and the history
curves (e_prim, e_dual, E_P) at every iteration.  Gates (the per-iteration
relative bar of 1e-5 on W_el and the map, 1e-4 on the final energy):
  float64: map and W_el <= 1e-5 at every sampled iteration, final E_P <= 1e-4;
  float32: the same (the float32 element steps stay within 1e-5 of the
  float64 oracle over the whole run); the scaled dual Lambda over the
  sampled elements within 1e-5 (float64) and 1e-4 (float32, measured 4e-6);
  all errors printed.  e_prim of a
  float32 run stops decreasing at the float32 rounding level of |J - U P|,
  so its curve is printed, not gated."""
import os
import sys

import numpy as np
import pytest

from paper_2107_05200_amd import meshgen as mg

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import make_fullsize_fixtures as fixtures  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def row_max(a, b):
    a = np.asarray(a, np.float64).reshape(len(b), -1)
    b = np.asarray(b, np.float64).reshape(len(b), -1)
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)))


CASES = [("sphere_cap_uv_289", 64), ("sphere_cap_uv_289", 32), ("twisted_cube_64", 64), ("twisted_cube_64", 32)]
# float32 element steps free-running over hundreds of iterations still meet
# the per-iteration bar on the map and W_el (measured: sphere cap <= 5e-7)
FP32_BOUND = {"sphere_cap_uv_289": 1e-5, "twisted_cube_64": 1e-5}


@pytest.mark.parametrize("name,prec", CASES)
def test_free_running_against_oracle_fixture(gpu_lib, name, prec):
    import torch
    from paper_2107_05200_amd.binding import Solver
    if not os.path.exists(fixtures.path_for(name)):
        pytest.skip(f"fixture {name} not written")
    fx = fixtures.read(name)
    gen, iters, at = fixtures.WORKLOADS[name]
    w = gen()
    vs, es = fixtures.samples(w)
    assert np.array_equal(vs, fx["vidx"]) and np.array_equal(es, fx["eidx"])
    say(f"case: {name} float{prec}, {iters} iterations against the oracle fixture")
    g = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=prec)
    g.init(w.x0).autotune()
    g.init(w.x0)
    done = 0
    worst = {"map": 0.0, "wel": 0.0, "lam": 0.0}
    for k in fx["iters"]:
        g.iterate(k - done, graph=True)
        done = k
        st = g.get_state()
        torch.cuda.synchronize()
        x = st["map"].cpu().numpy()[vs]
        wel = st["Wel"].cpu().numpy()[es]
        lam = st["Lam"].cpu().numpy()[es]
        e = {"map": rel(x, fx["map"][k]), "wel": rel(wel, fx["wel"][k]), "lam": rel(lam, fx["lam"][k])}
        m = {"map": row_max(x, fx["map"][k]), "wel": row_max(wel, fx["wel"][k]), "lam": row_max(lam, fx["lam"][k])}
        say(f"  k={k}: rel map {e['map']:.2e} W_el {e['wel']:.2e} Lambda {e['lam']:.2e}; "
            f"largest per row: map {m['map']:.2e} W_el {m['wel']:.2e} Lambda {m['lam']:.2e}")
        worst["map"] = max(worst["map"], e["map"])
        worst["wel"] = max(worst["wel"], e["wel"])
        worst["lam"] = max(worst["lam"], e["lam"])
    h = g.history()
    H = fx["hist"]
    assert h.shape[0] == H.shape[0] == iters
    eP = np.abs(h[:, 2] - H[:, 2]) / np.abs(H[:, 2])
    ep = np.abs(h[:, 0] - H[:, 0]) / H[:, 0]
    ed = np.abs(h[:, 1] - H[:, 1]) / H[:, 1]
    say(f"  E_P rel err: final {eP[-1]:.2e}, largest {eP.max():.2e}; e_prim rel err largest {ep.max():.2e} "
        f"(final {ep[-1]:.2e}); e_dual rel err largest {ed.max():.2e} (final {ed[-1]:.2e})")
    say(f"  final E_P device {h[-1, 2]:.12g} oracle {H[-1, 2]:.12g}; flips device {int(h[-1, 5])} oracle {int(H[-1, 5])}")
    g.close()
    assert eP[-1] <= 1e-4
    assert h[-1, 5] == H[-1, 5]
    bound = 1e-5 if prec == 64 else FP32_BOUND[name]
    # Lambda adds the float32 rounding of J - U P every iteration while its own
    # norm is small against |J|: 1e-4 in float32, 1e-5 in float64
    assert worst["map"] <= bound and worst["wel"] <= bound, worst
    assert worst["lam"] <= (1e-5 if prec == 64 else 1e-4), worst
