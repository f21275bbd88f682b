"""The measurement entry points (ffd_iterate_profiled, ffd_profile_solve_levels)
report what they claim and leave the iteration's results as they were:
state and history bitwise equal to a plain run on an identical handle."""
import sys

import numpy as np
import pytest

from paper_2107_05200_amd import meshgen as mg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(w):
    from paper_2107_05200_amd.binding import Solver
    return Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32)


def _same(a, b):
    import torch
    sa, sb = a.get_state(), b.get_state()
    torch.cuda.synchronize()
    for k in sa:
        assert torch.equal(sa[k], sb[k]), k
    ha, hb = a.history(), b.history()
    assert ha.shape == hb.shape
    assert np.array_equal(ha, hb, equal_nan=True)


def test_profiled_iterations_equal_plain_ones(gpu_lib):
    w = mg.twisted_cube(6)
    say("case: iterate_profiled against iterate, cube k=6")
    a = _solver(w)
    a.init(w.x0).iterate(7)
    b = _solver(w)
    b.init(w.x0)
    ph = b.iterate_profiled(7)
    say(f"  phases (ms summed over 7 iterations): {ph}")
    assert b.iteration() == 7
    assert all(ph[k] > 0.0 for k in ("wrhs", "solve_fwd", "solve_bwd", "local", "total"))
    assert ph["total"] >= ph["solve_fwd"] + ph["solve_bwd"] + ph["local"]
    _same(a, b)


def test_level_profile_covers_the_factor_and_leaves_the_iteration(gpu_lib):
    w = mg.twisted_cube(8)
    say("case: profile_solve_levels, cube k=8")
    a = _solver(w)
    a.init(w.x0).iterate(3)
    lv = a.profile_solve_levels(3)
    info = a.info()
    say(f"  {len(lv)} levels; nodes per level {[int(l['nodes']) for l in lv]}")
    assert len(lv) >= 2
    assert all(l["fwd_ms"] > 0.0 and l["bwd_ms"] > 0.0 and l["nodes"] >= 1 for l in lv)
    total = sum(l["bytes"] for l in lv)
    assert abs(total - 8.0 * info["factor_nnz"]) <= 1e-9 * total
    a.iterate(3)
    b = _solver(w)
    b.init(w.x0).iterate(6)
    _same(a, b)


def test_level_profile_argument_errors(gpu_lib):
    import ctypes as C
    from paper_2107_05200_amd.binding import FFDError, _check
    w = mg.twisted_cube(8)
    a = _solver(w)
    a.init(w.x0)
    with pytest.raises(FFDError):
        a.profile_solve_levels(0)
    out = (C.c_double * 10)()
    nl = C.c_int32(0)
    with pytest.raises(FFDError):  # room for one level only
        _check(a.lib.ffd_profile_solve_levels(a.h, 1, None, out, 1, C.byref(nl)))
    assert nl.value >= 2
