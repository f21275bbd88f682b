"""ffd_iterate_noalloc (the allocation-free variant of ffd_iterate, whose
local-step partial sums live in the library's fixed device scratch) against
ffd_iterate, through the C ABI: bitwise the same state and history, on two
calls in a row (a float32 tet cube, then a smaller float64 chart, so the
second call finds the scratch holding the first call's larger contents), and
its refusal when the history would have to grow."""
import sys

import numpy as np
import pytest

from paper_2107_05200_amd import meshgen as mg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(w, prec):
    from paper_2107_05200_amd.binding import Solver
    a = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=prec)
    b = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=prec)
    return a, b


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_matches_iterate(gpu_lib, order):
    import torch
    for w, prec, n in ((mg.twisted_cube(12), 32, 9), (mg.height_field_uv(), 64, 7)):
        say(f"case: ffd_iterate_noalloc vs ffd_iterate on {w.name} (m={w.m}) fp{prec}, {n} iterations")
        a, b = _pair(w, prec)
        a.init(w.x0).iterate(n)
        b.init(w.x0).iterate_noalloc(n)
        sa, sb = a.get_state(), b.get_state()
        torch.cuda.synchronize()
        for k in ("map", "U", "P", "Lam", "Wel"):
            assert torch.equal(sa[k], sb[k]), k
        ha, hb = a.history(), b.history()
        assert np.array_equal(np.isnan(ha), np.isnan(hb))
        assert np.array_equal(np.nan_to_num(ha), np.nan_to_num(hb))
        say(f"  bitwise equal: state and {ha.shape[0]} history records")
        a.close()
        b.close()


def test_noalloc_refuses_to_grow_the_history(gpu_lib):
    from paper_2107_05200_amd.binding import FFDError, Solver
    w = mg.height_field_uv(grid=8)
    s = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=64)
    s.init(w.x0)
    with pytest.raises(FFDError) as e:
        s.iterate_noalloc(1 << 20)
    assert "history" in str(e.value)
    assert s.iteration() == 0
    s.iterate_noalloc(3)
    assert s.iteration() == 3
    s.close()


def test_noalloc_refuses_a_mesh_beyond_the_scratch(gpu_lib):
    """A local step whose partial sums exceed the fixed scratch (4 MiB:
    (ceil(m / block) + blocks / 256) x 11 float64, so about 12M elements at
    the default block of 256) is refused before anything runs; the handle
    still iterates with ffd_iterate."""
    from paper_2107_05200_amd.binding import FFDError, Solver
    w = mg.flat_grid(grid=2500)  # 12,490,002 triangles
    say(f"case: ffd_iterate_noalloc refusal on {w.name} (m={w.m})")
    s = Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32)
    s.init(w.x0)
    with pytest.raises(FFDError) as e:
        s.iterate_noalloc(1)
    assert "scratch" in str(e.value)
    assert s.iteration() == 0
    s.iterate(1)
    assert s.iteration() == 1
    s.close()
