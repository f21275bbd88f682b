"""CPU tests of the C ABI library: it loads, exports every declared symbol,
and its host set-up (geometry, ordering, factorisation) is correct and reports
the documented errors.  No device calls."""
import os
import re

import numpy as np
import pytest

from paper_2107_05200_amd import binding, meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "ffd.h")).read()
    return sorted(set(re.findall(r"^\s*(?:ffd_status|void|const char\*)\s+(ffd_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    syms = _declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    # and the binding declares prototypes for all of them
    assert set(syms) <= set(binding._PROTOS)


@pytest.mark.parametrize("wk", [
    lambda: mg.height_field_uv(),
    lambda: mg.twisted_cube(10),
    lambda: mg.sphere_cap_uv(R=25),
    lambda: mg.disk_deformation(R=18),
    lambda: mg.flat_grid(5),
], ids=["height_field", "cube10", "sphere_cap", "disk", "flat"])
def test_factor_selfcheck(wk):
    w = wk()
    info = binding.analyze(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    assert info["selfcheck_residual"] < 1e-12
    assert info["n_free"] + info["n_pinned"] == w.n
    assert info["factor_nnz"] > 0 and info["n_levels"] >= 1


def test_factor_selfcheck_leaf_sizes_and_auto_pin():
    w = mg.sphere_cap_uv(R=12)
    for leaf in (1, 4, 16, 1000):
        info = binding.analyze(w.V, w.T, w.energy, w.rho, None, None, auto_pin=1, leaf_size=leaf)
        assert info["selfcheck_residual"] < 1e-12
        assert info["n_pinned"] == 1


def test_error_codes():
    w = mg.height_field_uv(grid=6)
    # no pins and no auto pin: singular
    with pytest.raises(binding.FFDError) as e:
        binding.analyze(w.V, w.T, w.energy, w.rho, None, None, auto_pin=0)
    assert e.value.status == -3
    # degenerate element (repeated vertex coordinates)
    V = w.V.copy()
    V[w.T[3, 1]] = V[w.T[3, 0]]
    with pytest.raises(binding.FFDError) as e:
        binding.analyze(V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    assert e.value.status == -2
    # index out of range
    T = w.T.copy()
    T[0, 0] = w.n
    with pytest.raises(binding.FFDError) as e:
        binding.analyze(w.V, T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    assert e.value.status == -1
    # non-finite source vertex
    V = w.V.copy()
    V[5, 0] = np.nan
    with pytest.raises(binding.FFDError) as e:
        binding.analyze(V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    assert e.value.status == -4
    # a second component without a pin
    T2 = np.concatenate([w.T, w.T + w.n])
    V2 = np.concatenate([w.V, w.V + 5.0])
    with pytest.raises(binding.FFDError) as e:
        binding.analyze(V2, T2, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    assert e.value.status == -3
    # repeated pin
    with pytest.raises(binding.FFDError) as e:
        binding.analyze(w.V, w.T, w.energy, w.rho, np.array([0, 0]), None)
    assert e.value.status == -1
    # option values and pinned positions are checked as ffd_create checks them
    with pytest.raises(binding.FFDError) as e:
        binding.analyze(w.V, w.T, 7, w.rho, w.pinned_idx, w.pinned_pos)
    assert e.value.status == -1
    with pytest.raises(binding.FFDError) as e:
        binding.analyze(w.V, w.T, w.energy, w.rho, w.pinned_idx, np.full_like(w.pinned_pos, np.inf))
    assert e.value.status == -4
    for bad in (0.0, -1.0, float("nan")):
        with pytest.raises(binding.FFDError) as e:
            binding.analyze(w.V, w.T, w.energy, bad, w.pinned_idx, w.pinned_pos)
        assert e.value.status == -1
    # empty mesh; a simplex dimension or input dimension the solver has no form for
    with pytest.raises(binding.FFDError) as e:
        binding.analyze(w.V, w.T[:0], w.energy, w.rho, w.pinned_idx, w.pinned_pos)
    assert e.value.status == -1
    T4 = np.concatenate([w.T, w.T[:, :2]], axis=1)  # 5 vertices per element
    with pytest.raises(binding.FFDError) as e:
        binding.analyze(np.concatenate([w.V, w.V[:, :2]], axis=1), T4, w.energy, w.rho, w.pinned_idx, None)
    assert e.value.status == -1
    with pytest.raises(binding.FFDError) as e:  # triangles with 4-D source vertices
        binding.analyze(np.concatenate([w.V, w.V[:, :1]], axis=1), w.T, w.energy, w.rho, w.pinned_idx, None)
    assert e.value.status == -1


def test_factor_matches_oracle_matrix_on_two_components():
    # two disjoint charts, each pinned: the forest case of the ordering
    w = mg.height_field_uv(grid=9)
    T2 = np.concatenate([w.T, w.T + w.n])
    V2 = np.concatenate([w.V, w.V + 5.0])
    pins = np.concatenate([w.pinned_idx, w.pinned_idx + w.n])
    info = binding.analyze(V2, T2, w.energy, w.rho, pins, None)
    assert info["selfcheck_residual"] < 1e-12
