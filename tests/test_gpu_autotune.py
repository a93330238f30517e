"""crkfr_autotune: the kernel-path autotuner and its JSON-lines cache.  The
trials leave the solver as they found it (state, clock, counters bitwise);
the chosen path is one that serves the configuration and steps like that
path set by hand; a second solver of the same configuration takes the path
from the cache without timing; a configuration that differs in any keyed
field (grid, arithmetic, limiter) is timed anew and appended.  The update's
workgroup shape (16-point elements) is tuned with the path and changes no
bit of the results."""
import json

import numpy as np
import pytest

from paper_2502_07517_amd import crkfr as C
from paper_2502_07517_amd import workloads as W
from oracle_runs import cfl_for

pytestmark = pytest.mark.gpu

DOM = (-5.0, 5.0, -5.0, 5.0)
NAMES = ("split", "tile", "face_update", "checker")


def _solver(n, N=3, dtype=C.FP64, limited=False):
    s = C.Solver(C.EULER2D, N, n, n, domain=DOM, dtype=dtype, cfl=cfl_for(N))
    if limited:
        s.set_limiter(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
    s.set_state(W.vortex2d(n, N, 0.0, DOM))
    return s


def test_autotune_restores_state_and_picks_a_serving_path(tmp_path):
    cache = tmp_path / "tune.jsonl"
    s = _solver(24)
    s.step(0.0)
    u0, d0 = s.get_state(), s.get_diag()[0]
    r = s.autotune(steps=3, cache=cache)
    assert not r["from_cache"]
    # N = 3, periodic 24 x 24, limiter off: every path serves it
    assert set(r["ms_per_step"]) == {"split", "tile", "face_update", "checker"}
    assert r["path"] == s.path_in_use()
    assert min(r["ms_per_step"], key=r["ms_per_step"].get) == NAMES[r["path"]]
    np.testing.assert_array_equal(s.get_state(), u0)
    d1 = s.get_diag()[0]
    for k in ("steps", "t", "dt", "n_troubled", "mass"):
        assert d1[k] == d0[k], k
    # the tuned solver steps like one with that path set by hand
    ref = _solver(24)
    ref.step(0.0)
    ref.set_path(r["path"])
    for _ in range(3):
        s.step(0.0)
        ref.step(0.0)
    np.testing.assert_array_equal(s.get_state(), ref.get_state())
    assert r["update_shape"] == s.update_shape_in_use() in (C.UPDATE_BLOCK, C.UPDATE_WAVE)
    entries = [json.loads(line) for line in cache.read_text().splitlines()]
    assert len(entries) == 1 and "N=3" in entries[0]["key"] and "nx=24" in entries[0]["key"]
    assert entries[0]["path"] == NAMES[r["path"]]
    assert entries[0]["update_shape"] == ("block", "wave")[r["update_shape"]]


def test_autotune_cache_hit_and_keyed_misses(tmp_path):
    cache = tmp_path / "tune.jsonl"
    first = _solver(16).autotune(steps=2, cache=cache)
    again = _solver(16)
    r = again.autotune(steps=2, cache=cache)
    assert r["from_cache"] and r["path"] == first["path"] and r["ms_per_step"] == {}
    assert again.path_in_use() == first["path"]
    assert r["update_shape"] == first["update_shape"] == again.update_shape_in_use()
    # other grid, other arithmetic, limiter on: each timed and appended
    for s in (_solver(20), _solver(16, dtype=C.MP32), _solver(16, limited=True)):
        r = s.autotune(steps=2, cache=cache)
        assert not r["from_cache"]
    lines = cache.read_text().splitlines()
    assert len(lines) == 4
    keys = [json.loads(line)["key"] for line in lines]
    assert len(set(keys)) == 4
    # limiter on: the tile-fused and checkerboard paths do not serve it and are not timed
    timed = json.loads(lines[-1])["ms_per_step"]
    assert "tile" not in timed and "checker" not in timed


def test_autotune_errors(tmp_path):
    s = C.Solver(C.EULER2D, 2, 8, 8)
    with pytest.raises(C.CrkfrError):
        s.autotune(steps=2)                   # no state
    s.set_state(W.vortex2d(8, 2, 0.0, (0.0, 1.0, 0.0, 1.0)))
    with pytest.raises(C.CrkfrError):
        s.autotune(steps=0)
    with pytest.raises(C.CrkfrError):
        s.autotune(steps=1, cache=tmp_path / "no_such_dir" / "tune.jsonl")


def test_default_path_rule():
    """Without a chosen path: with the limiter chain off the checkerboard
    step where it serves (2D, periodic, even sides), else the face-update
    path; the split path with the limiter chain on; a path set by hand
    stays."""
    s = C.Solver(C.EULER2D, 3, 8, 8)
    assert s.path_in_use() == C.PATH_CHECKER
    s.set_limiter(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
    assert s.path_in_use() == C.PATH_SPLIT
    s.set_limiter(blend=C.BLEND_OFF, scaling=1)
    assert s.path_in_use() == C.PATH_CHECKER
    assert C.Solver(C.EULER2D, 3, 9, 8).path_in_use() == C.PATH_FACE_UPDATE
    assert C.Solver(C.EULER2D, 3, 8, 8, bc=(C.FARFIELD,) * 4).path_in_use() == C.PATH_FACE_UPDATE
    assert C.Solver(C.EULER1D, 3, 8).path_in_use() == C.PATH_FACE_UPDATE
    s.set_path(C.PATH_FACE_UPDATE)
    s.set_limiter(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
    assert s.path_in_use() == C.PATH_FACE_UPDATE


def test_update_shape_rule_and_errors():
    """One wavefront per workgroup for the FP64 checkerboard's colour-0
    update and the limited FP64 split update, 256 lanes elsewhere; 16-point
    elements only; a shape set by hand stays until -1 restores the rule."""
    s = C.Solver(C.EULER2D, 3, 8, 8)
    assert s.update_shape_in_use() == C.UPDATE_WAVE            # FP64 checkerboard
    assert C.Solver(C.EULER2D, 3, 8, 8, dtype=C.MP32).update_shape_in_use() == C.UPDATE_BLOCK
    s.set_limiter(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
    assert s.update_shape_in_use() == C.UPDATE_WAVE            # limited FP64, split
    s.set_path(C.PATH_FACE_UPDATE)
    assert s.update_shape_in_use() == C.UPDATE_BLOCK
    m = C.Solver(C.EULER2D, 3, 8, 8, dtype=C.MP32)
    m.set_limiter(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
    assert m.update_shape_in_use() == C.UPDATE_BLOCK           # limited FP32 bulk
    assert C.Solver(C.EULER2D, 3, 9, 8).update_shape_in_use() == C.UPDATE_BLOCK   # face-update
    two = C.Solver(C.EULER2D, 2, 8, 8)
    two.set_update_shape(C.UPDATE_WAVE)
    assert two.update_shape_in_use() == C.UPDATE_BLOCK         # 9-point elements keep their workgroups
    s.set_update_shape(C.UPDATE_WAVE)
    assert s.update_shape_in_use() == C.UPDATE_WAVE
    s.set_update_shape(-1)
    assert s.update_shape_in_use() == C.UPDATE_BLOCK
    for bad in (-2, 2):
        with pytest.raises(C.CrkfrError):
            s.set_update_shape(bad)


@pytest.mark.parametrize("dtype", [C.FP64, C.MP32])
@pytest.mark.parametrize("path,limited", [(C.PATH_SPLIT, False), (C.PATH_SPLIT, True),
                                          (C.PATH_FACE_UPDATE, False), (C.PATH_FACE_UPDATE, True),
                                          (C.PATH_CHECKER, False)])
def test_update_shapes_step_alike(dtype, path, limited):
    """Both workgroup shapes of the update give the same states and counters
    bit for bit (ragged block counts: 10 x 6 elements, 10 x 10 with the
    limiter chain on 4-quadrant data)."""
    runs = []
    ny = 10 if limited else 6
    for shape in (C.UPDATE_BLOCK, C.UPDATE_WAVE):
        s = C.Solver(C.EULER2D, 3, 10, ny, domain=DOM, dtype=dtype, cfl=cfl_for(3))
        if limited:
            s.set_limiter(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
        s.set_state(W.euler2d_quadrants(11, 10, 3, dom=DOM) if limited else _vortex_rect(10, ny))
        s.set_path(path)
        s.set_update_shape(shape)
        assert s.path_in_use() == path and s.update_shape_in_use() == shape
        for _ in range(4):
            s.step(0.0)
        runs.append((s.get_state(), s.get_diag()[0]))
    np.testing.assert_array_equal(runs[0][0], runs[1][0])
    for k in ("steps", "t", "dt", "n_troubled", "n_flux_limited", "n_scaled", "min_theta_scale"):
        assert runs[0][1][k] == runs[1][1][k], k


def _vortex_rect(nx, ny):
    X, Y = W.node_coords_2d(nx, ny, 3, DOM)
    return W.euler2d_cons(*W.vortex_prim(X, Y, 0.0, DOM))
