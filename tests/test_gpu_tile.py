"""The tile-fused step (crkfr_set_fused) against the split step and the FP64
oracle: 2D Euler, N = 1 and 3, limiter chain off, on grids that fill the
tiles and on ragged grids with partial tiles, with every boundary kind, in
FP64 and FP32 bulk, eager steps and graph replay.

Tolerances: the two GPU paths evaluate the same expressions (the inner
faces' flux and the update read the same traces and fluxes, from LDS
instead of HBM): rel. L_inf <= 1e-13 in FP64 (contraction may differ in the
last bit), 1e-6 in FP32 bulk; against the oracle the split step's bounds
(FP64 rel. L_inf <= 1e-11, FP32 bulk rel. L1 <= 2e-6)."""
import numpy as np
import pytest

import oracle as O
from paper_2502_07517_amd import crkfr as C
from paper_2502_07517_amd import workloads as W
from gpu_cases import rel_l1, rel_linf
from oracle_runs import cfl_for

pytestmark = pytest.mark.gpu

DOM = (-5.0, 5.0, -5.0, 5.0)
BCS = {"periodic": (C.PERIODIC,) * 4, "outflow": (C.OUTFLOW,) * 4, "farfield": (C.FARFIELD,) * 4,
       "wall": (C.REFLECT,) * 4, "mixed": (C.PERIODIC, C.PERIODIC, C.REFLECT, C.FARFIELD)}


def _vortex(nx, ny, N):
    X, Y = W.node_coords_2d(nx, ny, N, DOM)
    return W.euler2d_cons(*W.vortex_prim(X, Y, 0.0, DOM))


def _pair(N, nx, ny, bc, dtype=C.FP64, scaling=0):
    out = []
    for path in (C.PATH_TILE, C.PATH_SPLIT):
        s = C.Solver(C.EULER2D, N, nx, ny, bc=bc, domain=DOM, dtype=dtype, cfl=cfl_for(N))
        if scaling:
            s.set_limiter(scaling=1)
        s.set_path(path)
        out.append(s)
    return out


@pytest.mark.parametrize("N", [1, 3])
@pytest.mark.parametrize("nx,ny", [(16, 8), (13, 11), (1, 1), (9, 5), (33, 17), (8, 4)])
def test_tile_equals_split_and_oracle_fp64(N, nx, ny):
    bc = BCS["periodic"]
    tile, split = _pair(N, nx, ny, bc)
    assert tile.path_in_use() == C.PATH_TILE and split.path_in_use() == C.PATH_SPLIT
    u0 = _vortex(nx, ny, N)
    ref = O.RefConfig.make(O.EULER2D, N, nx, ny, domain=DOM, cfl=cfl_for(N))
    dt = O.compute_dt(ref, u0)
    u = u0
    for s in (tile, split):
        s.set_state(u0)
    for _ in range(6):
        u, _, _, st = O.step(ref, u, dt)
        assert st == 0
        tile.step(dt)
        split.step(dt)
    ut, us = tile.get_state(), split.get_state()
    assert rel_linf(us, ut) <= 1e-13
    assert rel_linf(u.reshape(ut.shape), ut) <= 1e-11


@pytest.mark.parametrize("bc", list(BCS))
@pytest.mark.parametrize("N", [1, 3])
def test_tile_boundaries_equal_split(N, bc):
    nx, ny = 19, 10
    tile, split = _pair(N, nx, ny, BCS[bc])
    u0 = _vortex(nx, ny, N)
    for s in (tile, split):
        s.set_state(u0)
    for _ in range(5):
        tile.step(0.0)       # device time step: the rate reduction covers every element in both paths
        split.step(0.0)
    dt_, dsplit = tile.get_diag()[0], split.get_diag()[0]
    assert dt_["t"] == dsplit["t"]
    assert rel_linf(split.get_state(), tile.get_state()) <= 1e-13


@pytest.mark.parametrize("N", [1, 3])
def test_tile_fp32_bulk(N):
    nx, ny = 21, 12
    tile, split = _pair(N, nx, ny, BCS["periodic"], dtype=C.MP32)
    u0 = _vortex(nx, ny, N)
    ref = O.RefConfig.make(O.EULER2D, N, nx, ny, domain=DOM, cfl=cfl_for(N))
    dt = O.compute_dt(ref, u0)
    u = u0
    for s in (tile, split):
        s.set_state(u0)
    for _ in range(10):
        u, _, _, _ = O.step(ref, u, dt)
        tile.step(dt)
        split.step(dt)
    ut = tile.get_state()
    assert rel_l1(u.reshape(ut.shape), ut) <= 2e-6
    assert rel_linf(split.get_state(), ut) <= 1e-6
    # the FP64 means of both paths agree to the FP32 rounding of the face fluxes
    np.testing.assert_allclose(tile.get_means(), split.get_means(), rtol=1e-5, atol=1e-7)


def test_tile_scaling_limiter_and_counters():
    # 4-quadrant data, blending off, scaling on: the scaling acts in the inner
    # elements (tile kernel) and at tile edges (update phase) alike
    N, n = 3, 24
    tile, split = _pair(N, n, n, BCS["farfield"], scaling=1)
    u0 = W.euler2d_quadrants(11, n, N, dom=DOM)
    for s in (tile, split):
        s.set_state(u0)
    dt = split.compute_dt()
    for _ in range(4):
        tile.step(dt)
        split.step(dt)
    dtile, dsplit = tile.get_diag()[0], split.get_diag()[0]
    for k in ("n_scaled", "n_mean_inadmissible"):
        assert dtile[k] == dsplit[k], k
    # the split path's FP64 16-point elements take their derivatives on the
    # matrix cores, the tile kernel through DPP lanes: the sums round in a
    # different order
    assert dtile["min_theta_scale"] == pytest.approx(dsplit["min_theta_scale"], rel=1e-12)
    assert rel_linf(split.get_state(), tile.get_state()) <= 1e-13


def test_tile_graph_replay_equals_eager():
    N, n = 3, 24
    a, b = _pair(N, n, n, BCS["periodic"])
    b.set_path(C.PATH_TILE)
    u0 = _vortex(n, n, N)
    a.set_state(u0)
    b.set_state(u0)
    a.advance(0.0, 8)
    for _ in range(8):
        b.step(0.0)
    np.testing.assert_array_equal(a.get_state(), b.get_state())
    assert a.get_diag()[0]["steps"] == 8


def test_tile_path_selection():
    cases = [((C.EULER2D, 3, 8, 8), {}, True), ((C.EULER2D, 1, 8, 8), {}, True),
             ((C.EULER2D, 2, 8, 8), {}, False), ((C.EULER2D, 4, 8, 8), {}, False),
             ((C.TENMOM2D, 3, 8, 8), {}, False), ((C.EULER1D, 3, 8, 1), {}, False),
             ((C.EULER2D, 3, 8, 8), {"blend": C.BLEND_MH}, False)]
    for args, lim, want in cases:
        s = C.Solver(*args)
        # the default without the limiter chain: the checkerboard step on periodic 2D grids
        assert s.path_in_use() == (C.PATH_CHECKER if args[0] != C.EULER1D else C.PATH_FACE_UPDATE)
        s.set_path(C.PATH_TILE)
        if lim:
            s.set_limiter(**lim)
        assert s.path_in_use() == (C.PATH_TILE if want else C.PATH_FACE_UPDATE), args
    s = C.Solver(C.EULER2D, 3, 8, 8)
    s.set_path(C.PATH_TILE)
    s.set_scheme(dissipation=C.DISS_D1)
    assert s.path_in_use() == C.PATH_FACE_UPDATE
    s.set_scheme(dissipation=C.DISS_DCSX)
    assert s.path_in_use() == C.PATH_FACE_UPDATE
    s.set_scheme(dissipation=C.DISS_D2, central=C.CENTRAL_AE)
    assert s.path_in_use() == C.PATH_TILE
    with pytest.raises(C.CrkfrError):
        s.set_path(4)


def test_tile_extrapolated_central_part():
    # EA and AE central parts both go through the tile's inner faces
    N, n = 3, 20
    tile, split = _pair(N, n, n, BCS["periodic"])
    for s in (tile, split):
        s.set_scheme(central=C.CENTRAL_AE)
        s.set_state(_vortex(n, n, N))
    for _ in range(4):
        tile.step(0.0)
        split.step(0.0)
    assert rel_linf(split.get_state(), tile.get_state()) <= 1e-13
