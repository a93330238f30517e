"""The checkerboard step (CRKFR_PATH_CHECKER): colour-0 local procedure,
colour-1 local procedure with its face fluxes and update, colour-0 update
from the stored fluxes.  Against the face-update path (the same expressions
in the same order: rel. L_inf <= 1e-13 in FP64, 1e-6 in FP32 bulk) and the
FP64 oracle (rel. L_inf <= 1e-11), N = 1..4, on grids whose colour counts
fill the workgroups and on grids that leave them ragged, eager steps and
graph replay; configurations it does not serve fall back to the face-update
path."""
import numpy as np
import pytest

import oracle as O
from paper_2502_07517_amd import crkfr as C
from paper_2502_07517_amd import workloads as W
from gpu_cases import rel_linf
from oracle_runs import cfl_for

pytestmark = pytest.mark.gpu

DOM = (-5.0, 5.0, -5.0, 5.0)


def _vortex(nx, ny, N):
    X, Y = W.node_coords_2d(nx, ny, N, DOM)
    return W.euler2d_cons(*W.vortex_prim(X, Y, 0.0, DOM))


def _pair(N, nx, ny, dtype=C.FP64, central=None):
    out = []
    for path in (C.PATH_CHECKER, C.PATH_FACE_UPDATE):
        s = C.Solver(C.EULER2D, N, nx, ny, domain=DOM, dtype=dtype, cfl=cfl_for(N))
        if central is not None:
            s.set_scheme(central=central)
        s.set_path(path)
        out.append(s)
    return out


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("nx,ny", [(16, 8), (10, 6), (2, 2), (34, 18)])
def test_checker_equals_face_update_and_oracle_fp64(N, nx, ny):
    cb, fu = _pair(N, nx, ny)
    assert cb.path_in_use() == C.PATH_CHECKER
    u0 = _vortex(nx, ny, N)
    ref = O.RefConfig.make(O.EULER2D, N, nx, ny, domain=DOM, cfl=cfl_for(N))
    dt = O.compute_dt(ref, u0)
    u = u0
    for s in (cb, fu):
        s.set_state(u0)
    for _ in range(6):
        u, _, _, st = O.step(ref, u, dt)
        assert st == 0
        cb.step(dt)
        fu.step(dt)
    uc = cb.get_state()
    assert rel_linf(fu.get_state(), uc) <= 1e-13
    assert rel_linf(u.reshape(uc.shape), uc) <= 1e-11


@pytest.mark.parametrize("N", [2, 3])
def test_checker_device_time_step_and_counters(N):
    # device time steps: the colour-1 kernel and the colour-0 update both
    # feed the rate reduction, so the clocks agree
    cb, fu = _pair(N, 20, 12)
    for s in (cb, fu):
        s.set_state(_vortex(20, 12, N))
    for _ in range(5):
        cb.step(0.0)
        fu.step(0.0)
    dc, df = cb.get_diag()[0], fu.get_diag()[0]
    assert dc["t"] == pytest.approx(df["t"], rel=1e-14)
    assert dc["steps"] == df["steps"] == 5
    assert dc["mass"] == pytest.approx(df["mass"], rel=1e-14)
    assert rel_linf(fu.get_state(), cb.get_state()) <= 1e-13


@pytest.mark.parametrize("N", [1, 3, 4])
def test_checker_fp32_bulk(N):
    cb, fu = _pair(N, 18, 14, dtype=C.MP32)
    for s in (cb, fu):
        s.set_state(_vortex(18, 14, N))
    for _ in range(8):
        cb.step(0.0)
        fu.step(0.0)
    assert rel_linf(fu.get_state(), cb.get_state()) <= 1e-6
    np.testing.assert_allclose(cb.get_means(), fu.get_means(), rtol=1e-5, atol=1e-7)


def test_checker_extrapolated_central_part():
    cb, fu = _pair(3, 12, 12, central=C.CENTRAL_AE)
    for s in (cb, fu):
        s.set_state(_vortex(12, 12, 3))
    for _ in range(4):
        cb.step(0.0)
        fu.step(0.0)
    assert rel_linf(fu.get_state(), cb.get_state()) <= 1e-13


def test_checker_graph_replay_equals_eager():
    a, b = _pair(3, 16, 16)
    b.set_path(C.PATH_CHECKER)
    u0 = _vortex(16, 16, 3)
    a.set_state(u0)
    b.set_state(u0)
    a.advance(0.0, 8)
    for _ in range(8):
        b.step(0.0)
    np.testing.assert_array_equal(a.get_state(), b.get_state())


def test_checker_path_selection():
    def path(nx, ny, **kw):
        s = C.Solver(C.EULER2D, 3, nx, ny, **kw)
        s.set_path(C.PATH_CHECKER)
        return s
    assert path(8, 8).path_in_use() == C.PATH_CHECKER
    assert path(9, 8).path_in_use() == C.PATH_FACE_UPDATE            # odd side
    assert path(8, 7).path_in_use() == C.PATH_FACE_UPDATE
    assert path(8, 8, bc=(C.PERIODIC, C.PERIODIC, C.REFLECT, C.REFLECT)).path_in_use() == C.PATH_FACE_UPDATE
    s = path(8, 8)
    s.set_limiter(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
    assert s.path_in_use() == C.PATH_FACE_UPDATE
    s = path(8, 8)
    s.set_scheme(dissipation=C.DISS_D1)
    assert s.path_in_use() == C.PATH_FACE_UPDATE
    s = C.Solver(C.EULER1D, 3, 8)
    s.set_path(C.PATH_CHECKER)
    assert s.path_in_use() == C.PATH_FACE_UPDATE


def test_batch_of_checker_members():
    """Members whose own default is the checkerboard step run the face-update
    phases inside a batch; the batch matches them stepped alone to 1e-13."""
    N = 3
    sizes = [(16, 8), (12, 12), (20, 10)]
    seq, bat = [], []
    for nx, ny in sizes:
        for out in (seq, bat):
            s = C.Solver(C.EULER2D, N, nx, ny, domain=DOM, cfl=cfl_for(N))
            s.set_state(_vortex(nx, ny, N))
            out.append(s)
    assert all(s.path_in_use() == C.PATH_CHECKER for s in seq)
    for s in seq:
        for _ in range(4):
            s.step(0.0)
    b = C.Batch(bat)
    b.advance(4)
    b.sync()
    for s1, s2 in zip(seq, bat):
        assert rel_linf(s1.get_state(), s2.get_state()) <= 1e-13
        assert s1.get_diag()[0]["steps"] == s2.get_diag()[0]["steps"] == 4
