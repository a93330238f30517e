"""GPU parity of the solid-wall boundaries (Sec. 3.3, eq. reflect.time.avg)
and the admissibility stress tests of Sec. 5.2-5.3 (blast wave and Sedov
blasts) against the oracle.

With walls only there are no far-field ghosts, so the GPU state can be reset
to the oracle's state before each compared step: one step from the same
input is compared to rounding, which keeps the comparison tight on runs
whose limiter decisions would otherwise amplify rounding differences."""
import numpy as np
import pytest

import oracle as O
from gpu_cases import rel_l1
from oracle_runs import cfl_for
from paper_2502_07517_amd import crkfr as C
from paper_2502_07517_amd import workloads as W

pytestmark = pytest.mark.gpu
WALLS = (C.REFLECT,) * 4
LIM = dict(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
COUNTERS = ("n_troubled", "n_flux_limited", "n_lo_inadmissible", "n_slope_limited", "n_hancock_fallback",
            "n_scaled", "n_mean_inadmissible")


def _pair(eq, N, nx, ny=1, bc=WALLS, domain=(0, 1, 0, 1), dtype=C.FP64, source=None):
    ref = O.RefConfig.make(eq, N, nx, ny, bc=bc, domain=domain, cfl=cfl_for(N), source=1 if source else 0,
                           src=source[:4] if source else (0, 0, 0, 0), src_lin=source[4:] if source else (0, 0),
                           **LIM)
    gpu = C.Solver(eq, N, nx, ny, bc=bc, domain=domain, dtype=dtype, cfl=cfl_for(N))
    gpu.set_limiter(**LIM)
    if source:
        gpu.set_source(1, *source)
    return ref, gpu


def _single_steps(ref, gpu, u0, steps, every=1, tol=1e-12):
    """Oracle trajectory with the time step of eq. time.step.2d; every
    `every` steps the GPU takes the same step from the oracle's state."""
    u = np.ascontiguousarray(u0, dtype=np.float64)
    worst, acted = 0.0, 0
    for k in range(steps):
        dt = O.compute_dt(ref, u)
        un, _, do, st = O.step(ref, u, dt)
        assert st == 0
        if k % every == 0:
            gpu.set_state(u.copy())
            gpu.step(dt)
            ug = gpu.get_state().reshape(un.shape)
            dg, _ = gpu.get_diag()
            e = rel_l1(un, ug)
            worst = max(worst, e)
            assert e <= tol, (k, e)
            for key in COUNTERS:
                assert do[key] == dg[key], (k, key, do[key], dg[key])
            acted += do["n_flux_limited"] + do["n_scaled"]
        u = un
    return u, worst, acted


@pytest.mark.parametrize("N", [2, 3])
def test_blast_wave_walls_single_steps_fp64(N):
    ref, gpu = _pair(C.EULER1D, N, 100)
    u, worst, acted = _single_steps(ref, gpu, W.blast1d(100, N), 300, every=7)
    print(f"blast wave N={N}: worst single-step rel. L1 {worst:.2e}, limiter actions {acted}")
    assert acted > 0       # the flux limiter or the scaling limiter acted on compared steps


def test_blast_wave_walls_run_fp64_and_mp32():
    """Full runs to t = 0.038 with device time steps: admissible throughout;
    FP64 against the oracle's run, FP32 bulk against it within the
    limited-path bound."""
    N, nx, t_end = 3, 100, 0.038
    ref, _ = _pair(C.EULER1D, N, nx)
    u = W.blast1d(nx, N)
    t = 0.0
    while t < t_end - 1e-15:
        dt = min(O.compute_dt(ref, u), t_end - t)
        u, _, d, st = O.step(ref, u, dt)
        assert st == 0
        t += dt
    for dtype, tol in ((C.FP64, 1e-6), (C.MP32, 1e-2)):
        _, gpu = _pair(C.EULER1D, N, nx, dtype=dtype)
        gpu.set_state(W.blast1d(nx, N))
        gpu.advance(t_end, 100000)
        d, rc = gpu.get_diag()
        assert rc == 0 and abs(d["t"] - t_end) < 1e-12
        ug = gpu.get_state().reshape(u.shape)
        p = 0.4 * (ug[2] - 0.5 * ug[1] ** 2 / ug[0])
        assert ug[0].min() > 0 and p.min() > 0
        print(f"blast wave t = 0.038, dtype {dtype}: rel. L1 vs oracle {rel_l1(u, ug):.2e}")
        assert rel_l1(u, ug) <= tol, (dtype, rel_l1(u, ug))


def test_sedov1d_walls_single_steps_and_run_fp64():
    N, nx = 3, 201
    dom = (-1.0, 1.0, 0.0, 1.0)
    ref, gpu = _pair(C.EULER1D, N, nx, domain=dom)
    u, worst, acted = _single_steps(ref, gpu, W.sedov1d(nx, N), 600, every=29, tol=1e-11)
    assert acted > 0
    _, g2 = _pair(C.EULER1D, N, nx, domain=dom)
    g2.set_state(W.sedov1d(nx, N))
    g2.advance(0.001, 100000)
    d, rc = g2.get_diag()
    assert rc == 0 and abs(d["t"] - 0.001) < 1e-15
    ug = g2.get_state()
    p = 0.4 * (ug[2] - 0.5 * ug[1] ** 2 / ug[0])
    assert ug[0].min() > 0 and p.min() > 0
    m = ug[:, ::-1, ::-1].copy()
    m[1] *= -1.0
    assert np.max(np.abs(m - ug)) < 1e-9 * np.max(np.abs(ug))   # mirror symmetric about x = 0


@pytest.mark.parametrize("N", [2, 3, 4])
def test_euler2d_box_walls_fp64(N):
    n = 10
    ref, gpu = _pair(C.EULER2D, N, n, n + 2)
    X, Y = W.node_coords_2d(n, n + 2, N, (0, 1, 0, 1))
    st = W.quadrant_states_euler(9)
    rho, v1, v2, p = W._quadrant_fill(X, Y, 0.5 + 0.37 / n, 0.5 + 0.37 / (n + 2), st)
    _single_steps(ref, gpu, W.euler2d_cons(rho, v1, v2, p), 12, every=3)


def test_euler2d_walls_mixed_with_periodic_and_farfield_fp64():
    """Walls in x, far-field in y: multi-step parity from one input."""
    N, n = 3, 9
    bc = (C.REFLECT, C.REFLECT, C.FARFIELD, C.FARFIELD)
    ref, gpu = _pair(C.EULER2D, N, n, n, bc=bc)
    u0 = W.euler2d_quadrants(4, n, N)
    ghost = O.boundary_traces(ref, u0)
    gpu.set_state(u0.copy())
    u = u0.copy()
    for _ in range(8):
        dt = O.compute_dt(ref, u)
        u, _, _, st = O.step(ref, u, dt, ghost=ghost)
        gpu.step(dt)
    assert rel_l1(u, gpu.get_state().reshape(u.shape)) <= 1e-9


@pytest.mark.parametrize("N", [2, 4])
def test_tenmom_walls_source_fp64(N):
    nx, ny = 16, 6
    dom = (-2.0, 2.0, -0.5, 0.5)
    src = (25.0, 200.0, 1.0, 0.0, 0.0, 0.0)
    ref, gpu = _pair(C.TENMOM2D, N, nx, ny, domain=dom, source=src)
    _single_steps(ref, gpu, W.tenmom2d_quadrants(1, nx, ny, N, dom), 8, every=2)


def test_sedov2d_periodic_fp64():
    """2D Sedov test of Sec. 5.3 (p0 = 1e-5): single steps against the oracle
    and a GPU run that stays admissible."""
    N, n = 3, 16
    dom = (-1.5, 1.5, -1.5, 1.5)
    ref, gpu = _pair(C.EULER2D, N, n, n, bc=(C.PERIODIC,) * 4, domain=dom)
    _single_steps(ref, gpu, W.sedov2d(n, N, dom), 40, every=8, tol=1e-11)
    _, g2 = _pair(C.EULER2D, N, 32, 32, bc=(C.PERIODIC,) * 4, domain=dom)
    g2.set_state(W.sedov2d(32, N, dom))
    g2.advance(0.5, 100000)
    d, rc = g2.get_diag()
    assert rc == 0 and d["n_mean_inadmissible"] == 0
    ug = g2.get_state()
    p = 0.4 * (ug[3] - 0.5 * (ug[1] ** 2 + ug[2] ** 2) / ug[0])
    assert ug[0].min() > 0 and p.min() > 0


def test_walls_rejected_for_linear_advection():
    with pytest.raises(C.CrkfrError):
        C.Solver(C.LINADV1D, 3, 10, bc=WALLS)
