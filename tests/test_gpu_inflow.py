"""GPU parity of the time-dependent inflow boundaries (Sec. 3.3) against the
oracle: interface ghost values from the time averages of the boundary data,
F = F^- on fully inflow faces, the D2 flux elsewhere, the data at the half
time for the low-order flux."""
import math

import numpy as np
import pytest

import oracle as O
from gpu_cases import rel_l1, rel_linf
from oracle_runs import cfl_for
from paper_2502_07517_amd import crkfr as C
from paper_2502_07517_amd import workloads as W

pytestmark = pytest.mark.gpu
LIM = dict(blend=C.BLEND_MH, flux_limiter=1, scaling=1)


def _ghost_size(eq, N, nx, ny):
    M, nd = C.NVAR[eq], N + 1
    two_d = eq in (C.EULER2D, C.TENMOM2D)
    nq = nd if two_d else 1
    return 2 * ny * nq * M + (2 * nx * nd * M if two_d else 0)


def _pair(eq, N, nx, ny=1, *, bc, lim=None, domain=(0.0, 1.0, 0.0, 1.0), dtype=C.FP64, cfl=None,
          diss=C.DISS_D2):
    lim = lim or {}
    cfl = cfl or cfl_for(N, system=eq != C.LINADV1D)
    ref = O.RefConfig.make(eq, N, nx, ny, bc=bc, domain=domain, cfl=cfl, dissipation=diss, **lim)
    gpu = C.Solver(eq, N, nx, ny, bc=bc, domain=domain, dtype=dtype, cfl=cfl)
    gpu.set_scheme(0, diss, C.CENTRAL_EA)
    if lim:
        gpu.set_limiter(**lim)
    return ref, gpu


def _taylor(fn_derivs, t0, ncoef=5):
    return [fn_derivs(j, t0) / math.factorial(j) for j in range(ncoef)]


def _run_pair(ref, gpu, u0, steps, coef_at, dt):
    """Both advance with fixed dt, the inflow data re-anchored at t^n."""
    u = np.ascontiguousarray(u0, dtype=np.float64)
    gpu.set_state(u.copy())
    t, do = 0.0, None
    for _ in range(steps):
        coef = coef_at(t)
        ref.set_inflow(coef, t)
        gpu.set_inflow(coef, t)
        u, _, do, st = O.step(ref, u, dt, t=t)
        assert st == 0
        gpu.step(dt)
        t += dt
    return u, gpu.get_state().reshape(u.shape), do, gpu.get_diag()[0]


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_linadv_inflow_fp64(N):
    nx = 13
    ref, gpu = _pair(C.LINADV1D, N, nx, bc=(C.INFLOW, C.OUTFLOW, 0, 0))
    gs = _ghost_size(C.LINADV1D, N, nx, 1)

    def coef_at(t):
        cf = np.zeros((5, gs))
        cf[:, 0] = _taylor(lambda j, s: (-2 * np.pi) ** j * math.sin(-2 * np.pi * s + j * math.pi / 2), t)
        return cf
    x = W.node_coords_1d(nx, N, 0.0, 1.0)
    uo, ug, _, _ = _run_pair(ref, gpu, np.sin(2 * np.pi * x)[None], 25, coef_at, 0.4 * cfl_for(N, system=False) / nx)
    assert rel_linf(uo, ug) <= 1e-12


def _euler_inflow_coef(gs, N, nx, t, supersonic, right_too=True):
    """Time-varying inflow state at the left (and right) boundary of a 1D Euler run."""
    cf = np.zeros((5, gs))
    for side in range(2 if right_too else 1):
        v = (2.5 if supersonic else 0.3) * (1 if side == 0 else -1)
        # rho(t) = 1 + 0.2 sin(3 t + side), v and p constant: Taylor coefficients at t
        rho = _taylor(lambda j, s: 0.2 * 3.0 ** j * math.sin(3 * s + side + j * math.pi / 2), t)
        rho[0] += 1.0
        p = 1.0
        for j in range(5):
            cf[j, side * 3 + 0] = rho[j]
            cf[j, side * 3 + 1] = rho[j] * v
            cf[j, side * 3 + 2] = (p / 0.4 if j == 0 else 0.0) + 0.5 * rho[j] * v * v
    return cf


@pytest.mark.parametrize("supersonic", [False, True])
@pytest.mark.parametrize("N", [2, 3])
def test_euler1d_inflow_limited_fp64(N, supersonic):
    nx = 31
    ref, gpu = _pair(C.EULER1D, N, nx, bc=(C.INFLOW, C.INFLOW, 0, 0), lim=LIM)
    gs = _ghost_size(C.EULER1D, N, nx, 1)
    u0 = W.euler1d_riemann(4, nx, N)
    dt = 0.5 * O.compute_dt(ref, u0)
    uo, ug, do, dg = _run_pair(ref, gpu, u0, 20, lambda t: _euler_inflow_coef(gs, N, nx, t, supersonic), dt)
    assert rel_l1(uo, ug) <= 1e-9, rel_l1(uo, ug)
    assert do["n_troubled"] == dg["n_troubled"]


@pytest.mark.parametrize("diss", [C.DISS_D2, C.DISS_D1, C.DISS_DCSX])
def test_euler2d_inflow_left_outflow_right_fp64(diss):
    N, nx, ny = 3, 9, 7
    dom = (-5.0, 5.0, -5.0, 5.0)
    bc = (C.INFLOW, C.OUTFLOW, C.PERIODIC, C.PERIODIC)
    cfl = 0.5 * cfl_for(N)
    ref, gpu = _pair(C.EULER2D, N, nx, ny, bc=bc, domain=dom, cfl=cfl, diss=diss)
    gs = _ghost_size(C.EULER2D, N, nx, ny)
    X, Y = W.node_coords_2d(nx, ny, N, dom)
    u0 = W.euler2d_cons(*W.vortex_prim(X, Y, 0.0, dom))
    yq = W.node_coords_2d(1, ny, N, dom)[1][:, 0, :, 0]        # [ey][q] y of the left face points

    def coef_at(t):
        cf = np.zeros((5, gs))
        left = cf[:, : ny * (N + 1) * 4].reshape(5, ny, N + 1, 4)
        for j in range(5):
            amp = _taylor(lambda k, s: 0.1 * (2.0 ** k) * math.cos(2 * s + k * math.pi / 2), t)[j]
            rho = (1.0 if j == 0 else 0.0) + amp * np.sin(2 * np.pi * yq / 10)
            left[j, :, :, 0] = rho
            left[j, :, :, 1] = rho * 0.7
            left[j, :, :, 2] = 0.0
            left[j, :, :, 3] = (1.0 / 0.4 if j == 0 else 0.0) + 0.5 * rho * 0.49
        return cf
    uo, ug, _, _ = _run_pair(ref, gpu, u0, 10, coef_at, O.compute_dt(ref, u0))
    assert rel_linf(uo, ug) <= 1e-11, rel_linf(uo, ug)


def test_constant_inflow_equals_farfield_on_gpu():
    N, nx = 3, 31
    u0 = W.euler1d_riemann(2, nx, N)
    cf = O.RefConfig.make(O.EULER1D, N, nx, bc=(O.FARFIELD,) * 4, cfl=cfl_for(N))
    ghost = O.boundary_traces(cf, u0)
    a = C.Solver(C.EULER1D, N, nx, bc=(C.FARFIELD,) * 4, cfl=cfl_for(N))
    b = C.Solver(C.EULER1D, N, nx, bc=(C.INFLOW,) * 4, cfl=cfl_for(N))
    for s in (a, b):
        s.set_limiter(**LIM)
        s.set_state(u0.copy())
    b.set_inflow(ghost[None, :], 0.0)
    for _ in range(15):
        a.step(0.0)
        b.step(0.0)
    ua, ub = a.get_state(), b.get_state()
    assert np.max(np.abs(ua - ub)) <= 1e-13 * np.max(np.abs(ua))


def test_inflow_errors():
    s = C.Solver(C.EULER1D, 3, 8, bc=(C.FARFIELD,) * 4)
    with pytest.raises(C.CrkfrError):
        s.set_inflow(np.zeros((1, 6)), 0.0)          # no inflow boundary
    g = C.Solver(C.EULER1D, 3, 8, bc=(C.INFLOW, C.OUTFLOW, 0, 0))
    g.set_state(W.euler1d_riemann(0, 8, 3))
    with pytest.raises(C.CrkfrError):
        g.step(0.0)                                   # no data yet
    with pytest.raises(C.CrkfrError):
        C.Batch([g])
    with pytest.raises(C.CrkfrError):
        g.set_inflow(np.zeros((6, 6)), 0.0)          # too many coefficients
    cf = np.zeros((1, 6))
    cf[0, :3] = (1.0, 0.5, 2.5 + 0.125)
    g.set_inflow(cf, 0.0)
    g.step(0.0)


def test_inflow_graph_advance_and_batch_equal_steps():
    N, nx = 3, 24
    gs = _ghost_size(C.EULER1D, N, nx, 1)
    cf = _euler_inflow_coef(gs, N, nx, 0.0, True, right_too=False)

    def make():
        s = C.Solver(C.EULER1D, N, nx, bc=(C.INFLOW, C.OUTFLOW, 0, 0), cfl=cfl_for(N))
        s.set_limiter(**LIM)
        s.set_state(W.euler1d_riemann(1, nx, N))
        s.set_inflow(cf, 0.0)
        return s
    a, b, c = make(), make(), make()
    for _ in range(8):
        a.step(0.0)
    b.advance(10.0, 8)
    bt = C.Batch([c])
    bt.advance(8)
    bt.sync()
    assert np.array_equal(a.get_state(), b.get_state())
    assert np.array_equal(a.get_state(), c.get_state())
