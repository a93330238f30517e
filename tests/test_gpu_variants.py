"""GPU parity of the scheme options against the oracle: the dissipation
models D1 / D2 / D-CSX (Sec. 3.1.1, eqs. D1, D2, dcsx), the central part from
evaluated (EA, eq. evaluate) or extrapolated (AE, eq. extrapolate) flux
traces (Sec. 3.1.2), the cRK stage count (eqs. crk22-crk44), and Burgers'
equation (Sec. 5.1.3), unlimited and with the limiter chain, FP64 and the
FP32 bulk form."""
import math

import numpy as np
import pytest

import oracle as O
from gpu_cases import rel_l1, rel_linf
from oracle_runs import cfl_table
from paper_2502_07517_amd import crkfr as C
from paper_2502_07517_amd import workloads as W

pytestmark = pytest.mark.gpu

SCHEMES = [(C.DISS_D1, C.CENTRAL_EA), (C.DISS_DCSX, C.CENTRAL_EA), (C.DISS_D2, C.CENTRAL_AE),
           (C.DISS_DCSX, C.CENTRAL_AE), (C.DISS_D1, C.CENTRAL_AE)]
LIM = dict(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
FF = (C.FARFIELD,) * 4
WALLS = (C.REFLECT,) * 4


def _cfl(eq, N, s, diss):
    """System CFL of the Fourier tables for (N, s) and the dissipation; the
    D1 tables hold the pairs s = N+1 (min 4) only: other pairs take half the
    D2 value, which is below the D1 value for every tabulated pair."""
    s = s or min(N + 1, 4)
    kind = "cfl" if eq == C.LINADV1D else "cfl_system"
    if diss == C.DISS_D1:
        t = cfl_table(kind + "_d1")
        if (N, s) in t:
            return t[(N, s)]
        return 0.5 * cfl_table(kind)[(N, s)]
    return cfl_table(kind)[(N, s)]


def _pair(eq, N, nx, ny=1, *, stages=0, diss=C.DISS_D2, cen=C.CENTRAL_EA, dtype=C.FP64, lim=None,
          bc=(C.PERIODIC,) * 4, domain=(0.0, 1.0, 0.0, 1.0)):
    lim = lim or {}
    cfl = _cfl(eq, N, stages, diss)
    ref = O.RefConfig.make(eq, N, nx, ny, stages=stages or None, bc=bc, domain=domain, cfl=cfl,
                           dissipation=diss, central=cen, **lim)
    gpu = C.Solver(eq, N, nx, ny, bc=bc, domain=domain, dtype=dtype, cfl=cfl)
    gpu.set_scheme(stages, diss, cen)
    if lim:
        gpu.set_limiter(**lim)
    return ref, gpu


def _run(ref, gpu, u0, steps):
    """Same fixed dt on both sides; returns oracle state, GPU state, last diags."""
    ghost = O.boundary_traces(ref, u0) if O.has_farfield(ref) else None
    dt = O.compute_dt(ref, u0)
    u = np.ascontiguousarray(u0, dtype=np.float64)
    gpu.set_state(u.copy())
    do = None
    for _ in range(steps):
        u, _, do, st = O.step(ref, u, dt, ghost=ghost)
        assert st == 0
        gpu.step(dt)
    return u, gpu.get_state().reshape(u.shape), do, gpu.get_diag()[0]


def _smooth(eq, N):
    if eq == C.LINADV1D:
        return (eq, N, 37), dict(), W.linadv_modes(1, 37, N)
    if eq == C.EULER1D:
        return (eq, N, 23), dict(), W.euler1d_smooth(2, 23, N)
    if eq == C.BURGERS1D:
        # the smooth Burgers data (amplitude 0.2 on [0, 2 pi]) with a nonzero mean
        return (eq, N, 29), dict(domain=(0.0, 2 * np.pi, 0.0, 1.0)), W.burgers_sine(29, N, shift=0.05)
    if eq == C.TENMOM1D:
        u = W.tenmom1d_equilibrium(31, N)
        u[1] += 0.1 * np.sin(np.pi * W.node_coords_1d(31, N, 0.0, 4.0))
        return (eq, N, 31), dict(domain=(0.0, 4.0, 0.0, 1.0)), u
    if eq == C.EULER2D:
        dom = (-5.0, 5.0, -5.0, 5.0)
        return (eq, N, 9, 7), dict(domain=dom), W.euler2d_cons(*W.vortex_prim(*W.node_coords_2d(9, 7, N, dom)))
    dom = (-2.0, 2.0, -0.5, 0.5)
    return (eq, N, 7, 6), dict(domain=dom), W.tenmom2d_smooth(3, 7, 6, N, dom)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("eq", [C.LINADV1D, C.EULER1D, C.BURGERS1D, C.TENMOM1D, C.EULER2D, C.TENMOM2D])
def test_scheme_options_smooth_fp64(eq, scheme):
    N = 3
    args, kw, u0 = _smooth(eq, N)
    ref, gpu = _pair(*args, diss=scheme[0], cen=scheme[1], **kw)
    uo, ug, _, _ = _run(ref, gpu, u0, 10)
    assert rel_linf(uo, ug) <= 1e-11, rel_linf(uo, ug)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("stages", [2, 3, 4])
@pytest.mark.parametrize("diss", [C.DISS_D2, C.DISS_DCSX])
def test_stage_counts_fp64(N, stages, diss):
    dom = (-5.0, 5.0, -5.0, 5.0)
    ref, gpu = _pair(C.EULER2D, N, 6, 5, stages=stages, diss=diss, domain=dom)
    u0 = W.euler2d_cons(*W.vortex_prim(*W.node_coords_2d(6, 5, N, dom)))
    uo, ug, _, _ = _run(ref, gpu, u0, 6)
    assert rel_linf(uo, ug) <= 1e-11, rel_linf(uo, ug)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_scheme_options_limited_euler1d_fp64(scheme):
    N, nx = 3, 41
    ref, gpu = _pair(C.EULER1D, N, nx, diss=scheme[0], cen=scheme[1], lim=LIM, bc=FF)
    uo, ug, do, dg = _run(ref, gpu, W.euler1d_riemann(3, nx, N), 15)
    assert rel_l1(uo, ug) <= 1e-9, rel_l1(uo, ug)
    assert do["n_troubled"] == dg["n_troubled"]
    assert dg["n_mean_inadmissible"] == 0


@pytest.mark.parametrize("scheme", SCHEMES)
def test_scheme_options_limited_euler2d_walls_fp64(scheme):
    N, n = 3, 10
    ref, gpu = _pair(C.EULER2D, N, n, n + 1, diss=scheme[0], cen=scheme[1], lim=LIM, bc=WALLS)
    X, Y = W.node_coords_2d(n, n + 1, N, (0, 1, 0, 1))
    prim = W._quadrant_fill(X, Y, 0.5 + 0.37 / n, 0.5 + 0.37 / (n + 1), W.quadrant_states_euler(4))
    uo, ug, do, dg = _run(ref, gpu, W.euler2d_cons(*prim), 6)
    assert rel_l1(uo, ug) <= 1e-9, rel_l1(uo, ug)
    assert do["n_troubled"] == dg["n_troubled"]


@pytest.mark.parametrize("scheme", [(C.DISS_DCSX, C.CENTRAL_EA), (C.DISS_D1, C.CENTRAL_AE)])
def test_scheme_options_tenmom_farfield_limited_fp64(scheme):
    N, nx, ny = 3, 12, 6
    dom = (-2.0, 2.0, -0.5, 0.5)
    ref, gpu = _pair(C.TENMOM2D, N, nx, ny, diss=scheme[0], cen=scheme[1], lim=LIM, bc=FF, domain=dom)
    uo, ug, _, _ = _run(ref, gpu, W.tenmom2d_quadrants(2, nx, ny, N, dom), 6)
    assert rel_l1(uo, ug) <= 1e-9, rel_l1(uo, ug)


@pytest.mark.parametrize("scheme", [(C.DISS_D2, C.CENTRAL_EA), (C.DISS_DCSX, C.CENTRAL_EA),
                                    (C.DISS_D1, C.CENTRAL_AE)])
def test_scheme_options_mp32(scheme):
    dom = (-5.0, 5.0, -5.0, 5.0)
    n, N = 16, 3
    ref, gpu = _pair(C.EULER2D, N, n, n, diss=scheme[0], cen=scheme[1], dtype=C.MP32, domain=dom)
    uo, ug, _, _ = _run(ref, gpu, W.vortex2d(n, N, 0.0, dom), 10)
    assert rel_l1(uo, ug) <= 2e-6
    assert rel_linf(uo, ug) <= 2e-5


def _burgers_exact(x, t, amp=0.2):
    u = amp * np.sin(x)
    for _ in range(60):
        u = u - (u - amp * np.sin(x - u * t)) / (1.0 + amp * t * np.cos(x - u * t))
    return u


@pytest.mark.parametrize("N", [1, 3])
def test_burgers_orders_on_gpu(N):
    """u0 = 0.2 sin(x) on [0, 2 pi] to t = 2 with device time steps: the GPU
    errors against the exact solution equal the oracle's, EA converges at
    order N+1, AE at about N+1/2 for odd N (Sec. 5.1.3)."""
    grids = (128, 256)
    dom = (0.0, 2 * np.pi, 0.0, 1.0)
    _, w = O.gl(N)
    errs = {}
    for cen in (C.CENTRAL_EA, C.CENTRAL_AE):
        for nx in grids:
            ref, gpu = _pair(C.BURGERS1D, N, nx, cen=cen, domain=dom)
            gpu.set_state(W.burgers_sine(nx, N))
            gpu.advance(2.0, 100000)
            d, rc = gpu.get_diag()
            assert rc == 0 and abs(d["t"] - 2.0) < 1e-12
            x = W.node_coords_1d(nx, N, 0.0, 2 * np.pi)
            e = gpu.get_state().reshape(1, nx, N + 1)[0] - _burgers_exact(x, 2.0)
            errs[(cen, nx)] = math.sqrt(np.sum(e ** 2 * w[None, :]) / nx)
        # the oracle's error on the finest grid with its own time steps
        u = W.burgers_sine(grids[-1], N)
        t = 0.0
        while t < 2.0 - 1e-14:
            dt = min(O.compute_dt(ref, u), 2.0 - t)
            u, _, _, _ = O.step(ref, u, dt)
            t += dt
        eo = u[0] - _burgers_exact(W.node_coords_1d(grids[-1], N, 0.0, 2 * np.pi), 2.0)
        eo = math.sqrt(np.sum(eo ** 2 * w[None, :]) / grids[-1])
        assert abs(eo - errs[(cen, grids[-1])]) <= 1e-6 * eo
    o_ea = math.log2(errs[(C.CENTRAL_EA, grids[0])] / errs[(C.CENTRAL_EA, grids[1])])
    o_ae = math.log2(errs[(C.CENTRAL_AE, grids[0])] / errs[(C.CENTRAL_AE, grids[1])])
    print(f"Burgers N={N}: EA order {o_ea:.2f}, AE order {o_ae:.2f}")
    assert o_ea > N + 0.8 and N + 0.2 < o_ae < N + 0.8


def test_burgers_shock_limited_fp64_and_mp32():
    """Burgers past the shock time (t = 6 > 5) with the limiter chain: single
    steps from the oracle's states agree to rounding (FP64)."""
    N, nx = 3, 40
    dom = (0.0, 2 * np.pi, 0.0, 1.0)
    ref, gpu = _pair(C.BURGERS1D, N, nx, lim=LIM, domain=dom)
    u = W.burgers_sine(nx, N)
    t, k, worst, troubled = 0.0, 0, 0.0, 0
    while t < 6.0 - 1e-12:
        dt = min(O.compute_dt(ref, u), 6.0 - t)
        un, _, do, st = O.step(ref, u, dt)
        assert st == 0
        if k % 9 == 0:
            gpu.set_state(u.copy())
            gpu.step(dt)
            dg, _ = gpu.get_diag()
            worst = max(worst, rel_l1(un, gpu.get_state().reshape(un.shape)))
            assert do["n_troubled"] == dg["n_troubled"]
            troubled += do["n_troubled"]
        u, t, k = un, t + dt, k + 1
    assert worst <= 1e-12 and troubled > 0
    _, g32 = _pair(C.BURGERS1D, N, nx, lim=LIM, domain=dom, dtype=C.MP32)
    g32.set_state(W.burgers_sine(nx, N))
    g32.advance(6.0, 100000)
    assert rel_l1(u, g32.get_state().reshape(u.shape)) <= 1e-3


def test_dcsx_graph_advance_matches_steps():
    """D-CSX enlarges the trace buffers: an advance captured after the
    change equals stepping with the device time step."""
    N, n = 3, 8
    dom = (-5.0, 5.0, -5.0, 5.0)
    u0 = W.vortex2d(n, N, 0.0, dom)
    a = C.Solver(C.EULER2D, N, n, n, domain=dom)
    b = C.Solver(C.EULER2D, N, n, n, domain=dom)
    b.set_state(u0.copy())
    b.advance(10.0, 3)          # a graph with the default scheme first
    for s in (a, b):
        s.set_scheme(0, C.DISS_DCSX, C.CENTRAL_AE)
        s.set_state(u0.copy())
    for _ in range(7):
        a.step(0.0)
    b.advance(10.0, 7)
    assert np.array_equal(a.get_state(), b.get_state())


def test_set_scheme_rejects_bad_options():
    s = C.Solver(C.EULER1D, 3, 8)
    for bad in ((1, 0, 0), (5, 0, 0), (0, 3, 0), (0, 0, 2), (0, -1, 0)):
        with pytest.raises(C.CrkfrError):
            s.set_scheme(*bad)
    s.set_scheme(2, C.DISS_D1, C.CENTRAL_AE)


def test_default_cfl_follows_scheme():
    """With no CFL given the solver takes the Fourier value of its scheme:
    D1 gives a smaller time step than D2."""
    u0 = W.euler1d_smooth(0, 16, 3)
    s = C.Solver(C.EULER1D, 3, 16)
    s.set_state(u0.copy())
    dt2 = s.compute_dt()
    s.set_scheme(0, C.DISS_D1, C.CENTRAL_EA)
    dt1 = s.compute_dt()
    assert abs(dt1 / dt2 - C.fourier_cfl(3, 0, 1, 1e-10, C.DISS_D1) / C.fourier_cfl(3, 0, 1, 1e-10)) < 1e-12
    assert dt1 < dt2


def _batch_members(dtype):
    """Uneven 2D Euler members with different scheme options per member."""
    opts = [(0, C.DISS_DCSX, C.CENTRAL_AE), (0, C.DISS_D1, C.CENTRAL_EA), (2, C.DISS_D2, C.CENTRAL_EA),
            (3, C.DISS_DCSX, C.CENTRAL_EA)]
    out = []
    for i, (stages, diss, cen) in enumerate(opts):
        N, n = (3, 2, 3, 2)[i], 7 + 3 * i
        s = C.Solver(C.EULER2D, N, n, n + 1, bc=(C.FARFIELD,) * 4, dtype=dtype, cfl=_cfl(C.EULER2D, N, stages, diss))
        s.set_scheme(stages, diss, cen)
        s.set_limiter(**LIM)
        X, Y = W.node_coords_2d(n, n + 1, N, (0, 1, 0, 1))
        prim = W._quadrant_fill(X, Y, 0.5 + 0.37 / n, 0.5 + 0.37 / (n + 1), W.quadrant_states_euler(i))
        s.set_state(W.euler2d_cons(*prim))
        out.append(s)
    return out


@pytest.mark.parametrize("dtype", [C.FP64, C.MP32])
def test_batch_with_scheme_options_equals_sequential(dtype):
    seq, bat = _batch_members(dtype), _batch_members(dtype)
    for s in seq:
        for _ in range(5):
            s.step(0.0)
    b = C.Batch(bat)
    with pytest.raises(C.CrkfrError):
        bat[0].set_scheme(0, C.DISS_D2, C.CENTRAL_EA)     # a live batch holds the member's buffers
    b.step()
    b.advance(4)
    b.sync()
    for s1, s2 in zip(seq, bat):
        assert np.array_equal(s1.get_state(), s2.get_state())
    b.close()
    bat[0].set_scheme(0, C.DISS_D2, C.CENTRAL_EA)
