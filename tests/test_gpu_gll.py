"""GPU parity with Gauss-Legendre-Lobatto solution points and the g2
correction (Sec. 2, eqs. soln.points, fr.equiv) against the oracle:
unlimited runs of every equation, first-order blending with the flux and
scaling limiters, the smoothness indicator's alpha, FP32 bulk, batches."""
import numpy as np
import pytest

import oracle as O
from gpu_cases import rel_l1, rel_linf
from oracle_runs import cfl_table
from paper_2502_07517_amd import crkfr as C
from paper_2502_07517_amd import workloads as W

pytestmark = pytest.mark.gpu
GLL = C.POINTS_GLL
FO = dict(blend=C.BLEND_FO, flux_limiter=1, scaling=1)


def _cfl(eq, N, blend=False):
    """The g2 Fourier CFL; with blending at most the end subcells' width
    w_0 = 1/(N(N+1)) (the first-order subcell update's limit)."""
    c = cfl_table("cfl_gll" if eq == C.LINADV1D else "cfl_system_gll")[(N, min(N + 1, 4))]
    return min(c, 1.0 / (N * (N + 1))) if blend else c


def _pair(eq, N, nx, ny=1, *, lim=None, bc=(C.PERIODIC,) * 4, domain=(0.0, 1.0, 0.0, 1.0), dtype=C.FP64):
    lim = lim or {}
    cfl = _cfl(eq, N, blend=bool(lim))
    ref = O.RefConfig.make(eq, N, nx, ny, bc=bc, domain=domain, cfl=cfl, points=GLL, **lim)
    gpu = C.Solver(eq, N, nx, ny, bc=bc, domain=domain, dtype=dtype, cfl=cfl, points=GLL)
    if lim:
        gpu.set_limiter(**lim)
    return ref, gpu


def _run(ref, gpu, u0, steps):
    ghost = O.boundary_traces(ref, u0) if O.has_farfield(ref) else None
    dt = O.compute_dt(ref, u0)
    u = np.ascontiguousarray(u0, dtype=np.float64)
    gpu.set_state(u.copy())
    do = a = None
    for _ in range(steps):
        u, a, do, st = O.step(ref, u, dt, ghost=ghost)
        assert st == 0
        gpu.step(dt)
    return u, gpu.get_state().reshape(u.shape), a, do, gpu


def _smooth(eq, N):
    if eq in (C.LINADV1D, C.BURGERS1D):
        x = W.node_coords_1d(23, N, 0.0, 1.0, points=GLL)
        return (eq, N, 23), {}, (0.3 + 0.5 * np.sin(2 * np.pi * x) + 0.1 * np.cos(6 * np.pi * x))[None]
    if eq == C.EULER1D:
        x = W.node_coords_1d(23, N, 0.0, 1.0, points=GLL)
        return (eq, N, 23), {}, W.euler1d_cons(1 + 0.3 * np.sin(2 * np.pi * x), 0.5 + 0.2 * np.cos(2 * np.pi * x),
                                              1 + 0.2 * np.sin(2 * np.pi * (x + 0.3)))
    if eq == C.TENMOM1D:
        x = W.node_coords_1d(23, N, 0.0, 1.0, points=GLL)
        one = np.ones_like(x)
        return (eq, N, 23), {}, W.tenmom_cons(1 + 0.3 * np.sin(2 * np.pi * x), 0.4 * one, 0.1 * one,
                                              1 + 0.2 * np.cos(2 * np.pi * x), 0.1 * one, 0.9 * one)
    dom = (-5.0, 5.0, -5.0, 5.0)
    X, Y = W.node_coords_2d(9, 7, N, dom, points=GLL)
    if eq == C.EULER2D:
        return (eq, N, 9, 7), dict(domain=dom), W.euler2d_cons(*W.vortex_prim(X, Y, 0.0, dom))
    s = 2 * np.pi / 10
    return (eq, N, 9, 7), dict(domain=dom), W.tenmom_cons(1 + 0.3 * np.sin(s * (X + Y)), 0.3 + 0 * X, -0.2 + 0 * X,
                                                          1 + 0.2 * np.cos(s * X), 0.1 + 0 * X,
                                                          0.9 + 0.1 * np.sin(s * Y))


@pytest.mark.parametrize("N", [1, 2, 3, 4])
@pytest.mark.parametrize("eq", [C.LINADV1D, C.BURGERS1D, C.EULER1D, C.TENMOM1D, C.EULER2D, C.TENMOM2D])
def test_gll_unlimited_fp64(eq, N):
    args, kw, u0 = _smooth(eq, N)
    ref, gpu = _pair(*args, **kw)
    uo, ug, _, _, _ = _run(ref, gpu, u0, 8)
    assert rel_linf(uo, ug) <= 1e-11, rel_linf(uo, ug)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_fo_limited_euler1d_fp64(N):
    nx = 41
    ref, gpu = _pair(C.EULER1D, N, nx, lim=FO, bc=(C.FARFIELD,) * 4)
    x = W.node_coords_1d(nx, N, 0.0, 1.0, points=GLL)
    (rl, vl, pl), (rr, vr, pr) = W.riemann_states_1d(5)
    left = x < 0.5 + 0.37 / nx
    u0 = W.euler1d_cons(np.where(left, rl, rr), np.where(left, vl, vr), np.where(left, pl, pr))
    uo, ug, ao, do, g = _run(ref, gpu, u0, 15)
    assert rel_l1(uo, ug) <= 1e-9, rel_l1(uo, ug)
    dg, _ = g.get_diag()
    assert do["n_troubled"] == dg["n_troubled"] > 0
    assert np.max(np.abs(g.get_alpha().reshape(ao.shape) - ao)) <= 1e-9


@pytest.mark.parametrize("N", [2, 3])
def test_gll_fo_limited_euler2d_fp64(N):
    n = 10
    ref, gpu = _pair(C.EULER2D, N, n, n + 1, lim=FO, bc=(C.REFLECT,) * 4)
    X, Y = W.node_coords_2d(n, n + 1, N, (0, 1, 0, 1), points=GLL)
    prim = W._quadrant_fill(X, Y, 0.5 + 0.37 / n, 0.5 + 0.37 / (n + 1), W.quadrant_states_euler(3))
    uo, ug, _, do, g = _run(ref, gpu, W.euler2d_cons(*prim), 6)
    assert rel_l1(uo, ug) <= 1e-9, rel_l1(uo, ug)
    dg, _ = g.get_diag()
    assert do["n_troubled"] == dg["n_troubled"] > 0


def test_gll_mp32_vortex():
    N, n = 3, 16
    dom = (-5.0, 5.0, -5.0, 5.0)
    ref, gpu = _pair(C.EULER2D, N, n, n, domain=dom, dtype=C.MP32)
    X, Y = W.node_coords_2d(n, n, N, dom, points=GLL)
    uo, ug, _, _, _ = _run(ref, gpu, W.euler2d_cons(*W.vortex_prim(X, Y, 0.0, dom)), 10)
    assert rel_l1(uo, ug) <= 2e-6
    assert rel_linf(uo, ug) <= 2e-5


def test_gll_options_and_default_cfl():
    s = C.Solver(C.EULER1D, 3, 8, points=GLL)
    with pytest.raises(C.CrkfrError):
        s.set_limiter(blend=C.BLEND_MH)
    assert abs(s.cfl() - C.fourier_cfl(3, 0, 1, 1e-10, points=GLL)) < 1e-12
    assert abs(s.cfl() - _cfl(C.EULER1D, 3)) < 1e-6
    s.set_limiter(blend=C.BLEND_FO)
    assert abs(s.cfl() - 1.0 / 12.0) < 1e-15       # capped by the end subcell width
    s.set_limiter(blend=C.BLEND_OFF)
    assert abs(s.cfl() - _cfl(C.EULER1D, 3)) < 1e-6
    with pytest.raises(C.CrkfrError):
        C.Solver(C.EULER1D, 3, 8, points=2)


def test_gll_batch_equals_sequential():
    def make():
        out = []
        for i, (N, n) in enumerate([(2, 9), (3, 12), (3, 7)]):
            _, g = _pair(C.EULER2D, N, n, n + 1, lim=FO, bc=(C.FARFIELD,) * 4)
            X, Y = W.node_coords_2d(n, n + 1, N, (0, 1, 0, 1), points=GLL)
            prim = W._quadrant_fill(X, Y, 0.5 + 0.37 / n, 0.5 + 0.37 / (n + 1), W.quadrant_states_euler(i))
            g.set_state(W.euler2d_cons(*prim))
            out.append(g)
        return out
    seq, bat = make(), make()
    for s in seq:
        for _ in range(5):
            s.step(0.0)
    b = C.Batch(bat)
    b.advance(5)
    b.sync()
    for s1, s2 in zip(seq, bat):
        assert np.array_equal(s1.get_state(), s2.get_state())
