"""Pins of the oracle's second solution-point family: Gauss-Legendre-Lobatto
(GLL) points with the g2 correction function (Sec. 2, eqs. soln.points,
fr.equiv), with first-order (FO) blending as the low-order scheme.

  * the GLL rule: end points, interior nodes at the roots of P_N' (numpy),
    exact to degree 2N-1 and not 2N;
  * g2 built from its definition as a combination of right Radau polynomials
    (Huynh's g2 = N/(2N+1) R_{N+1} + (N+1)/(2N+1) R_N, left-correction form)
    has g_L'(xi_p) = -l_p(0)/w_p and g_R'(xi_p) = l_p(1)/w_p at the GLL nodes,
    the identity through which the step applies the correction;
  * single Legendre modes sampled at GLL nodes put all their energy in their
    own shell of the smoothness indicator (exact modal projection);
  * with GLL points the EA and AE central parts coincide (the traces are
    nodal values), as the paper states for Burgers;
  * linear advection converges at order N+1 with GLL/g2 and the Radau/GL
    errors are smaller at equal resolution (Sec. 5.1.1); Burgers with GLL/g2:
    near order N+1 for N = 2 and about N+1/2 for odd N (Sec. 5.1.3, Fig. b);
  * the Fourier CFL of GLL/g2 is the stability limit of the step;
  * FO blending with the flux and scaling limiters keeps a Riemann problem
    admissible and conserves the means exactly; MUSCL-Hancock with GLL points
    is rejected.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle as O
from oracle_runs import cfl_table
from paper_2502_07517_amd import workloads as W

GLL = O.POINTS_GLL


def _cfl_gll(N, system=True):
    return cfl_table("cfl_system_gll" if system else "cfl_gll")[(N, min(N + 1, 4))]


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gll_rule(N):
    xi, w = O.gll(N)
    assert xi[0] == 0.0 and xi[-1] == 1.0
    if N > 1:
        inner = np.sort(npleg.Legendre.basis(N).deriv().roots().real)
        assert np.max(np.abs(2 * xi[1:-1] - 1 - inner)) < 1e-14
    for k in range(2 * N + 1):
        exact = 1.0 / (k + 1)
        err = abs(np.dot(w, xi ** k) - exact)
        if k <= 2 * N - 1:
            assert err < 1e-14, (k, err)
        else:
            assert err > 1e-6, (k, err)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_g2_identity_at_gll_nodes(N):
    P = npleg.Legendre.basis

    def radau_right(k):          # zero at x = 1, one at x = -1
        return ((-1) ** k / 2.0) * (P(k) - P(k - 1))
    gL = (N / (2 * N + 1.0)) * radau_right(N + 1) + ((N + 1) / (2 * N + 1.0)) * radau_right(N)
    assert abs(gL(-1.0) - 1.0) < 1e-14 and abs(gL(1.0)) < 1e-14
    xi, w = O.gll(N)
    l0, l1 = O.lagrange_at(N, xi, 0.0), O.lagrange_at(N, xi, 1.0)
    # on [0, 1]: g_L(xi) = gL(2 xi - 1), g_R(xi) = g_L(1 - xi)
    dgL = 2.0 * gL.deriv()(2 * xi - 1)
    dgR = -2.0 * gL.deriv()(2 * (1 - xi) - 1)
    assert np.max(np.abs(dgL + l0 / w)) < 1e-12 * np.max(np.abs(l0 / w))
    assert np.max(np.abs(dgR - l1 / w)) < 1e-12 * np.max(np.abs(l1 / w))
    # with GL points the g2 identity does not hold (Radau's does)
    xg, wg = O.gl(N)
    assert np.max(np.abs(2.0 * gL.deriv()(2 * xg - 1) + O.lagrange_at(N, xg, 0.0) / wg)) > 1e-3


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_single_modes_fill_their_own_shell(N):
    cfg = O.RefConfig.make(O.LINADV1D, N, 1, points=GLL)
    xi, _ = O.gll(N)
    for k in range(N + 1):
        ue = np.sqrt(2 * k + 1) * npleg.Legendre.basis(k)(2 * xi - 1)
        _, e = O.indicator_raw(cfg, ue[None])
        assert abs(e[k] - 1.0) < 1e-12
        assert np.sum(np.delete(e, k)) < 1e-24


@pytest.mark.parametrize("eq", [O.BURGERS1D, O.EULER1D, O.EULER2D])
@pytest.mark.parametrize("N", [2, 3])
def test_ea_equals_ae_with_gll(eq, N):
    if eq == O.BURGERS1D:
        x = W.node_coords_1d(12, N, 0.0, 1.0, points=GLL)
        args, u = (eq, N, 12), (0.3 + np.sin(2 * np.pi * x))[None]
    elif eq == O.EULER1D:
        x = W.node_coords_1d(12, N, 0.0, 1.0, points=GLL)
        args, u = (eq, N, 12), W.euler1d_cons(1 + 0.3 * np.sin(2 * np.pi * x), 0.5 + 0 * x,
                                              1 + 0.2 * np.cos(2 * np.pi * x))
    else:
        X, Y = W.node_coords_2d(5, 4, N, (0, 1, 0, 1), points=GLL)
        args, u = (eq, N, 5, 4), W.euler2d_cons(1 + 0.3 * np.sin(2 * np.pi * (X + Y)), 0.4 + 0 * X,
                                                -0.3 + 0 * X, 1 + 0.2 * np.cos(2 * np.pi * X))
    outs = []
    for cen in (O.CENTRAL_EA, O.CENTRAL_AE):
        cfg = O.RefConfig.make(*args, cfl=_cfl_gll(N), points=GLL, central=cen)
        v = u.copy()
        for _ in range(4):
            v, _, _, st = O.step(cfg, v, O.compute_dt(cfg, v))
            assert st == 0
        outs.append(v)
    assert np.max(np.abs(outs[0] - outs[1])) < 1e-13 * np.max(np.abs(outs[0]))


def _linadv_error(N, nx, points, nsteps):
    x = W.node_coords_1d(nx, N, 0.0, 1.0, points=points)
    cfg = O.RefConfig.make(O.LINADV1D, N, nx, cfl=0.1, points=points)
    u = np.sin(2 * np.pi * x)[None]
    T = 1.0
    for _ in range(nsteps):
        u, _, _, _ = O.step(cfg, u, T / nsteps)
    _, w = O.nodes(N, points)
    # error of the polynomial at GL points (exact quadrature of its square)
    xg, wg = O.gl(N + 2)
    L = np.stack([O.lagrange_at(N, O.nodes(N, points)[0], s) for s in xg])      # [j][p]
    uh = u[0] @ L.T
    xe = (np.arange(nx)[:, None] + xg[None, :]) / nx
    return math.sqrt(np.sum((uh - np.sin(2 * np.pi * (xe - T))) ** 2 * wg[None, :]) / nx)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_linear_advection_gll_order_and_radau_smaller_errors(N):
    grids = (10, 20, 40)
    steps = [int(40 * n / 10 * (N + 1)) for n in grids]     # same small dt for both families
    e_gll = [_linadv_error(N, n, GLL, s) for n, s in zip(grids, steps)]
    e_gl = [_linadv_error(N, n, O.POINTS_GL, s) for n, s in zip(grids, steps)]
    order = math.log2(e_gll[-2] / e_gll[-1])
    assert order > N + 0.8, (e_gll, order)
    assert all(a < b for a, b in zip(e_gl, e_gll)), (e_gl, e_gll)


def _burgers_error(N, nx, points):
    cfg = O.RefConfig.make(O.BURGERS1D, N, nx, domain=(0.0, 2 * np.pi, 0.0, 1.0), cfl=_cfl_gll(N),
                           points=points)
    u = W.burgers_sine(nx, N, points=points)
    t = 0.0
    while t < 2.0 - 1e-14:
        dt = min(O.compute_dt(cfg, u), 2.0 - t)
        u, _, _, st = O.step(cfg, u, dt)
        assert st == 0
        t += dt
    xg, wg = O.gl(N + 2)
    L = np.stack([O.lagrange_at(N, O.nodes(N, points)[0], s) for s in xg])
    uh = u[0] @ L.T
    x = (np.arange(nx)[:, None] + xg[None, :]) * (2 * np.pi / nx)
    ue = 0.2 * np.sin(x)
    for _ in range(60):
        ue = ue - (ue - 0.2 * np.sin(x - 2.0 * ue)) / (1.0 + 0.4 * np.cos(x - 2.0 * ue))
    return math.sqrt(np.sum((uh - ue) ** 2 * wg[None, :]) / nx)


@pytest.mark.parametrize("N,grids,lo,hi", [(1, (128, 256), 1.2, 1.7), (2, (128, 256), 2.7, 3.2),
                                           (3, (64, 128), 3.2, 3.6)])
def test_burgers_gll_orders(N, grids, lo, hi):
    """Measured 1.45, 2.75 and 3.36: the even degree is near its optimal
    order, the odd ones near N+1/2 (a method-of-lines DGSEM computation with
    RK4 and small steps, the spatial scheme GLL/g2 is equivalent to, shows
    1.43, 2.82 and 3.39 on the same grids)."""
    e = [_burgers_error(N, n, GLL) for n in grids]
    order = math.log2(e[0] / e[1])
    assert lo < order < hi, (e, order)


@pytest.mark.parametrize("N", [1, 2, 3])
def test_gll_cfl_is_the_stability_limit(N):
    nx = 10
    cfl = _cfl_gll(N, system=False)
    x = W.node_coords_1d(nx, N, 0.0, 1.0, points=GLL)
    u0 = np.sin(2 * np.pi * x)[None] + 1e-3 * np.random.default_rng(2).standard_normal((1, nx, N + 1))
    cfg = O.RefConfig.make(O.LINADV1D, N, nx, cfl=cfl, points=GLL)
    for fac, stable in ((0.98, True), (1.1, False)):
        u = u0.copy()
        for _ in range(4000):
            u, _, _, _ = O.step(cfg, u, fac * cfl / nx)
            if not np.isfinite(u).all() or np.abs(u).max() > 1e3:
                break
        grown = not np.isfinite(u).all() or np.abs(u).max() > 10 * np.abs(u0).max()
        assert grown != stable, (N, fac)


def test_g2_cfl_values():
    """GLL/g2 with degree N has the CFL number of Radau/GL with degree N-1
    (1, then the Radau values), the familiar DG-with-lumping relation."""
    assert abs(_cfl_gll(1, system=False) - 1.0) < 1e-6
    for N in (2, 3):
        assert abs(_cfl_gll(N, system=False) - cfl_table("cfl")[(N - 1, N)]) < 1e-6


@pytest.mark.parametrize("N", [2, 3, 4])
def test_fo_blending_with_gll_admissible_and_conservative(N):
    nx = 40
    x = W.node_coords_1d(nx, N, 0.0, 1.0, points=GLL)
    left = x < 0.5 + 0.37 / nx
    u = W.euler1d_cons(np.where(left, 1.0, 0.125), 0 * x, np.where(left, 1.0, 0.1))
    # the time step also keeps the first-order update on the end subcells
    # (width w_0 = 1/(N(N+1))) admissible, the condition of Theorem 1
    cfl = min(_cfl_gll(N), 1.0 / (N * (N + 1)))
    cfg = O.RefConfig.make(O.EULER1D, N, nx, bc=(O.OUTFLOW,) * 4, cfl=cfl, points=GLL,
                           blend=O.BLEND_FO, flux_limiter=1, scaling=1)
    _, w = O.gll(N)
    m0 = (u * w).sum(axis=(1, 2))
    troubled = 0
    for _ in range(20):
        u, _, d, st = O.step(cfg, u, O.compute_dt(cfg, u))
        assert st == 0
        troubled += d["n_troubled"]
        p = 0.4 * (u[2] - 0.5 * u[1] ** 2 / u[0])
        assert u[0].min() > 0 and p.min() > 0
    assert troubled > 0
    # the waves have not reached the boundaries, where the gas is at rest: no
    # mass crosses them, so the total mass is conserved to rounding
    assert abs((u[0] * w).sum() - m0[0]) < 1e-13 * m0[0]
    bad = O.RefConfig.make(O.EULER1D, N, nx, cfl=_cfl_gll(N), points=GLL, blend=O.BLEND_MH)
    assert O.step(bad, u, 1e-4)[3] == -1


@pytest.mark.parametrize("N", [2, 3, 4])
def test_gll_fourier_cfl_too_large_for_the_subcell_update(N):
    """At the g2 Fourier CFL the first-order update on the end subcells
    (width w_0 = 1/(N(N+1)) < CFL) is not admissible, and the flux limiter
    cannot keep the means admissible: the reason for the w_0 cap."""
    nx = 40
    x = W.node_coords_1d(nx, N, 0.0, 1.0, points=GLL)
    left = x < 0.5 + 0.37 / nx
    u = W.euler1d_cons(np.where(left, 1.0, 0.125), 0 * x, np.where(left, 1.0, 0.1))
    assert _cfl_gll(N) > O.gll(N)[1][0]
    cfg = O.RefConfig.make(O.EULER1D, N, nx, bc=(O.OUTFLOW,) * 4, cfl=_cfl_gll(N), points=GLL,
                           blend=O.BLEND_FO, flux_limiter=1, scaling=1)
    sts = []
    for _ in range(20):
        u, _, _, st = O.step(cfg, u, O.compute_dt(cfg, u))
        sts.append(st)
        if st:
            break
    assert -5 in sts
