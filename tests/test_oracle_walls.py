"""Pins of the oracle's solid-wall boundaries (Sec. 3.3, eq. reflect.time.avg)
and of the admissibility stress tests the paper runs with them.

The wall rule is pinned against the interior scheme itself: a run on [0, 1]
with walls equals the right half of a run on the doubled periodic domain
whose left half holds the mirror image of the data (the mirror image of the
interior traces is exactly the wall's ghost), with the whole limiter chain
on."""
import numpy as np
import pytest

import oracle as O
from oracle_runs import cfl_for
from paper_2502_07517_amd import workloads as W

LIM = dict(blend=O.BLEND_MH, flux_limiter=1, scaling=1)


def _mirror_1d(u):
    """u[var][ex][p] on [0,1] -> doubled [-1,1]: left half = mirrored image."""
    m = u[:, ::-1, ::-1].copy()
    m[1] *= -1.0
    return np.concatenate([m, u], axis=1)


@pytest.mark.parametrize("N", [2, 3])
def test_wall_equals_mirrored_periodic_run_1d(N):
    nx, steps = 20, 25
    rng = np.random.default_rng(N)
    x = W.node_coords_1d(nx, N, 0.0, 1.0)
    rho = 1.0 + 0.5 * np.where(x < 0.43, 1.0, 0.2) + 0.1 * np.sin(7 * x)
    v = 0.6 * np.sin(3 * x) + rng.uniform(-0.1, 0.1)
    p = np.where(x < 0.43, 2.0, 0.3)
    u = np.stack([rho, rho * v, p / 0.4 + 0.5 * rho * v * v])
    cw = O.RefConfig.make(O.EULER1D, N, nx, bc=(O.REFLECT,) * 4, domain=(0, 1, 0, 1), cfl=cfl_for(N), **LIM)
    cd = O.RefConfig.make(O.EULER1D, N, 2 * nx, bc=(O.PERIODIC,) * 4, domain=(-1, 1, 0, 1), cfl=cfl_for(N), **LIM)
    ud = _mirror_1d(u)
    dt = 0.5 * O.compute_dt(cw, u)
    tw = 0
    for _ in range(steps):
        u, _, dw, _ = O.step(cw, u, dt)
        ud, _, dd, _ = O.step(cd, ud, dt)
        tw += dw["n_troubled"]
    assert tw > 0      # the limiter chain takes part
    assert np.max(np.abs(ud[:, nx:] - u)) < 1e-12 * np.max(np.abs(u))


@pytest.mark.parametrize("eq", [O.EULER2D, O.TENMOM2D])
@pytest.mark.parametrize("d", [0, 1])
def test_wall_equals_mirrored_periodic_run_2d(eq, d):
    N, n, steps = 2, 8, 8
    M = O.nvar(eq)
    if eq == O.EULER2D:
        u = W.euler2d_quadrants(5, n, N, split=(0.43, 0.56))
    else:
        u = W.tenmom2d_quadrants(5, n, n, N, dom=(0, 1, 0, 1), split=(0.43, 0.56))
    u = u.reshape(M, n, n, N + 1, N + 1)
    flip = [1 + d] + ([4] if eq == O.TENMOM2D else [])
    if d == 0:
        m = u[:, :, ::-1, :, ::-1].copy()
        for v in flip:
            m[v] *= -1.0
        ud = np.concatenate([m, u], axis=2)
        dom_d, nxd, nyd = (-1, 1, 0, 1), 2 * n, n
        bcw, bcd = (O.REFLECT, O.REFLECT, O.PERIODIC, O.PERIODIC), (O.PERIODIC,) * 4
    else:
        m = u[:, ::-1, :, ::-1, :].copy()
        for v in flip:
            m[v] *= -1.0
        ud = np.concatenate([m, u], axis=1)
        dom_d, nxd, nyd = (0, 1, -1, 1), n, 2 * n
        bcw, bcd = (O.PERIODIC, O.PERIODIC, O.REFLECT, O.REFLECT), (O.PERIODIC,) * 4
    cw = O.RefConfig.make(eq, N, n, n, bc=bcw, domain=(0, 1, 0, 1), cfl=cfl_for(N), **LIM)
    cd = O.RefConfig.make(eq, N, nxd, nyd, bc=bcd, domain=dom_d, cfl=cfl_for(N), **LIM)
    dt = 0.5 * O.compute_dt(cw, u)
    uw = u.reshape(M, -1).copy()
    udd = ud.reshape(M, -1).copy()
    for _ in range(steps):
        uw, _, _, st = O.step(cw, uw, dt)
        udd, _, _, _ = O.step(cd, udd, dt)
        assert st == 0
    half = udd.reshape(ud.shape)[:, :, n:] if d == 0 else udd.reshape(ud.shape)[:, n:]
    assert np.max(np.abs(half - uw.reshape(u.shape))) < 1e-12 * np.max(np.abs(uw))


def test_walls_conserve_mass_exactly_and_stop_mass_flux():
    """No mass crosses a wall: the mass flux of eq. reflect.time.avg is
    (-F1 + F1)/2 - lambda/2 (U1 - U1) = 0, so the total mass is constant."""
    N, n = 3, 10
    u = W.euler2d_quadrants(2, n, N)
    cfg = O.RefConfig.make(O.EULER2D, N, n, n, bc=(O.REFLECT,) * 4, cfl=cfl_for(N), **LIM)
    _, w = O.gl(N)
    W2 = np.outer(w, w)

    def mass(u):
        return (u.reshape(4, n, n, N + 1, N + 1)[0] * W2).sum()
    m0 = mass(u)
    for _ in range(20):
        u, _, d, st = O.step(cfg, u, O.compute_dt(cfg, u))
        assert st == 0
    assert abs(mass(u) - m0) < 1e-13 * m0


def _euler1d(rho, v, p):
    return np.stack([rho, rho * v, p / 0.4 + 0.5 * rho * v * v])


def _node_pressure(u):
    return 0.4 * (u[2] - 0.5 * u[1] ** 2 / u[0])


def _blast(nx, N):
    x = W.node_coords_1d(nx, N, 0.0, 1.0)
    p = np.where(x < 0.1, 1000.0, np.where(x > 0.9, 100.0, 0.01))
    return _euler1d(np.ones_like(x), np.zeros_like(x), p)


def _run_until(cfg, u, t_end, max_steps):
    t, k, ok = 0.0, 0, True
    while t < t_end - 1e-15 and k < max_steps:
        dt = min(O.compute_dt(cfg, u), t_end - t)
        if not np.isfinite(dt) or dt <= 0:
            return u, t, False
        u, _, d, st = O.step(cfg, u, dt)
        t += dt
        k += 1
        if st != 0 or d["n_mean_inadmissible"] or not np.all(np.isfinite(u)):
            return u, t, False
        if np.min(u[0]) <= 0 or np.min(_node_pressure(u)) <= 0:
            ok = False
    return u, t, ok


@pytest.mark.slow
def test_blast_wave_admissible_with_limiters_and_not_without():
    """Woodward-Colella blast wave between walls (Sec. 5.2): with the flux
    limiter and the scaling limiter every node stays admissible up to
    t = 0.038; without them the scheme produces negative pressure."""
    N, nx = 3, 100
    cfg = O.RefConfig.make(O.EULER1D, N, nx, bc=(O.REFLECT,) * 4, cfl=cfl_for(N), **LIM)
    u, t, ok = _run_until(cfg, _blast(nx, N), 0.038, 20000)
    assert ok and abs(t - 0.038) < 1e-12
    assert np.max(u[0]) > 3.0          # the colliding shocks compress the gas
    cfg0 = O.RefConfig.make(O.EULER1D, N, nx, bc=(O.REFLECT,) * 4, cfl=cfl_for(N), blend=O.BLEND_MH)
    _, _, ok0 = _run_until(cfg0, _blast(nx, N), 0.038, 20000)
    assert not ok0


def _sedov1d(nx, N):
    x = W.node_coords_1d(nx, N, -1.0, 1.0)
    dx = 2.0 / nx
    E = np.where(np.abs(x) <= dx / 2, 3.2e6 / dx, 1e-12)
    z = np.zeros_like(x)
    return np.stack([np.ones_like(x), z, E])


@pytest.mark.slow
def test_sedov_1d_admissible_and_symmetric():
    """1D Sedov blast between walls on [-1, 1] with 201 elements (Sec. 5.2,
    E = 3.2e6/dx in the central element, 1e-12 elsewhere): admissible at
    every node up to t = 0.001 and mirror symmetric about x = 0."""
    N, nx = 3, 201
    cfg = O.RefConfig.make(O.EULER1D, N, nx, bc=(O.REFLECT,) * 4, domain=(-1, 1, 0, 1), cfl=cfl_for(N), **LIM)
    u, t, ok = _run_until(cfg, _sedov1d(nx, N), 0.001, 100000)
    assert ok and abs(t - 0.001) < 1e-15
    m = u[:, ::-1, ::-1].copy()
    m[1] *= -1.0
    assert np.max(np.abs(m - u)) < 1e-9 * np.max(np.abs(u))
    assert np.max(u[0]) > 2.0           # the blast shock compresses the gas
