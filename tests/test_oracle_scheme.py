"""Scheme-level pins of the oracle: exact translation and convergence order,
conservation, equal means of the blended scheme, admissibility (Theorem 1 +
scaling), CFL stability by brute force, the first-order limit against an
independent finite-volume code, linear-data exactness of MUSCL-Hancock, and the
source-term ODE limit."""
import numpy as np
import pytest

import oracle
from oracle_runs import cfl_for, run, l1_error_1d, l1_error_2d
from paper_2502_07517_amd import workloads as W
import riemann_exact

O = oracle


# ---------------------------------------------------------------- smooth orders
def test_linadv_translation_order_N3():
    # Sec. 5.1.1 / C1: u_t + u_x = 0 on periodic [0,1]; exact solution is a translation
    errs = []
    ns = [25, 50, 100]
    for nx in ns:
        cfg = O.RefConfig.make(O.LINADV1D, 3, nx, cfl=cfl_for(3, system=False))
        u0 = W.linadv_modes(1, nx, 3)
        u, nsteps, _ = run(cfg, u0, 1.0)
        ex = W.linadv_modes(1, nx, 3, t=1.0)
        errs.append(l1_error_1d(u.reshape(1, nx, 4), ex.reshape(1, nx, 4), 3, 1.0 / nx, 1.0)[0])
    eoc = np.log(np.array(errs[:-1]) / np.array(errs[1:])) / np.log(2.0)
    assert errs[-1] < 1e-6
    assert np.all(eoc >= 3.8), (errs, eoc)


@pytest.mark.parametrize("N", [1, 2])
def test_linadv_orders_low_degree(N):
    errs = []
    for nx in [20, 40, 80]:
        cfg = O.RefConfig.make(O.LINADV1D, N, nx, cfl=cfl_for(N, system=False))
        u, _, _ = run(cfg, W.linadv_modes(2, nx, N), 0.5)
        ex = W.linadv_modes(2, nx, N, t=0.5)
        errs.append(l1_error_1d(u.reshape(1, nx, N + 1), ex.reshape(1, nx, N + 1), N, 1.0 / nx, 1.0)[0])
    eoc = np.log(errs[0] / errs[1]) / np.log(2), np.log(errs[1] / errs[2]) / np.log(2)
    assert min(eoc) >= N + 1 - 0.25, (errs, eoc)


@pytest.mark.slow
@pytest.mark.parametrize("N,grids,min_eoc", [(2, (64, 128), 2.65), (3, (32, 64), 3.8)])
def test_vortex_order(N, grids, min_eoc):
    # Sec. 5.3.1: isentropic vortex, exact solution = translation.  N = 2 is
    # still pre-asymptotic here (EOC 2.72 at 64->128, 2.82 at 128->256).
    dom = (-5.0, 5.0, -5.0, 5.0)
    errs = []
    for n in grids:
        cfg = O.RefConfig.make(O.EULER2D, N, n, n, domain=dom, cfl=cfl_for(N))
        u0 = W.vortex2d(n, N, 0.0, dom)
        u, _, _ = run(cfg, u0, 0.5)
        ex = W.vortex2d(n, N, 0.5, dom)
        h = 10.0 / n
        errs.append(l1_error_2d(u, ex, N, h, h, 100.0)[0])
    eoc = np.log(errs[0] / errs[1]) / np.log(2)
    assert eoc >= min_eoc, (errs, eoc)


def test_vortex_indicator_does_not_activate():
    # Sec. 5.3.1: the limiter does not activate on a resolved vortex
    dom = (-5.0, 5.0, -5.0, 5.0)
    n, N = 64, 3
    cfg = O.RefConfig.make(O.EULER2D, N, n, n, domain=dom, cfl=cfl_for(N), blend=O.BLEND_MH,
                           flux_limiter=1, scaling=1)
    u0 = W.vortex2d(n, N, 0.0, dom)
    dt = O.compute_dt(cfg, u0)
    u1, alpha, d, st = O.step(cfg, u0, dt)
    assert st == 0
    assert np.all(alpha == 0.0)
    assert d["n_flux_limited"] == 0 and d["n_scaled"] == 0
    # with no active limiter the result equals the unlimited scheme
    cfg0 = O.RefConfig.make(O.EULER2D, N, n, n, domain=dom, cfl=cfl_for(N))
    u2, _, _, _ = O.step(cfg0, u0, dt)
    assert np.array_equal(u1, u2)


# ---------------------------------------------------------------- conservation
def _total(cfg, u):
    return O.means(cfg, u).sum(axis=(1, 2))


@pytest.mark.parametrize("blend,lim", [(O.BLEND_OFF, 0), (O.BLEND_MH, 1), (O.BLEND_FO, 1)])
def test_conservation_euler2d_periodic(blend, lim):
    # eq. upmean: sum of element means is conserved on a periodic grid
    n, N = 12, 3
    cfg = O.RefConfig.make(O.EULER2D, N, n, n, cfl=cfl_for(N), blend=blend, flux_limiter=lim, scaling=lim)
    u = W.euler2d_smooth_periodic(4, n, N, amp=0.4)
    if blend != O.BLEND_OFF:
        u = W.euler2d_quadrants(5, n, N)   # jumps; periodic wrap adds more jumps
    m0 = _total(cfg, u)
    u, _, diags = run(cfg, u, 10.0, max_steps=20)
    m1 = _total(cfg, u)
    assert np.all(np.abs(m1 - m0) <= 1e-13 * np.abs(m0).max() * 10), (m0, m1)


def test_conservation_tenmom_with_random_alpha():
    n, N = 10, 2
    cfg = O.RefConfig.make(O.TENMOM2D, N, n, n, cfl=cfl_for(N), blend=O.BLEND_MH, flux_limiter=1,
                           scaling=1, indicator=O.IND_GIVEN)
    u = W.tenmom2d_quadrants(3, n, n, N, dom=(0, 1, 0, 1))
    rng = np.random.default_rng(0)
    m0 = _total(cfg, u)
    for _ in range(5):
        dt = O.compute_dt(cfg, u)
        u, _, d, st = O.step(cfg, u, dt, alpha_given=rng.uniform(0, 1, n * n))
        assert st == 0
    assert np.allclose(_total(cfg, u), m0, atol=1e-13, rtol=0)


# ---------------------------------------------------------------- equal means (P-8)
@pytest.mark.parametrize("eq", [O.EULER1D, O.EULER2D])
def test_blended_mean_independent_of_element_alpha(eq):
    # eqs. low.order.cell.avg.update / blended.cell.avg.update: for the same
    # face fluxes, low-order, high-order and blended means coincide.  A
    # checkerboard change of alpha_e keeps every face average, hence every F.
    N = 3
    if eq == O.EULER1D:
        nx, ny = 16, 1
        u = W.euler1d_riemann(2, nx, N)
        chk = (-1.0) ** np.arange(nx)
    else:
        nx = ny = 8
        u = W.euler2d_quadrants(2, nx, N)
        chk = ((-1.0) ** (np.arange(ny)[:, None] + np.arange(nx)[None, :])).ravel()
    cfg = O.RefConfig.make(eq, N, nx, ny, cfl=cfl_for(N), blend=O.BLEND_MH, indicator=O.IND_GIVEN,
                           bc=(O.PERIODIC,) * 4)
    rng = np.random.default_rng(1)
    a1 = rng.uniform(0.3, 0.7, nx * ny)
    a2 = a1 + 0.25 * chk
    dt = O.compute_dt(cfg, u)
    u1, _, _, _ = O.step(cfg, u, dt, alpha_given=a1)
    u2, _, _, _ = O.step(cfg, u, dt, alpha_given=a2)
    assert np.abs(u1 - u2).max() > 1e-6          # nodal values do differ
    m1, m2 = O.means(cfg, u1), O.means(cfg, u2)
    assert np.allclose(m1, m2, atol=1e-13, rtol=0)


# ---------------------------------------------------------------- admissibility (P-9, P-5)
def _random_hard_euler2d(seed, n, N):
    rng = np.random.default_rng(seed)
    st = [(rng.uniform(0.05, 2.0), rng.uniform(-3, 3), rng.uniform(-3, 3), 10 ** rng.uniform(-4, 1))
          for _ in range(4)]
    return W.euler2d_quadrants(seed, n, N, states=st)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("blend", [O.BLEND_FO, O.BLEND_MH])
def test_theorem1_admissible_means_and_nodes(seed, blend):
    # Theorem 1 + scaling: means admissible after the flux limiter, every node
    # admissible after scaling, for random alpha fields and hard data
    n, N = 10, 3
    cfg = O.RefConfig.make(O.EULER2D, N, n, n, cfl=cfl_for(N), blend=blend, flux_limiter=1, scaling=1,
                           indicator=O.IND_GIVEN, bc=(O.FARFIELD,) * 4)
    u = _random_hard_euler2d(seed, n, N)
    ghost = O.boundary_traces(cfg, u)
    rng = np.random.default_rng(seed)
    _, w = O.gl(N)
    for _ in range(4):
        # Theorem 1 assumes an admissible low-order scheme: keep the subcell
        # Courant number of the nodal Rusanov speeds below 1/2
        sx = np.zeros(u.shape[1:]); sy = np.zeros(u.shape[1:])
        for idx in np.ndindex(*u.shape[1:]):
            sx[idx], sy[idx] = O.sigma(O.EULER2D, u[(slice(None),) + idx])
        dt = min(O.compute_dt(cfg, u), 0.5 * w.min() / (n * (sx + sy)).max())
        u, _, d, st = O.step(cfg, u, dt, alpha_given=rng.uniform(0, 1, n * n), ghost=ghost)
        assert st == 0 and d["n_mean_inadmissible"] == 0, d
        ub = O.means(cfg, u)
        assert ub[0].min() > 0
        pbar = 0.4 * (ub[3] - 0.5 * (ub[1] ** 2 + ub[2] ** 2) / ub[0])
        assert pbar.min() > 0
        rho = u[0]
        p = 0.4 * (u[3] - 0.5 * (u[1] ** 2 + u[2] ** 2) / u[0])
        assert rho.min() > 0 and p.min() > 0


def test_flux_limiter_inactive_when_admissible():
    n, N = 12, 3
    cfg = O.RefConfig.make(O.EULER2D, N, n, n, cfl=cfl_for(N), blend=O.BLEND_MH, flux_limiter=1, scaling=1,
                           indicator=O.IND_CONST, alpha_const=0.5)
    u = W.euler2d_smooth_periodic(0, n, N, amp=0.1)
    _, _, d, _ = O.step(cfg, u, O.compute_dt(cfg, u))
    assert d["n_flux_limited"] == 0 and d["min_theta_flux"] == 1.0


def test_without_positivity_fixes_pressure_goes_negative():
    # the admissibility corrections are needed (Sec. 5.2): a strong blast with
    # the limiters off produces a negative pressure; with them on it does not
    n, N = 40, 3
    x = W.node_coords_1d(n, N, -1, 1)
    rho = np.ones_like(x)
    p = np.where(np.abs(x) < 0.05, 1e3, 1e-6)
    u0 = W.euler1d_cons(rho, np.zeros_like(x), p)
    def neg_p(u):
        return (0.4 * (u[2] - 0.5 * u[1] ** 2 / u[0])).min() < 0 or u[0].min() < 0
    bad = False
    cfg = O.RefConfig.make(O.EULER1D, N, n, domain=(-1, 1, 0, 1), cfl=cfl_for(N), bc=(O.OUTFLOW,) * 4)
    u = u0.copy()
    for _ in range(10):
        dt = O.compute_dt(cfg, u)
        u, _, _, _ = O.step(cfg, u, dt)
        if neg_p(u):
            bad = True
            break
    assert bad
    cfg = O.RefConfig.make(O.EULER1D, N, n, domain=(-1, 1, 0, 1), cfl=cfl_for(N), bc=(O.OUTFLOW,) * 4,
                           blend=O.BLEND_MH, flux_limiter=1, scaling=1)
    u = u0.copy()
    for _ in range(30):
        dt = O.compute_dt(cfg, u)
        u, _, d, st = O.step(cfg, u, dt)
        assert st == 0 and not neg_p(u)


@pytest.mark.parametrize("seed", range(6))
def test_scaling_limiter_element(seed):
    # Zhang-Shu scaling: mean unchanged, P_k >= eps after, theta = 1 if admissible,
    # and the pressure root agrees with the closed-form root of the quadratic
    rng = np.random.default_rng(seed)
    N = 3
    cfg = O.RefConfig.make(O.EULER2D, N, 1, 1, scaling=1)
    _, w = O.gl(N)
    W2 = np.outer(w, w).ravel()
    rho = rng.uniform(0.5, 1.5, 16)
    v1, v2 = rng.uniform(-1, 1, 16), rng.uniform(-1, 1, 16)
    p = rng.uniform(0.5, 1.5, 16)
    p[rng.integers(0, 16)] = -0.3                       # one bad node
    ue = W.euler2d_cons(rho, v1, v2, p)
    ubar = ue @ W2
    out, th, bad = O.scale_element(cfg, ue)
    assert not bad and 0 < th < 1
    assert np.allclose(out @ W2, ubar, atol=1e-14)
    pn = 0.4 * (out[3] - 0.5 * (out[1] ** 2 + out[2] ** 2) / out[0])
    pbar = 0.4 * (ubar[3] - 0.5 * (ubar[1] ** 2 + ubar[2] ** 2) / ubar[0])
    eps = min(1e-13, pbar)
    assert pn.min() >= eps * (1 - 1e-9)
    # closed form: rho p(t) = 0.4 (rho E - |m|^2/2) along ubar + t (u - ubar) is quadratic
    tmin = 1.0
    for k in range(16):
        d = ue[:, k] - ubar
        # rho(t) (E(t) - eps/0.4) - |m(t)|^2/2 = A t^2 + B t + C
        r0, r1 = ubar[0], d[0]
        E0, E1 = ubar[3] - eps / 0.4, d[3]
        A = r1 * E1 - 0.5 * (d[1] ** 2 + d[2] ** 2)
        B = r0 * E1 + r1 * E0 - (ubar[1] * d[1] + ubar[2] * d[2])
        C = r0 * E0 - 0.5 * (ubar[1] ** 2 + ubar[2] ** 2)
        if A * 1 + B + C >= 0:   # node already admissible
            continue
        roots = np.roots([A, B, C])
        roots = roots[np.isreal(roots)].real
        roots = roots[(roots >= 0) & (roots <= 1)]
        tmin = min(tmin, roots.min())
    assert abs(th - tmin) < 1e-12
    ok = W.euler2d_cons(rho, v1, v2, np.abs(p) + 0.1)
    out2, th2, _ = O.scale_element(cfg, ok)
    assert th2 == 1.0 and np.array_equal(out2, ok)


# ---------------------------------------------------------------- CFL (P-6)
@pytest.mark.parametrize("N", [1, 2, 3])
def test_cfl_stability_brute_force(N):
    nx = 10
    cfl = cfl_for(N, system=False)
    u0 = W.linadv_modes(3, nx, N) + 1e-3 * np.random.default_rng(0).standard_normal((1, nx, N + 1))
    cfg = O.RefConfig.make(O.LINADV1D, N, nx, cfl=cfl)
    dx = 1.0 / nx
    for fac, stable in ((0.98, True), (1.1, False)):
        u = u0.copy()
        for _ in range(4000):
            u, _, _, _ = O.step(cfg, u, fac * cfl * dx)
        grown = not np.isfinite(u).all() or np.abs(u).max() > 10 * np.abs(u0).max()
        assert grown != stable, (N, fac, np.abs(u).max())


def test_cfl_values_close_to_published_lw_table():
    # cross-check only: CFL numbers recalled from the LWFR D2/Radau table the
    # paper refers to (0.333, 0.170, 0.103, 0.069 for N = 1..4)
    for N, ref in ((1, 0.333), (2, 0.170), (3, 0.103), (4, 0.069)):
        assert abs(cfl_for(N, system=False) - ref) < 2e-3


@pytest.mark.parametrize("N", [2, 3, 4])
def test_system_cfl_stable_and_upwind_cfl_unstable_for_euler(N):
    # With the Rusanov speed above the speed of the slow fields the upwind
    # CFL is unstable for a system; the all-ratio CFL (2/((N+1)(N+2))) is not.
    nx = 16
    x = W.node_coords_1d(nx, N, 0, 1)
    u0 = W.euler1d_cons(np.full(x.shape, 0.275), np.full(x.shape, 3.0), np.full(x.shape, 1.484))
    noise = 1e-10 * np.random.default_rng(0).standard_normal(u0.shape)
    assert abs(cfl_for(N) - 2.0 / ((N + 1) * (N + 2))) < 1e-5
    for cfl, stable in ((cfl_for(N), True), (cfl_for(N, system=False), False)):
        cfg = O.RefConfig.make(O.EULER1D, N, nx, cfl=cfl)
        u = u0 + noise
        for _ in range(600):
            u, _, _, _ = O.step(cfg, u, O.compute_dt(cfg, u))
        grown = not np.isfinite(u).all() or np.abs(u - u0).max() > 1e2 * np.abs(noise).max()
        assert grown != stable, (N, cfl, np.abs(u - u0).max())


# ---------------------------------------------------------------- first-order limit (P-11)
def _fv_rusanov_nonuniform_1d(u, N, dx, dt, gamma=1.4):
    """Independent first-order Rusanov finite volumes on the GL subcell grid of a
    periodic 1D Euler mesh: cell widths w_p dx, outflow-free periodic wrap."""
    _, w = np.polynomial.legendre.leggauss(N + 1)
    w = 0.5 * w
    M, nx, nd = u.shape
    U = u.reshape(M, nx * nd)
    h = np.tile(w, nx) * dx

    def flux(q):
        r, m, E = q
        v = m / r
        p = (gamma - 1) * (E - 0.5 * m * v)
        return np.stack([m, m * v + p, (E + p) * v]), np.abs(v) + np.sqrt(gamma * p / r)

    L, R = U, np.roll(U, -1, axis=1)
    fL, sL = flux(L)
    fR, sR = flux(R)
    lam = np.maximum(sL, sR)
    Fh = 0.5 * (fL + fR) - 0.5 * lam * (R - L)         # flux at the right face of each cell
    Un = U - dt / h * (Fh - np.roll(Fh, 1, axis=1))
    return Un.reshape(M, nx, nd)


def test_alpha_one_first_order_equals_subcell_fv():
    N, nx = 3, 12
    cfg = O.RefConfig.make(O.EULER1D, N, nx, cfl=cfl_for(N), blend=O.BLEND_FO, indicator=O.IND_CONST,
                           alpha_const=1.0)
    u = W.euler1d_riemann(4, nx, N)
    dt = O.compute_dt(cfg, u)
    u1, _, _, _ = O.step(cfg, u, dt)
    ref = _fv_rusanov_nonuniform_1d(u.reshape(3, nx, N + 1), N, 1.0 / nx, dt)
    assert np.allclose(u1.reshape(3, nx, N + 1), ref, atol=1e-13, rtol=0)


def test_mh_translates_linear_data_exactly():
    # MUSCL-Hancock on subcells is exact for linear data under linear advection
    N, nx = 3, 10
    cfg = O.RefConfig.make(O.LINADV1D, N, nx, adv=0.7, blend=O.BLEND_MH, indicator=O.IND_CONST,
                           alpha_const=1.0, bc=(O.OUTFLOW,) * 4, cfl=cfl_for(N, system=False))
    x = W.node_coords_1d(nx, N, 0, 1)
    u = (2.0 + 3.0 * x)[None]
    dt = 0.5 * cfl_for(N, system=False) / nx
    u1, _, _, _ = O.step(cfg, u, dt)
    ex = (2.0 + 3.0 * (x - 0.7 * dt))[None]
    inner = slice(1, nx - 1)
    assert np.allclose(u1.reshape(1, nx, N + 1)[:, inner], ex[:, inner], atol=1e-13)


# ---------------------------------------------------------------- Riemann vs exact (C2)
@pytest.mark.slow
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_euler1d_riemann_converges_to_exact(seed):
    # C2 analogue: L1 error of the density against the exact Riemann solution
    N, t_end = 4, 0.05
    errs = []
    for nx in [100, 200, 400]:
        cfg = O.RefConfig.make(O.EULER1D, N, nx, cfl=cfl_for(N), blend=O.BLEND_MH, flux_limiter=1, scaling=1,
                               bc=(O.FARFIELD,) * 4)
        u, _, diags = run(cfg, W.euler1d_riemann(seed, nx, N), t_end)
        assert all(d["n_mean_inadmissible"] == 0 for d in diags)
        L, R = W.riemann_states_1d(seed)
        x = W.node_coords_1d(nx, N, 0, 1)
        rex = riemann_exact.density_profile(L, R, x, t_end, x0=0.5 + W.OFF_FACE / nx)
        _, w = O.gl(N)
        errs.append((np.abs(u[0] - rex) * w).sum() / nx)
    rate = np.log2(errs[0] / errs[2]) / 2
    assert errs[0] > errs[1] > errs[2] and rate > 0.45, (errs, rate)


# ---------------------------------------------------------------- source ODE limit (P-13)
def test_source_uniform_state_linear_potential_exact():
    # App. B: with a uniform state and a linear potential W = gx x + gy y the
    # system is the ODE rho' = 0, m' = -rho grad W / 2, E' = -(v grad W) terms;
    # its solution is a polynomial of degree 2 in t, reproduced by cRK44.
    n, N = 4, 3
    gx, gy = 0.7, -0.4
    cfg = O.RefConfig.make(O.TENMOM2D, N, n, n, cfl=cfl_for(N), source=1, src_lin=(gx, gy))
    rho, v1, v2, p11, p12, p22 = 1.3, 0.2, -0.1, 1.0, 0.2, 0.8
    shape = (n, n, N + 1, N + 1)
    u = W.tenmom_cons(*(np.full(shape, x) for x in (rho, v1, v2, p11, p12, p22)))
    dt, steps = 0.01, 7
    for _ in range(steps):
        u, _, _, _ = O.step(cfg, u, dt)
    t = dt * steps
    m1 = rho * v1 - 0.5 * rho * gx * t
    m2 = rho * v2 - 0.5 * rho * gy * t
    E11 = 0.5 * p11 + 0.5 * rho * v1 ** 2 - 0.5 * gx * (rho * v1 * t - 0.25 * rho * gx * t ** 2)
    E22 = 0.5 * p22 + 0.5 * rho * v2 ** 2 - 0.5 * gy * (rho * v2 * t - 0.25 * rho * gy * t ** 2)
    E12 = (0.5 * p12 + 0.5 * rho * v1 * v2
           - 0.25 * gx * (rho * v2 * t - 0.25 * rho * gy * t ** 2)
           - 0.25 * gy * (rho * v1 * t - 0.25 * rho * gx * t ** 2))
    ex = [rho, m1, m2, E11, E12, E22]
    for v in range(6):
        assert np.allclose(u[v], ex[v], atol=1e-13, rtol=0), v


# ---------------------------------------------------------------- indicator
def test_indicator_modal_energy_shells():
    # energies of orthonormal Legendre modes land in shell max(i, j)
    N = 3
    xi, _ = O.gl(N)
    L = O.legendre_orthonormal(N, xi)
    cfg = O.RefConfig.make(O.EULER2D, N, 1, 1)
    for (i, j) in [(0, 0), (2, 1), (1, 3), (3, 3)]:
        eps = 5.0 + np.outer(L[j], L[i]).ravel()        # [q][p]: L_i(xi_p) L_j(xi_q)
        rho = np.ones(16)
        p = eps / rho
        ue = W.euler2d_cons(rho, np.zeros(16), np.zeros(16), p)
        a, e = O.indicator_raw(cfg, ue)
        expect = np.zeros(N + 1)
        expect[0] += 25.0
        expect[max(i, j)] += 1.0 if (i, j) != (0, 0) else 0.0
        if (i, j) == (0, 0):
            expect[0] = 36.0
        assert np.allclose(e, expect, atol=1e-12), (i, j, e)
    # smooth constant data: alpha = 0; a pure top mode: alpha = alpha_max
    ue = W.euler2d_cons(np.ones(16), np.zeros(16), np.zeros(16), np.ones(16))
    assert O.indicator_raw(cfg, ue)[0] == 0.0
    eps = 0.01 + np.outer(L[3], L[3]).ravel()
    ue = W.euler2d_cons(np.ones(16), np.zeros(16), np.zeros(16), eps)
    assert O.indicator_raw(cfg, ue)[0] == 1.0


# ---------------------------------------------------------------- MLP backprop (P-14)
def test_mlp_gradient_matches_finite_differences():
    dims = [5, 8, 6, 1]
    rng = np.random.default_rng(0)
    npar = sum(dims[i + 1] * dims[i] + dims[i + 1] for i in range(3))
    params = 0.5 * rng.standard_normal(npar)
    x = rng.standard_normal((7, 5))
    t = rng.uniform(0, 1, 7)
    loss, g = O.mlp_loss_grad(dims, params, x, t)
    h = 1e-6
    for k in range(npar):
        pp, pm = params.copy(), params.copy()
        pp[k] += h
        pm[k] -= h
        fd = (O.mlp_loss_grad(dims, pp, x, t)[0] - O.mlp_loss_grad(dims, pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-8 * max(1.0, abs(fd)), k
    y = O.mlp_forward(dims, params, x)
    assert abs(np.mean((y - t) ** 2) - loss) < 1e-15
