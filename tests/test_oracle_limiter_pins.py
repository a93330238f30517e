"""Hand-computed pins of three parts of the oracle's limiter chain (Sec. 4):

1. the smoothness indicator's logistic transition (the Hennemann et al.
   indicator the paper refers to): threshold T(N) = 0.5 10^(-1.8 (N+1)^(1/4))
   and slope ln(9999)/T, which put alpha at 1/2 where the energy ratio E
   equals T, at 0.9999 where E = 2T and at 1/(1 + sqrt(9999)) where E = T/2;
2. the flux limiter for admissibility in means (Sec. 4.3): candidates of the
   low-order update (eq. low.order.update) of the two face-adjacent
   subcells, eps = 0.1 P_k of the low-order candidate, the concavity bound
   for theta and the direction share of the 2D update;
3. the MUSCL-Hancock predictor on the Gauss-Legendre subcells (Sec. 4.2):
   minmod slopes on the non-uniform subcell grid, slope scaling that keeps
   the reconstructed face values at P_k >= 0.1 P_k(u_p), the Hancock half
   step and the zero-slope fallback.

Each expected value is computed here from those definitions with numpy
(independent Gauss-Legendre rule, Legendre polynomials and fluxes), so a
changed exponent, slope, epsilon fraction, candidate factor or scaling in
the oracle fails one of them."""
import math

import numpy as np
import pytest

import oracle as O

GAMMA = 1.4


def gl01(N):
    x, w = np.polynomial.legendre.leggauss(N + 1)
    return 0.5 * (x + 1.0), 0.5 * w


def legendre_on01(k, x):
    """orthonormal Legendre polynomial of degree k on [0, 1]"""
    c = np.zeros(k + 1)
    c[k] = 1.0
    return math.sqrt(2 * k + 1) * np.polynomial.legendre.legval(2.0 * np.asarray(x) - 1.0, c)


def threshold(N):
    return 0.5 * 10.0 ** (-1.8 * (N + 1) ** 0.25)


# ---------------------------------------------------------------- 1. indicator transition
# energy ratio as a multiple of T, and the alpha the logistic's design fixes
TRANSITION = [(1.0, 0.5), (2.0, 9999.0 / 10000.0), (0.5, 1.0 / (1.0 + math.sqrt(9999.0))),
              (1.5, 1.0 / (1.0 + 9999.0 ** -0.5))]


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("ratio,alpha", TRANSITION)
def test_indicator_transition_1d(N, ratio, alpha):
    # linear advection: the indicator quantity is u; u = 1 + a L_N has e_N / (e_0 + e_N) = a^2 / (1 + a^2)
    E = ratio * threshold(N)
    a = math.sqrt(E / (1.0 - E))
    xi, _ = gl01(N)
    ue = 1.0 + a * legendre_on01(N, xi)
    cfg = O.RefConfig.make(O.LINADV1D, N, 4, blend=O.BLEND_MH)
    got, en = O.indicator_raw(cfg, ue)
    assert en[N] / en.sum() == pytest.approx(E, rel=1e-12)
    assert got == pytest.approx(alpha, rel=1e-9, abs=1e-12)


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("ratio,alpha", TRANSITION)
@pytest.mark.parametrize("shell", ["N", "N-1"])
def test_indicator_transition_2d_euler(N, ratio, alpha, shell):
    # 2D Euler at rest with rho = 1: the quantity rho p = p.  One tensor mode
    # (N, 0) puts the energy into shell N (the first ratio of E); the mode
    # (N-1, N-1) puts it into shell N-1 (the second ratio)
    E = ratio * threshold(N)
    a = math.sqrt(E / (1.0 - E))
    xi, _ = gl01(N)
    X, Y = np.meshgrid(xi, xi)          # [q][p]: p the x index
    if shell == "N":
        p = 1.0 + a * legendre_on01(N, X)
    else:
        p = 1.0 + a * legendre_on01(N - 1, X) * legendre_on01(N - 1, Y)
    assert p.min() > 0.0
    np_ = (N + 1) ** 2
    ue = np.zeros((4, np_))
    ue[0] = 1.0
    ue[3] = p.reshape(-1) / (GAMMA - 1.0)
    cfg = O.RefConfig.make(O.EULER2D, N, 4, 4, blend=O.BLEND_MH)
    got, en = O.indicator_raw(cfg, ue.reshape(-1))
    k = N if shell == "N" else N - 1
    assert en[k] / en[: k + 1].sum() == pytest.approx(E, rel=1e-10)
    assert got == pytest.approx(alpha, rel=1e-8, abs=1e-12)


@pytest.mark.parametrize("N", [2, 3, 4])
def test_indicator_below_alpha_min_is_zero(N):
    # at E = 0 the logistic gives 1/(1 + 9999) = 1e-4 < alpha_min = 1e-3: alpha = 0;
    # at E = 0.75 T it gives 1/(1 + 9999^(1/4)) = 0.0909..., above alpha_min
    xi, _ = gl01(N)
    cfg = O.RefConfig.make(O.LINADV1D, N, 4, blend=O.BLEND_MH)
    assert O.indicator_raw(cfg, np.full(N + 1, 2.0))[0] == 0.0
    E = 0.75 * threshold(N)
    ue = 1.0 + math.sqrt(E / (1.0 - E)) * legendre_on01(N, xi)
    assert O.indicator_raw(cfg, ue)[0] == pytest.approx(1.0 / (1.0 + 9999.0 ** 0.25), rel=1e-9)


# ---------------------------------------------------------------- 2. flux limiter
def euler_p(u):
    """pressure of 1D (rho, m, E) or 2D (rho, m1, m2, E) Euler states"""
    u = np.asarray(u, dtype=float)
    kin = 0.5 * (u[1:-1] ** 2).sum() / u[0]
    return (GAMMA - 1.0) * (u[-1] - kin)


def euler_c(u):
    return math.sqrt(GAMMA * euler_p(u) / u[0])


def limit_by_hand(F, fLO, dt, sides, frac=0.1):
    """The limiter of Sec. 4.3 written out: for density then pressure, the
    candidates u - k (F - adj) + dt S (side A, below the face) and
    u - k (adj - F) + dt S (side B) with F and with fLO; eps = 0.1 P(fLO
    candidate); where P(F candidate) < eps the concavity bound
    theta = (P_lo - eps) / (P_lo - P_F); F <- theta F + (1 - theta) fLO.
    Returns F and the theta of each constraint."""
    F = np.array(F, dtype=float)
    fLO = np.asarray(fLO, dtype=float)
    thetas = []
    for P in (lambda u: u[0], euler_p):
        th = 1.0
        for side, (u, adj, S, k) in sides.items():
            sgn = 1.0 if side == "A" else -1.0
            cand = lambda G: np.asarray(u) - k * sgn * (G - np.asarray(adj)) + dt * np.asarray(S)
            Plo, PF = P(cand(fLO)), P(cand(F))
            eps = frac * Plo
            if PF < eps:
                th = min(th, (Plo - eps) / (Plo - PF))
        F = th * F + (1.0 - th) * fLO
        thetas.append(th)
    return F, thetas


def test_flux_limiter_1d_face_by_hand():
    # subcells: A (rho 1, p 1), B (rho 0.125, p 0.1); adjacent subface fluxes
    # equal to fLO, so the fLO candidates are the subcell states themselves
    uA = np.array([1.0, 0.0, 2.5])
    uB = np.array([0.125, 0.0, 0.25])
    fLO = np.array([0.3, 0.5, 0.9])
    F = fLO + np.array([-0.2, 0.05, -0.5])
    kA, kB, dt = 0.7, 1.0, 0.01
    z = np.zeros(3)
    sides = {"A": (uA, fLO, z, kA), "B": (uB, fLO, z, kB)}
    Fh, (th_rho, th_p) = limit_by_hand(F, fLO, dt, sides)
    # side B's density candidate 0.125 - 0.2 falls below 0.0125: theta = 0.1125 / 0.2
    assert th_rho == pytest.approx(0.5625, rel=1e-14)
    assert 0.0 < th_p < 1.0
    cfg = O.RefConfig.make(O.EULER1D, 3, 8)
    Fo, th, bad = O.flux_limit_face(cfg, F, fLO, dt, A=(uA, fLO, z, kA), B=(uB, fLO, z, kB))
    assert not bad
    np.testing.assert_allclose(Fo, Fh, rtol=1e-14, atol=1e-15)
    assert th == pytest.approx(min(th_rho, th_p), rel=1e-14)
    # after the density pass the density bound is attained exactly (no over-limiting)
    F1 = th_rho * F + (1.0 - th_rho) * fLO
    assert uB[0] + kB * (F1[0] - fLO[0]) == pytest.approx(0.1 * uB[0], rel=1e-13)


@pytest.mark.parametrize("frac", [0.05, 0.3])
def test_flux_limiter_margin_option(frac):
    # eps_rel of the limiter options replaces the 0.1 of eps = 0.1 P(fLO candidate)
    uA = np.array([1.0, 0.0, 2.5])
    uB = np.array([0.125, 0.0, 0.25])
    fLO = np.array([0.3, 0.5, 0.9])
    F = fLO + np.array([-0.2, 0.05, -0.5])
    z = np.zeros(3)
    sides = {"A": (uA, fLO, z, 0.7), "B": (uB, fLO, z, 1.0)}
    Fh, ths = limit_by_hand(F, fLO, 0.01, sides, frac=frac)
    assert 0.0 < ths[0] < 1.0
    cfg = O.RefConfig.make(O.EULER1D, 3, 8, eps_rel=frac)
    Fo, th, bad = O.flux_limit_face(cfg, F, fLO, 0.01, A=sides["A"], B=sides["B"])
    np.testing.assert_allclose(Fo, Fh, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("floor", [1e-3, 2e-2])
@pytest.mark.parametrize("which", ["rho", "p"])
def test_scaling_floor_option(floor, which):
    # Zhang-Shu scaling with eps = min(eps_abs, P(mean)): a node below the floor
    # ends exactly at it for the density (linear in the scaling factor), and at
    # it within the bisection's resolution for the pressure; the mean is kept
    N = 3
    xi, w = gl01(N)
    rho = np.array([1.0, 0.5, 1e-5 if which == "rho" else 0.7, 1.2])
    p = np.array([1.0, 1e-6 if which == "p" else 0.6, 0.8, 0.9])
    v = np.array([0.1, -0.3, 0.2, 0.0])
    ue = np.stack([rho, rho * v, p / 0.4 + 0.5 * rho * v * v]).reshape(-1)
    cfg = O.RefConfig.make(O.EULER1D, N, 4, scaling=1, eps_abs=floor)
    out, th, bad = O.scale_element(cfg, ue)
    assert not bad and 0.0 < th < 1.0
    o = out.reshape(3, N + 1)
    if which == "rho":
        assert o[0].min() == pytest.approx(floor, rel=1e-12)
    else:
        pmin = min(euler_p(o[:, k]) for k in range(N + 1))
        assert floor * (1 - 1e-9) <= pmin <= floor * (1 + 1e-9)
    np.testing.assert_allclose((o * w).sum(axis=1), (ue.reshape(3, N + 1) * w).sum(axis=1), rtol=1e-14)


def test_flux_limiter_1d_admissible_f_is_kept_and_missing_side():
    uA = np.array([1.0, 0.2, 2.5])
    fLO = np.array([0.3, 0.5, 0.9])
    F = fLO + np.array([0.01, -0.02, 0.03])
    cfg = O.RefConfig.make(O.EULER1D, 3, 8)
    z = np.zeros(3)
    Fo, th, bad = O.flux_limit_face(cfg, F, fLO, 0.01, A=(uA, fLO, z, 0.5))
    assert th == 1.0 and not bad
    np.testing.assert_array_equal(Fo, F)
    # one-sided (boundary) face: only side A's candidate constrains F
    F = fLO + np.array([2.0, 0.0, 0.0])
    Fh, ths = limit_by_hand(F, fLO, 0.01, {"A": (uA, fLO, z, 0.5)})
    Fo, th, bad = O.flux_limit_face(cfg, F, fLO, 0.01, A=(uA, fLO, z, 0.5))
    assert 0.0 < ths[0] < 1.0
    np.testing.assert_allclose(Fo, Fh, rtol=1e-14)


def test_flux_limiter_inadmissible_low_order_candidate():
    # a low-order candidate outside the admissible set: theta = 0, F = fLO, counted
    uA = np.array([0.01, 0.0, 0.025])
    fLO = np.array([0.3, 0.5, 0.9])
    cfg = O.RefConfig.make(O.EULER1D, 3, 8)
    z = np.zeros(3)
    Fo, th, bad = O.flux_limit_face(cfg, fLO + 0.1, fLO, 0.01, A=(uA, np.zeros(3), z, 1.0))
    assert bad and th == 0.0
    np.testing.assert_allclose(Fo, fLO, rtol=1e-15)


def test_lo_factor_by_hand():
    # eq. low.order.update of a face-adjacent subcell, split into directions
    # with shares phi_d proportional to sigma_d / (w h_d): the factor of the
    # flux difference across a face normal to d is dt / (w_i h_d phi_d)
    N, nx, ny = 3, 8, 5
    dom = (0.0, 2.0, 0.0, 1.5)
    dx, dy = 2.0 / nx, 1.5 / ny
    _, w = gl01(N)
    u = np.array([1.3, 0.4, -0.9, 3.1])
    v1, v2 = u[1] / u[0], u[2] / u[0]
    sx, sy = abs(v1) + euler_c(u), abs(v2) + euler_c(u)
    cfg = O.RefConfig.make(O.EULER2D, N, nx, ny, domain=dom)
    dt = 0.003
    for d in (0, 1):
        for t in range(N + 1):
            for i in (0, N):
                ax = sx / ((w[i] if d == 0 else w[t]) * dx)
                ay = sy / ((w[t] if d == 0 else w[i]) * dy)
                phi = (ax if d == 0 else ay) / (ax + ay)
                want = dt / (w[i] * (dx if d == 0 else dy) * phi)
                assert O.lo_factor(cfg, d, t, i, u, dt) == pytest.approx(want, rel=1e-14)
    cfg1 = O.RefConfig.make(O.EULER1D, N, nx, domain=dom)
    for i in (0, N):
        assert O.lo_factor(cfg1, 0, 0, i, u[[0, 1, 3]], dt) == pytest.approx(dt / (w[i] * dx), rel=1e-14)


def test_flux_limiter_2d_face_by_hand():
    # a y face: the candidate factors of the 2D low-order update, then density
    # and pressure limiting with both theta strictly inside (0, 1)
    N, n = 3, 16
    cfg = O.RefConfig.make(O.EULER2D, N, n, n)
    uA = np.array([0.9, 0.1, 0.3, 2.0])
    uB = np.array([0.2, 0.05, -0.02, 0.3])
    dt, t = 0.004, 2
    kA = O.lo_factor(cfg, 1, t, N, uA, dt)
    kB = O.lo_factor(cfg, 1, t, 0, uB, dt)
    fLO = np.array([0.05, 0.02, 0.4, 0.1])
    adjA = fLO + np.array([0.01, 0.0, 0.01, 0.02])
    adjB = fLO - np.array([0.01, 0.0, 0.0, 0.01])
    # F pulls side B's density below 0.1 of its low-order value, then its pressure
    delta = np.array([-0.2 / kB, 0.3 / kB, 0.0, -0.35 / kB])
    F = fLO + delta
    S = np.array([0.0, 0.0, -0.1, 0.0])
    sides = {"A": (uA, adjA, S, kA), "B": (uB, adjB, S, kB)}
    Fh, (th_rho, th_p) = limit_by_hand(F, fLO, dt, sides)
    assert 0.0 < th_rho < 1.0 and 0.0 < th_p < 1.0, (th_rho, th_p)
    Fo, th, bad = O.flux_limit_face(cfg, F, fLO, dt, A=(uA, adjA, S, kA), B=(uB, adjB, S, kB))
    assert not bad
    np.testing.assert_allclose(Fo, Fh, rtol=1e-13, atol=1e-15)
    assert th == pytest.approx(min(th_rho, th_p), rel=1e-13)


# ---------------------------------------------------------------- 3. MUSCL-Hancock predictor
def euler1d_flux(u):
    v = u[1] / u[0]
    p = euler_p(u)
    return np.array([u[1], u[1] * v + p, (u[2] + p) * v])


def mh_by_hand(u, e, N, dx, dt):
    """Predicted face values of the subcells of element e of a periodic 1D
    Euler grid u[var][elem][node]: reference positions of the GL points,
    subfaces at the cumulative weights, minmod slopes across neighbours
    (the neighbour elements' points across the faces), slope scaled so that
    both face values keep rho, p >= 0.1 of the subcell's (concavity bound
    per constraint), Hancock half step, zero slope when a predicted value
    breaks the same bounds.  Returns xm, xp [node][var] and the counts."""
    xi, w = gl01(N)
    sub = np.concatenate([[0.0], np.cumsum(w)])
    sub[-1] = 1.0
    ne = u.shape[1]
    P = [lambda s: s[0], euler_p]
    xm, xp = np.zeros((N + 1, 3)), np.zeros((N + 1, 3))
    nlim = nfb = 0
    for p in range(N + 1):
        up_ = u[:, e, p]
        if p > 0:
            um, xleft = u[:, e, p - 1], xi[p - 1]
        else:
            um, xleft = u[:, (e - 1) % ne, N], xi[N] - 1.0
        if p < N:
            un, xright = u[:, e, p + 1], xi[p + 1]
        else:
            un, xright = u[:, (e + 1) % ne, 0], 1.0 + xi[0]
        s1 = (up_ - um) / (xi[p] - xleft)
        s2 = (un - up_) / (xright - xi[p])
        s = np.where(s1 * s2 <= 0.0, 0.0, np.where(np.abs(s1) < np.abs(s2), s1, s2))
        hm, hp = sub[p] - xi[p], sub[p + 1] - xi[p]
        eps = [0.1 * Pk(up_) for Pk in P]
        for k, Pk in enumerate(P):
            th = 1.0
            for h in (hm, hp):
                Pf = Pk(up_ + s * h)
                if Pf < eps[k]:
                    th = min(th, (Pk(up_) - eps[k]) / (Pk(up_) - Pf))
            if th < 1.0:
                nlim += 1
                s = th * s
        fm, fp = up_ + s * hm, up_ + s * hp
        delta = -0.5 * dt * (euler1d_flux(fp) - euler1d_flux(fm)) / (w[p] * dx)
        a, b = fm + delta, fp + delta
        if all(Pk(v) >= eps[k] for v in (a, b) for k, Pk in enumerate(P)):
            xm[p], xp[p] = a, b
        else:
            nfb += 1
            xm[p], xp[p] = up_, up_
    return xm, xp, nlim, nfb


def mh_case():
    """Three elements, N = 3, density 1.  In element 1 the momentum rises
    steeply while the energy is flat over its first two nodes, so the
    reconstructed value at the right face of subcell 1 loses pressure."""
    N, ne = 3, 3
    u = np.zeros((3, ne, N + 1))
    u[0] = 1.0
    u[1] = [[0.0, 0.2, 0.5, 0.8], [1.0, 1.5, 2.0, 2.2], [2.0, 1.5, 1.0, 0.5]]
    u[2] = [[1.0, 1.0, 1.0, 1.2], [1.375, 1.375, 2.5, 2.9], [2.6, 2.0, 1.5, 1.2]]
    return N, ne, u


@pytest.mark.parametrize("dt,expect_fallback", [(1e-4, False), (0.3, True), (0.5, True)])
def test_mh_slope_scaling_and_fallback_by_hand(dt, expect_fallback):
    N, ne, u = mh_case()
    assert all(euler_p(u[:, e, k]) > 0 for e in range(ne) for k in range(N + 1))
    dx = 1.0 / ne
    cfg = O.RefConfig.make(O.EULER1D, N, ne, blend=O.BLEND_MH)
    for e in range(ne):
        xm_h, xp_h, nlim, nfb = mh_by_hand(u, e, N, dx, dt)
        (xm, xp, _, _), (cl, cf) = O.mh_predict(cfg, u.reshape(-1), e, 0, dt)
        np.testing.assert_allclose(xm, xm_h, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(xp, xp_h, rtol=1e-12, atol=1e-14)
        assert (cl, cf) == (nlim, nfb)
    # the case exercises both branches: some slope is scaled, and at the large
    # step some Hancock value falls back to the subcell state
    totals = [mh_by_hand(u, e, N, dx, dt)[2:] for e in range(ne)]
    assert sum(t[0] for t in totals) >= 1
    assert (sum(t[1] for t in totals) >= 1) == expect_fallback
