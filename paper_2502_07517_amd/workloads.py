"""Seeded synthetic inputs for the cRKFR step: initial conditions sampled at
the solution points (collocation), Gauss-Legendre by default.

This module holds no arithmetic of the method.  It only draws seeded problem
data and samples analytic initial conditions at node positions, which it takes
from numpy's Gauss-Legendre rule (Gauss-Legendre-Lobatto: the end points and
the roots of numpy's P_N').  Both the oracle tests and the HIP path read their
inputs from here.

Node layout of every returned array: ``u[var][ey][ex][q][p]`` (1D: ``u[var][ex][p]``),
p the x-node, q the y-node.
"""
import numpy as np

GAMMA = 1.4


def gl_nodes(N):
    """Gauss-Legendre nodes on [0, 1] from numpy's rule."""
    x, _ = np.polynomial.legendre.leggauss(N + 1)
    return 0.5 * (x + 1.0)


def gll_nodes(N):
    """Gauss-Legendre-Lobatto nodes on [0, 1]: 0, 1 and the roots of P_N'."""
    inner = np.sort(np.polynomial.legendre.Legendre.basis(N).deriv().roots().real) if N > 1 else np.zeros(0)
    return 0.5 * (np.concatenate([[-1.0], inner, [1.0]]) + 1.0)


def solution_nodes(N, points=0):
    return gll_nodes(N) if points == 1 else gl_nodes(N)


def node_coords_1d(nx, N, x0, x1, points=0):
    xi = solution_nodes(N, points)
    dx = (x1 - x0) / nx
    return x0 + (np.arange(nx)[:, None] + xi[None, :]) * dx          # [ex][p]


def node_coords_2d(nx, ny, N, dom, points=0):
    x0, x1, y0, y1 = dom
    xi = solution_nodes(N, points)
    dx, dy = (x1 - x0) / nx, (y1 - y0) / ny
    X = x0 + (np.arange(nx)[None, :, None, None] + xi[None, None, None, :]) * dx
    Y = y0 + (np.arange(ny)[:, None, None, None] + xi[None, None, :, None]) * dy
    shape = (ny, nx, N + 1, N + 1)
    return np.broadcast_to(X, shape).copy(), np.broadcast_to(Y, shape).copy()   # [ey][ex][q][p]


# ---------------------------------------------------------------- 1D scalar
def linadv_modes(seed, nx, N, t=0.0, adv=1.0):
    """u0 = sin(2 pi x) + sum_{k=1..4} a_k sin(2 pi k x + phi_k) on periodic [0,1],
    a_k ~ U[0, 0.1], phi_k ~ U[0, 2 pi); exact solution is u0(x - adv t)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 0.1, 4)
    ph = rng.uniform(0.0, 2.0 * np.pi, 4)
    x = node_coords_1d(nx, N, 0.0, 1.0) - adv * t
    u = np.sin(2 * np.pi * x)
    for k in range(4):
        u = u + a[k] * np.sin(2 * np.pi * (k + 1) * x + ph[k])
    return u[None].copy()


# ---------------------------------------------------------------- Euler helpers
def euler1d_cons(rho, v, p, gamma=GAMMA):
    return np.stack([rho, rho * v, p / (gamma - 1.0) + 0.5 * rho * v * v])


def euler2d_cons(rho, v1, v2, p, gamma=GAMMA):
    return np.stack([rho, rho * v1, rho * v2, p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2)])


def tenmom_cons(rho, v1, v2, p11, p12, p22):
    return np.stack([rho, rho * v1, rho * v2,
                     0.5 * p11 + 0.5 * rho * v1 * v1,
                     0.5 * p12 + 0.5 * rho * v1 * v2,
                     0.5 * p22 + 0.5 * rho * v2 * v2])


def riemann_states_1d(seed):
    """Left/right (rho, v, p) with rho ~ U[0.1,2], v ~ U[-1,1], p ~ U[0.1,2]."""
    rng = np.random.default_rng(seed)
    L = (rng.uniform(0.1, 2.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 2.0))
    R = (rng.uniform(0.1, 2.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 2.0))
    return L, R


# Discontinuities are placed 0.37 of an element off the element faces, so the
# smoothness indicator sees them at t = 0 (a jump on a face leaves every element
# constant and the first step unlimited).
OFF_FACE = 0.37


def euler1d_riemann(seed, nx, N, x0=0.0, x1=1.0, xs=None, gamma=GAMMA):
    """Seeded Riemann data, jump at xs (default: domain centre + 0.37 dx)."""
    if xs is None:
        xs = 0.5 * (x0 + x1) + OFF_FACE * (x1 - x0) / nx
    (rl, vl, pl), (rr, vr, pr) = riemann_states_1d(seed)
    x = node_coords_1d(nx, N, x0, x1)
    left = x < xs
    rho = np.where(left, rl, rr)
    v = np.where(left, vl, vr)
    p = np.where(left, pl, pr)
    return euler1d_cons(rho, v, p, gamma)


def euler1d_smooth(seed, nx, N, x0=0.0, x1=1.0, amp=0.3, gamma=GAMMA):
    """Periodic smooth Euler data: one sine mode with a seeded phase per field."""
    ph = np.random.default_rng(seed).uniform(0.0, 1.0, 3)
    x = (node_coords_1d(nx, N, x0, x1) - x0) / (x1 - x0)
    rho = 1.0 + amp * np.sin(2 * np.pi * (x + ph[0]))
    v = 0.5 + amp * np.sin(2 * np.pi * (x + ph[1]))
    p = 1.0 + amp * np.cos(2 * np.pi * (x + ph[2]))
    return euler1d_cons(rho, v, p, gamma)


def burgers_sine(nx, N, amp=0.2, x0=0.0, x1=2 * np.pi, shift=0.0, points=0):
    """Burgers data u0 = shift + amp sin(x) (the smooth Burgers test uses amp
    0.2 on [0, 2 pi]: smooth until t = 1/amp = 5)."""
    return (shift + amp * np.sin(node_coords_1d(nx, N, x0, x1, points)))[None].copy()


def blast1d(nx, N):
    """Woodward-Colella blast wave on [0, 1] (Sec. 5.2): p = 1000, 0.01, 100
    left of 0.1, between, right of 0.9; rho = 1, v = 0."""
    x = node_coords_1d(nx, N, 0.0, 1.0)
    p = np.where(x < 0.1, 1000.0, np.where(x > 0.9, 100.0, 0.01))
    return euler1d_cons(np.ones_like(x), np.zeros_like(x), p)


def sedov1d(nx, N, gamma=GAMMA):
    """1D Sedov blast on [-1, 1] (Sec. 5.2): rho = 1, v = 0, E = 3.2e6/dx in
    the element around x = 0 and 1e-12 elsewhere (nx odd)."""
    x = node_coords_1d(nx, N, -1.0, 1.0)
    dx = 2.0 / nx
    E = np.where(np.abs(x) <= dx / 2, 3.2e6 / dx, 1e-12)
    return np.stack([np.ones_like(x), np.zeros_like(x), E])


# ---------------------------------------------------------------- 2D Euler
def vortex_prim(X, Y, t=0.0, dom=(-5.0, 5.0, -5.0, 5.0), beta=5.0, mach=0.5,
                angle_deg=45.0, gamma=GAMMA):
    """Isentropic vortex (Sec. 5.3.1): exact solution at time t is the initial
    data translated by (u0, v0) t, wrapped periodically on the domain."""
    a = np.deg2rad(angle_deg)
    u0, v0 = mach * np.cos(a), mach * np.sin(a)
    x0, x1, y0, y1 = dom
    Lx, Ly = x1 - x0, y1 - y0
    xs = np.mod(X - u0 * t - x0, Lx) + x0
    ys = np.mod(Y - v0 * t - y0, Ly) + y0
    r2 = xs * xs + ys * ys
    rho = (1.0 - beta ** 2 * (gamma - 1.0) / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)) ** (1.0 / (gamma - 1.0))
    v1 = u0 - beta * ys / (2 * np.pi) * np.exp(0.5 * (1.0 - r2))
    v2 = v0 + beta * xs / (2 * np.pi) * np.exp(0.5 * (1.0 - r2))
    p = rho ** gamma
    return rho, v1, v2, p


def vortex2d(n, N, t=0.0, dom=(-5.0, 5.0, -5.0, 5.0), gamma=GAMMA):
    X, Y = node_coords_2d(n, n, N, dom)
    rho, v1, v2, p = vortex_prim(X, Y, t, dom, gamma=gamma)
    return euler2d_cons(rho, v1, v2, p, gamma)


def sedov2d(n, N, dom=(-1.5, 1.5, -1.5, 1.5), gamma=GAMMA):
    """2D Sedov test of Sec. 5.3 on a periodic square: gas at rest, Gaussian
    density and pressure bumps (sigma_rho 0.25, sigma_p 0.15) over rho0 = 1,
    p0 = 1e-5."""
    X, Y = node_coords_2d(n, n, N, dom)
    r2 = X * X + Y * Y
    sr, sp = 0.25, 0.15
    rho = 1.0 + np.exp(-r2 / (2 * sr * sr)) / (4 * np.pi * sr * sr)
    p = 1e-5 + (gamma - 1.0) * np.exp(-r2 / (2 * sp * sp)) / (4 * np.pi * sp * sp)
    z = np.zeros_like(X)
    return euler2d_cons(rho, z, z, p, gamma)


def quadrant_states_euler(seed, rho_rng=(0.1, 2.0), v_rng=(-1.0, 1.0), p_rng=(0.1, 2.0)):
    rng = np.random.default_rng(seed)
    return [(rng.uniform(*rho_rng), rng.uniform(*v_rng), rng.uniform(*v_rng), rng.uniform(*p_rng))
            for _ in range(4)]


def _quadrant_fill(X, Y, xs, ys, states):
    q = (X >= xs).astype(int) + 2 * (Y >= ys).astype(int)   # 0: SW, 1: SE, 2: NW, 3: NE
    cols = []
    for c in range(len(states[0])):
        vals = np.array([s[c] for s in states])
        cols.append(vals[q])
    return cols


def _split(dom, nx, ny, split):
    if split is not None:
        return split
    return (0.5 * (dom[0] + dom[1]) + OFF_FACE * (dom[1] - dom[0]) / nx,
            0.5 * (dom[2] + dom[3]) + OFF_FACE * (dom[3] - dom[2]) / ny)


def euler2d_quadrants(seed, n, N, dom=(0.0, 1.0, 0.0, 1.0), gamma=GAMMA, states=None, split=None):
    """Seeded 4-quadrant Riemann data, split lines at the domain centre + 0.37 h."""
    X, Y = node_coords_2d(n, n, N, dom)
    st = states if states is not None else quadrant_states_euler(seed)
    xs, ys = _split(dom, n, n, split)
    rho, v1, v2, p = _quadrant_fill(X, Y, xs, ys, st)
    return euler2d_cons(rho, v1, v2, p, gamma)


# Lax-Liu configuration 12 as printed in Sec. 5.3.2, ordered SW, SE, NW, NE
RIEMANN2D_CFG12 = [(0.8, 0.0, 0.0, 1.0), (1.0, 0.0, 0.7276, 1.0),
                   (1.0, 0.7276, 0.0, 1.0), (0.5313, 0.0, 0.0, 0.4)]


def euler2d_smooth_periodic(seed, n, N, dom=(0.0, 1.0, 0.0, 1.0), amp=0.2, gamma=GAMMA):
    """Smooth positive periodic data with seeded low Fourier modes."""
    rng = np.random.default_rng(seed)
    X, Y = node_coords_2d(n, n, N, dom)
    Lx, Ly = dom[1] - dom[0], dom[3] - dom[2]
    cols = []
    for base in (1.0, 0.3, -0.2, 1.0):
        f = np.full(X.shape, base)
        for _ in range(3):
            kx, ky = rng.integers(0, 3, 2)
            ph = rng.uniform(0, 2 * np.pi)
            f = f + amp * rng.uniform(0.2, 1.0) * np.sin(2 * np.pi * (kx * X / Lx + ky * Y / Ly) + ph)
        cols.append(f)
    rho, v1, v2, p = cols
    rho = np.abs(rho) + 0.3
    p = np.abs(p) + 0.3
    return euler2d_cons(rho, v1, v2, p, gamma)


# ---------------------------------------------------------------- single-element patterns
def _rand_prim(rng, n):
    return (rng.uniform(0.1, 2.0, n), rng.uniform(-1.0, 1.0, n), rng.uniform(-1.0, 1.0, n), rng.uniform(0.1, 2.0, n))


def element_patterns_1d(seed, nx, N, gamma=GAMMA):
    """1D Euler states built element by element: a jump at a uniformly random
    position inside the element (60 %), a smooth profile (20 %) or a constant
    (20 %), between seeded random states; elements are independent."""
    rng = np.random.default_rng(seed)
    xi = gl_nodes(N)[None, :]
    kind = rng.uniform(size=(nx, 1))
    pos = rng.uniform(0.0, 1.0, (nx, 1))
    A, B = _rand_prim(rng, nx), _rand_prim(rng, nx)
    amp, k, ph = rng.uniform(0.0, 0.5, (nx, 1)), rng.uniform(0.5, 3.0, (nx, 1)), rng.uniform(0, 2 * np.pi, (nx, 1))
    cols = []
    for c in (0, 1, 3):
        a, b = A[c][:, None], B[c][:, None]
        jump = np.where(xi < pos, a, b)
        smooth = a * (1.0 + amp * np.sin(2 * np.pi * k * xi + ph))
        cols.append(np.where(kind < 0.6, jump, np.where(kind < 0.8, smooth, a + 0.0 * xi)))
    rho, v, p = cols
    return np.stack([rho, rho * v, p / (gamma - 1.0) + 0.5 * rho * v * v])


def element_patterns_2d(seed, nx, ny, N, gamma=GAMMA):
    """2D Euler states built element by element: a straight discontinuity
    through a random point of the element at a random angle (60 %), a smooth
    profile (20 %) or a constant (20 %), between seeded random states."""
    rng = np.random.default_rng(seed)
    ne = nx * ny
    xi = gl_nodes(N)
    XI, ETA = np.meshgrid(xi, xi)                        # [q][p]
    XI, ETA = XI[None], ETA[None]
    kind = rng.uniform(size=(ne, 1, 1))
    px, py = rng.uniform(0, 1, (ne, 1, 1)), rng.uniform(0, 1, (ne, 1, 1))
    th = rng.uniform(0, 2 * np.pi, (ne, 1, 1))
    side = (XI - px) * np.cos(th) + (ETA - py) * np.sin(th) < 0
    A, B = _rand_prim(rng, ne), _rand_prim(rng, ne)
    amp, k, ph = rng.uniform(0.0, 0.5, (ne, 1, 1)), rng.uniform(0.5, 3.0, (ne, 1, 1)), rng.uniform(0, 2 * np.pi, (ne, 1, 1))
    cols = []
    for c in range(4):
        a, b = A[c][:, None, None], B[c][:, None, None]
        jump = np.where(side, a, b)
        smooth = a * (1.0 + amp * np.sin(2 * np.pi * k * (XI * np.cos(th) + ETA * np.sin(th)) + ph))
        cols.append(np.where(kind < 0.6, jump, np.where(kind < 0.8, smooth, a + 0.0 * XI)).reshape(ny, nx, N + 1, N + 1))
    rho, v1, v2, p = cols
    return euler2d_cons(rho, v1, v2, p, gamma)


# ---------------------------------------------------------------- ten-moment
def tenmom_quadrant_states(seed):
    """rho ~ U[0.5,2], v_i ~ U[-1,1], p11, p22 ~ U[0.5,2], p12 = r sqrt(p11 p22), r ~ U[-0.8,0.8]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(4):
        rho = rng.uniform(0.5, 2.0)
        v1, v2 = rng.uniform(-1.0, 1.0, 2)
        p11, p22 = rng.uniform(0.5, 2.0, 2)
        r = rng.uniform(-0.8, 0.8)
        out.append((rho, v1, v2, p11, r * np.sqrt(p11 * p22), p22))
    return out


def tenmom2d_quadrants(seed, nx, ny, N, dom=(-2.0, 2.0, -0.5, 0.5), split=None):
    X, Y = node_coords_2d(nx, ny, N, dom)
    st = tenmom_quadrant_states(seed)
    xs, ys = _split(dom, nx, ny, split)
    rho, v1, v2, p11, p12, p22 = _quadrant_fill(X, Y, xs, ys, st)
    return tenmom_cons(rho, v1, v2, p11, p12, p22)


def tenmom2d_smooth(seed, nx, ny, N, dom=(-2.0, 2.0, -0.5, 0.5), amp=0.1):
    rng = np.random.default_rng(seed)
    X, Y = node_coords_2d(nx, ny, N, dom)
    Lx, Ly = dom[1] - dom[0], dom[3] - dom[2]

    def field(base):
        f = np.full(X.shape, base)
        for _ in range(2):
            kx, ky = rng.integers(0, 3, 2)
            f = f + amp * np.sin(2 * np.pi * (kx * X / Lx + ky * Y / Ly) + rng.uniform(0, 2 * np.pi))
        return f

    rho, v1, v2 = field(1.0), field(0.2), field(-0.1)
    p11, p22, p12 = field(1.0), field(0.8), field(0.1)
    return tenmom_cons(rho, v1, v2, p11, p12, p22)


# Two-rarefaction problem of the ten-moment system with the source (the 1D
# system): (rho, v1, v2, P11, P12, P22) = (1, -4, 0, 9, 7, 9) left of the jump,
# (1, 4, 0, 9, 7, 9) right of it; potential W = 25 exp(-200 (x - 2)^2).  The
# domain [0, 4] with the jump at the potential's centre x = 2 (OFF_FACE of an
# element to the right) is a reading: the paper gives no domain.
TWO_RARE_SOURCE = (25.0, 200.0, 2.0, 0.0, 0.0, 0.0)   # amp, kappa, xc, yc, gx, gy


def tenmom1d_two_rarefaction(nx, N, dom=(0.0, 4.0), xs=None):
    x0, x1 = dom
    if xs is None:
        xs = 0.5 * (x0 + x1) + OFF_FACE * (x1 - x0) / nx
    x = node_coords_1d(nx, N, x0, x1)
    one = np.ones_like(x)
    v1 = np.where(x < xs, -4.0, 4.0)
    return tenmom_cons(one, v1, 0.0 * one, 9.0 * one, 7.0 * one, 9.0 * one)


def tenmom1d_equilibrium(nx, N, dom=(0.0, 4.0), T=10.0, amp=25.0, kappa=200.0, xc=2.0):
    """Rest state in the potential W = amp exp(-kappa (x - xc)^2): rho =
    exp(-W / (2 T)), v = 0, P11 = P22 = rho T, P12 = 0, for which the x
    momentum balance dP11/dx = -rho W_x / 2 of eq. tenmom.source holds."""
    x = node_coords_1d(nx, N, dom[0], dom[1])
    W = amp * np.exp(-kappa * (x - xc) ** 2)
    rho = np.exp(-W / (2.0 * T))
    z = 0.0 * rho
    return tenmom_cons(rho, z, z, rho * T, z, rho * T)


def batch_instances(seed, count, sides=(64, 512), degrees=(2, 3, 4)):
    """Seeded draw of uneven instances: grid side n ~ U{sides}, N ~ U{degrees}, states per quadrant."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(sides[0], sides[1] + 1))
        N = int(rng.choice(degrees))
        out.append({"n": n, "N": N, "seed": int(rng.integers(0, 2 ** 31 - 1))})
    return out
