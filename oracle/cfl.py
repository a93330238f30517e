"""Fourier stability analysis giving CFL(N) for the time-step rule (eq.
time.step.2d).  The paper takes CFL(N) from tables of earlier work that it does
not print; this recomputes them for the scheme actually built: Gauss-Legendre
points, Radau correction, D2 dissipation (equivalent to D-CSX for linear
problems, Sec. 3.1.1), cRK tableau of s stages.

Test infrastructure only.  For u_t + a u_x = 0 the local cRK procedure gives
U = P u with P = sum_i b_i R_i, R_1 = I, R_i = I - nu_a sum_{j<i} a_ij D R_j
(eq. linear.avg), nu_a = a dt/dx.  The D2 flux with dissipation speed lambda
(eq. D2, eq. rusanov.wave.speed) is
    F*_{e+1/2} = a (U_e(1) + U_{e+1}(0))/2 - lambda (U_{e+1}(0) - U_e(1))/2,
and the FR update (eq. crkfr.avg) of a Fourier mode U_{e+1} = exp(i k) U_e is
    u^{n+1} = [I - (nu_a D + b_R (F_R - nu_a l(1)^T) - b_L (F_L - nu_a l(0)^T)) P] u^n
with the face operators F_R, F_L scaled by dt/dx and b_R = l(1)/w, b_L = l(0)/w.
CFL is the largest nu = lambda dt/dx whose amplification matrix has spectral
radius <= 1 + tol for every wavenumber and every speed ratio a/lambda in the
given set.  With the ratio 1 (upwind, a scalar linear flux) this is the table
the paper refers to; for systems, where the Rusanov speed exceeds the speed of
all but the fastest field, the ratios span [0, 1].

With the D1 dissipation (eq. D1) the dissipative part acts on the solution
at the current time instead of the time average: the face operators split
into a central part applied to U = P u and a dissipative part applied to u.
D-CSX (eq. dcsx) equals D2 for a linear flux.

With Gauss-Legendre-Lobatto points (points = 1) the same formulas hold with
the GLL nodes and weights: the g2 correction enters through the same
identity g_R'(xi_p) = l_p(1)/w_p (eq. fr.equiv).
"""
import numpy as np

from .oracle import nodes, diff_matrix, lagrange_at, tableau


def amplification_matrix(N, s, nu, kappa, ratio=1.0, d1=False, points=0):
    xi, w = nodes(N, points)
    D = diff_matrix(N, xi)
    l0 = lagrange_at(N, xi, 0.0)
    l1 = lagrange_at(N, xi, 1.0)
    a, b, _ = tableau(s)
    nu_a = ratio * nu
    I = np.eye(N + 1)
    R = []
    for i in range(s):
        Ri = I.copy()
        for j in range(i):
            Ri = Ri - nu_a * a[i, j] * D @ R[j]
        R.append(Ri)
    P = sum(b[i] * R[i] for i in range(s))
    E = np.exp(1j * kappa)
    FRc = 0.5 * nu_a * (l1 + E * l0)
    FLc = 0.5 * nu_a * (np.conj(E) * l1 + l0)
    FRd = -0.5 * nu * (E * l0 - l1)
    FLd = -0.5 * nu * (l0 - np.conj(E) * l1)
    central = nu_a * D + np.outer(l1 / w, FRc - nu_a * l1) - np.outer(l0 / w, FLc - nu_a * l0)
    diss = np.outer(l1 / w, FRd) - np.outer(l0 / w, FLd)
    return I - central @ P - diss @ (I if d1 else P)


def max_growth(N, s, nu, nk=4096, ratios=(1.0,), d1=False, points=0):
    ks = np.linspace(0.0, 2.0 * np.pi, nk)
    return max(np.max(np.abs(np.linalg.eigvals(amplification_matrix(N, s, nu, k, r, d1, points))))
               for r in ratios for k in ks)


SYSTEM_RATIOS = tuple(np.linspace(0.0, 1.0, 21))


def cfl_number(N, s=None, tol=1e-12, nk=4096, iters=50, ratios=(1.0,), d1=False, points=0):
    """Largest stable nu by bisection on max_{k, ratio} rho(G) <= 1 + tol."""
    if s is None:
        s = min(N + 1, 4)
    lo, hi = 0.0, 1.0
    while max_growth(N, s, hi, nk, ratios, d1, points) <= 1.0 + tol:
        hi *= 2.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if max_growth(N, s, mid, nk, ratios, d1, points) <= 1.0 + tol:
            lo = mid
        else:
            hi = mid
    return lo
