"""Pins of the oracle's reference-element operators and tableaux against
independent constructions (numpy's Gauss rule and polynomial algebra)."""
import numpy as np
import numpy.polynomial.legendre as npleg
import numpy.polynomial.polynomial as nppoly
import pytest

import oracle


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_gl_nodes_weights_match_numpy_and_exactness(N):
    # Sec. 2, eq. soln.points: GL rule on [0,1], exact to degree 2N+1
    xi, w = oracle.gl(N)
    x, wn = npleg.leggauss(N + 1)
    assert np.allclose(xi, 0.5 * (x + 1.0), atol=1e-15, rtol=0)
    assert np.allclose(w, 0.5 * wn, atol=1e-15, rtol=0)
    assert abs(w.sum() - 1.0) < 1e-15
    for k in range(2 * N + 2):
        assert abs(np.dot(w, xi ** k) - 1.0 / (k + 1)) < 1e-14
    # not exact one degree higher
    k = 2 * N + 2
    assert abs(np.dot(w, xi ** k) - 1.0 / (k + 1)) > 1e-8


def _interp_deriv_matrix(xi):
    """D[i][j] = l_j'(xi_i) from numpy's polynomial fit of each cardinal function."""
    n = len(xi)
    D = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        c = nppoly.polyfit(xi, e, n - 1)
        D[:, j] = nppoly.polyval(xi, nppoly.polyder(c))
    return D


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_diff_matrix(N):
    # eq. diff.matrix
    xi, _ = oracle.gl(N)
    D = oracle.diff_matrix(N, xi)
    assert np.allclose(D, _interp_deriv_matrix(xi), atol=1e-10)
    for k in range(N + 1):
        assert np.allclose(D @ xi ** k, k * xi ** max(k - 1, 0) if k else 0.0, atol=1e-12)
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-12)
    assert np.allclose(np.linalg.matrix_power(D, N + 1), 0.0, atol=1e-9)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_radau_identity(N):
    # eq. fr.equiv: g_R'(xi_p) = l_p(1)/w_p, g_L'(xi_p) = -l_p(0)/w_p for the
    # right/left Radau polynomials g_R = (P_{N+1} + P_N)/2 in x = 2 xi - 1
    xi, w = oracle.gl(N)
    l0 = oracle.lagrange_at(N, xi, 0.0)
    l1 = oracle.lagrange_at(N, xi, 1.0)
    cR = np.zeros(N + 2)
    cR[N + 1] = 0.5
    cR[N] = 0.5
    dcR = npleg.legder(cR)
    x = 2 * xi - 1
    gR_prime = 2.0 * npleg.legval(x, dcR)        # d/dxi = 2 d/dx
    gL_prime = -2.0 * npleg.legval(-x, dcR)      # g_L(xi) = g_R(1 - xi)
    assert abs(npleg.legval(1.0, cR) - 1.0) < 1e-14 and abs(npleg.legval(-1.0, cR)) < 1e-14
    assert np.allclose(gR_prime, l1 / w, atol=1e-11)
    assert np.allclose(gL_prime, -l0 / w, atol=1e-11)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_lagrange_cardinal_and_boundary_values(N):
    xi, _ = oracle.gl(N)
    for p in range(N + 1):
        assert np.allclose(oracle.lagrange_at(N, xi, xi[p]), np.eye(N + 1)[p], atol=1e-14)
    # boundary values reproduce polynomials of degree N
    for k in range(N + 1):
        assert abs(oracle.lagrange_at(N, xi, 1.0) @ xi ** k - 1.0) < 1e-12
        assert abs(oracle.lagrange_at(N, xi, 0.0) @ xi ** k - (1.0 if k == 0 else 0.0)) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_orthonormal_legendre(N):
    xi, w = oracle.gl(N)
    L = oracle.legendre_orthonormal(N, xi)
    G = (L * w[None, :]) @ L.T
    assert np.allclose(G, np.eye(N + 1), atol=1e-13)


@pytest.mark.parametrize("s,order", [(2, 2), (3, 3), (4, 4)])
def test_tableau_order_conditions(s, order):
    # eqs. crk22, crk33, crk44 give RK methods of order s
    a, b, c = oracle.tableau(s)
    assert np.allclose(np.triu(a), 0.0)                     # strictly lower triangular
    assert abs(b.sum() - 1) < 1e-15
    assert abs(b @ c - 1 / 2) < 1e-15
    if order >= 3:
        assert abs(b @ c ** 2 - 1 / 3) < 1e-15
        assert abs(b @ a @ c - 1 / 6) < 1e-15
    if order >= 4:
        assert abs(b @ c ** 3 - 1 / 4) < 1e-15
        assert abs(b @ (c * (a @ c)) - 1 / 8) < 1e-15
        assert abs(b @ a @ c ** 2 - 1 / 12) < 1e-15
        assert abs(b @ a @ a @ c - 1 / 24) < 1e-15


@pytest.mark.parametrize("N,s", [(1, 2), (2, 3), (3, 4)])
def test_local_crk_linear_closed_form(N, s):
    # App. A, eq. linear.avg: U = sum_{m<=N} (-a dt)^m/(m+1)! d_x^m u, F = a U
    rng = np.random.default_rng(N)
    a_adv, dx, dt = 1.3, 0.1, 0.02
    cfg = oracle.RefConfig.make(oracle.LINADV1D, N, 10, stages=s, adv=a_adv, domain=(0, 1, 0, 1))
    xi, _ = oracle.gl(N)
    D = _interp_deriv_matrix(xi) / dx
    u = rng.standard_normal(N + 1)
    F, G, U, S = oracle.local_crk(cfg, u, dt)
    Uref = np.zeros(N + 1)
    term = u.copy()
    fact = 1.0
    for m in range(N + 1):
        fact *= (m + 1)
        Uref += (-a_adv * dt) ** m / fact * term
        term = D @ term
    assert np.allclose(U[0], Uref, atol=1e-13)
    assert np.allclose(F[0], a_adv * Uref, atol=1e-13)
    assert np.allclose(S, 0.0)
