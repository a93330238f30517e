"""Pins of the oracle's physics: flux Jacobian spectra (finite differences),
rotational symmetry, the ten-moment reduction to Euler with gamma = 3, and the
admissibility functions."""
import numpy as np
import pytest

import oracle
from paper_2502_07517_amd import workloads as W


def fd_jacobian(eq, u, direction, gamma=1.4, h=1e-6):
    M = len(u)
    J = np.zeros((M, M))
    for j in range(M):
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        fp = oracle.flux(eq, up, gamma)[direction]
        fm = oracle.flux(eq, um, gamma)[direction]
        J[:, j] = (fp - fm) / (2 * h)
    return J


@pytest.mark.parametrize("seed", range(5))
def test_euler_spectral_radius(seed):
    # eq. spectral.radius.1d and the 2D radii: sigma = |v| + c
    rng = np.random.default_rng(seed)
    rho, v1, v2, p = rng.uniform(0.2, 2), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.2, 2)
    u1 = W.euler1d_cons(np.array(rho), np.array(v1), np.array(p))
    ev = np.linalg.eigvals(fd_jacobian(oracle.EULER1D, u1, 0))
    c = np.sqrt(1.4 * p / rho)
    assert np.allclose(np.sort(ev.real), np.sort([v1 - c, v1, v1 + c]), atol=1e-6)
    assert abs(oracle.sigma(oracle.EULER1D, u1)[0] - (abs(v1) + c)) < 1e-13
    u2 = W.euler2d_cons(np.array(rho), np.array(v1), np.array(v2), np.array(p))
    for d, v in ((0, v1), (1, v2)):
        ev = np.linalg.eigvals(fd_jacobian(oracle.EULER2D, u2, d))
        assert np.allclose(np.sort(ev.real), np.sort([v - c, v, v, v + c]), atol=1e-6)
        assert abs(oracle.sigma(oracle.EULER2D, u2)[d] - (abs(v) + c)) < 1e-13


@pytest.mark.parametrize("seed", range(5))
def test_tenmoment_eigenvalues(seed):
    # eq. tmp: x-direction eigenvalues v1 +- sqrt(3 P11/rho), v1 +- sqrt(P11/rho), v1, v1
    rng = np.random.default_rng(100 + seed)
    rho, v1, v2 = rng.uniform(0.5, 2), rng.uniform(-1, 1), rng.uniform(-1, 1)
    p11, p22 = rng.uniform(0.5, 2, 2)
    p12 = rng.uniform(-0.8, 0.8) * np.sqrt(p11 * p22)
    u = W.tenmom_cons(*(np.array(x) for x in (rho, v1, v2, p11, p12, p22)))
    ev = np.sort(np.linalg.eigvals(fd_jacobian(oracle.TENMOM2D, u, 0)).real)
    a, b = np.sqrt(3 * p11 / rho), np.sqrt(p11 / rho)
    assert np.allclose(ev, np.sort([v1 - a, v1 - b, v1, v1, v1 + b, v1 + a]), atol=1e-5)
    ev = np.sort(np.linalg.eigvals(fd_jacobian(oracle.TENMOM2D, u, 1)).real)
    a, b = np.sqrt(3 * p22 / rho), np.sqrt(p22 / rho)
    assert np.allclose(ev, np.sort([v2 - a, v2 - b, v2, v2, v2 + b, v2 + a]), atol=1e-5)
    sx, sy = oracle.sigma(oracle.TENMOM2D, u)
    assert abs(sx - (abs(v1) + np.sqrt(3 * p11 / rho))) < 1e-13
    assert abs(sy - (abs(v2) + np.sqrt(3 * p22 / rho))) < 1e-13


def test_tenmoment_reduces_to_euler_gamma3():
    # x-only data (v2 = 0, P12 = 0): (rho, rho v1, E11) obeys 1D Euler with gamma = 3
    rng = np.random.default_rng(7)
    for _ in range(5):
        rho, v1, p11, p22 = rng.uniform(0.3, 2), rng.uniform(-1, 1), rng.uniform(0.3, 2), rng.uniform(0.3, 2)
        u = W.tenmom_cons(*(np.array(x) for x in (rho, v1, 0.0, p11, 0.0, p22)))
        f, _ = oracle.flux(oracle.TENMOM2D, u)
        ue = W.euler1d_cons(np.array(rho), np.array(v1), np.array(p11), gamma=3.0)
        fe, _ = oracle.flux(oracle.EULER1D, ue, gamma=3.0)
        assert np.allclose(ue, u[[0, 1, 3]], atol=1e-14)
        assert np.allclose(f[[0, 1, 3]], fe, atol=1e-13)


@pytest.mark.parametrize("eq,perm,sign", [
    (oracle.EULER2D, [0, 2, 1, 3], None),
    (oracle.TENMOM2D, [0, 2, 1, 5, 4, 3], None),
])
def test_rotational_symmetry(eq, perm, sign):
    # swapping x and y maps g onto f of the permuted state
    rng = np.random.default_rng(3)
    for _ in range(5):
        if eq == oracle.EULER2D:
            u = W.euler2d_cons(*(np.array(x) for x in (rng.uniform(0.3, 2), rng.uniform(-1, 1),
                                                      rng.uniform(-1, 1), rng.uniform(0.3, 2))))
        else:
            p11, p22 = rng.uniform(0.5, 2, 2)
            u = W.tenmom_cons(*(np.array(x) for x in (rng.uniform(0.3, 2), rng.uniform(-1, 1), rng.uniform(-1, 1),
                                                     p11, 0.3 * np.sqrt(p11 * p22), p22)))
        f, g = oracle.flux(eq, u)
        fs, gs = oracle.flux(eq, u[perm])
        assert np.allclose(g[perm], fs, atol=1e-13)
        assert np.allclose(f[perm], gs, atol=1e-13)


def test_admissibility_functions():
    u = W.euler2d_cons(np.array(1.2), np.array(0.3), np.array(-0.4), np.array(0.7))
    assert abs(oracle.adm(oracle.EULER2D, 0, u) - 1.2) < 1e-15
    assert abs(oracle.adm(oracle.EULER2D, 1, u) - 0.7) < 1e-14
    p11, p12, p22 = 1.5, -0.4, 0.9
    u = W.tenmom_cons(*(np.array(x) for x in (0.8, 0.2, 0.5, p11, p12, p22)))
    assert abs(oracle.adm(oracle.TENMOM2D, 1, u) - p11) < 1e-14
    assert abs(oracle.adm(oracle.TENMOM2D, 2, u) - (p11 * p22 - p12 ** 2)) < 1e-13
    assert oracle.nadm(oracle.LINADV1D) == 0 and oracle.nadm(oracle.TENMOM2D) == 3
