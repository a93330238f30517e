"""Pins of the oracle's learned troubled-cell indicator: its features (the
modal energies the smoothness indicator of Sec. 4 compares), the network's
forward map, the feature-box fallback to the indicator, and its wiring into
the step."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2502_07517_amd import workloads as W


def _legendre_on_01(n, xi):
    """Orthonormal Legendre polynomial of degree n on [0, 1] (numpy's series)."""
    c = np.zeros(n + 1)
    c[n] = 1.0
    return math.sqrt(2 * n + 1) * np.polynomial.legendre.legval(2.0 * xi - 1.0, c)


def _euler2d_element_with_pressure(N, pfun):
    """One 2D Euler element, rho = 1, v = 0, pressure pfun(xi_x, xi_y) at the
    nodes, so that the indicator quantity rho * p equals the pressure."""
    xi = W.gl_nodes(N)
    X, Y = np.meshgrid(xi, xi)          # [q][p]
    p = pfun(X, Y)
    ue = np.zeros((4, N + 1, N + 1))
    ue[0] = 1.0
    ue[3] = p / 0.4
    return ue.reshape(4, -1)


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("i,j", [(1, 0), (0, 2), (2, 1), (1, 1)])
def test_features_of_a_single_mode(N, i, j):
    """p = a + b L_i(x) L_j(y): only shells 0 and max(i, j) carry energy,
    a^2 and b^2, so feature K = max(i,j) is log10(b^2/(a^2+b^2))/6 + 1 and all
    other features sit at the floor -1."""
    if max(i, j) > N:
        pytest.skip("mode above the degree")
    a, b = 2.0, 0.3
    ue = _euler2d_element_with_pressure(
        N, lambda X, Y: a + b * _legendre_on_01(i, X) * _legendre_on_01(j, Y))
    cfg = O.RefConfig.make(O.EULER2D, N, 1, 1)
    f = O.indicator_features(cfg, ue)
    K = max(i, j)
    want = np.full(N, -1.0)
    want[K - 1] = math.log10(b * b / (a * a + b * b)) / 6.0 + 1.0
    assert np.allclose(f, want, atol=1e-12), (f, want)


def test_features_constant_state_at_floor():
    ue = _euler2d_element_with_pressure(3, lambda X, Y: 1.7 + 0 * X)
    cfg = O.RefConfig.make(O.EULER2D, 3, 1, 1)
    assert np.all(O.indicator_features(cfg, ue) == -1.0)


def test_features_two_modes_cumulative_share():
    """Shells 1 and 3 with energies b1^2, b3^2: r_1 = b1^2/(a^2+b1^2),
    r_2 = 0, r_3 = b3^2/(a^2+b1^2+b3^2)."""
    a, b1, b3 = 1.5, 0.4, 0.05
    ue = _euler2d_element_with_pressure(
        3, lambda X, Y: a + b1 * _legendre_on_01(1, X) + b3 * _legendre_on_01(3, Y))
    cfg = O.RefConfig.make(O.EULER2D, 3, 1, 1)
    f = O.indicator_features(cfg, ue)
    r1 = b1 ** 2 / (a ** 2 + b1 ** 2)
    r3 = b3 ** 2 / (a ** 2 + b1 ** 2 + b3 ** 2)
    want = [math.log10(r1) / 6 + 1, -1.0, math.log10(r3) / 6 + 1]
    assert np.allclose(f, want, atol=1e-12)


# ------------------------------------------------------------- network forward map
def _npar(dims):
    return sum(dims[i + 1] * dims[i] + dims[i + 1] for i in range(len(dims) - 1))


def test_mlp_zero_weights_give_sigmoid_of_bias():
    dims = [3, 4, 4, 1]
    p = np.zeros(_npar(dims))
    p[-1] = math.log(3.0)                      # sigmoid(log 3) = 3/4
    y = O.mlp_forward(dims, p, np.random.default_rng(0).standard_normal((5, 3)))
    assert np.allclose(y, 0.75, atol=1e-15)


def test_mlp_saturated_unit_is_a_step():
    """One hidden unit with a huge weight on input 2 acts as sign(x_2);
    output = sigmoid(v sign + c) with v = c = log(3)/2 (3/4 or 1/2)."""
    dims = [3, 1, 1]
    W1 = np.array([0.0, 0.0, 1e6]); b1 = np.array([0.0])
    v = np.array([math.log(3.0) / 2]); c = np.array([math.log(3.0) / 2])
    p = np.concatenate([W1, b1, v, c])
    x = np.array([[5.0, -5.0, 0.3], [-5.0, 5.0, -0.3]])
    y = O.mlp_forward(dims, p, x)
    assert np.allclose(y, [0.75, 0.5], atol=1e-12)


def test_mlp_hidden_permutation_and_sign_invariance():
    """Permuting hidden units, or flipping a unit's in- and out-weights
    (tanh is odd), leaves the output unchanged; a transposed weight layout
    or a wrong activation fails this."""
    dims = [3, 5, 4, 1]
    rng = np.random.default_rng(1)
    p = rng.standard_normal(_npar(dims))
    x = rng.standard_normal((9, 3))
    y = O.mlp_forward(dims, p, x)
    W1 = p[:15].reshape(5, 3); b1 = p[15:20]
    W2 = p[20:40].reshape(4, 5); b2 = p[40:44]
    W3 = p[44:48].reshape(1, 4); b3 = p[48:49]
    perm = np.array([3, 0, 4, 1, 2])
    s = np.array([1, -1, 1, -1, -1])
    W1q, b1q = (W1 * s[:, None])[perm], (b1 * s)[perm]
    W2q = (W2 * s[None, :])[:, perm]
    q = np.concatenate([W1q.ravel(), b1q, W2q.ravel(), b2, W3.ravel(), b3])
    assert np.allclose(O.mlp_forward(dims, q, x), y, atol=1e-14)


# ------------------------------------------------------------- learned alpha and the step
def _selector_net(N, k, gain, v, c):
    """dims [N, 1, 1]: alpha = sigmoid(v tanh(gain x_k) + c)."""
    W1 = np.zeros(N); W1[k] = gain
    return [N, 1, 1], np.concatenate([W1, [0.0], [v], [c]])


@pytest.mark.parametrize("k", [0, 1, 2])
def test_learned_alpha_reads_the_right_feature(k):
    N = 3
    ue = _euler2d_element_with_pressure(
        N, lambda X, Y: 1.0 + 0.2 * _legendre_on_01(k + 1, X))
    dims, p = _selector_net(N, k, 1e6, math.log(3.0) / 2, math.log(3.0) / 2)
    lo, hi = -np.ones(N), np.ones(N)
    cfg = O.RefConfig.make(O.EULER2D, N, 1, 1, blend=O.BLEND_MH, indicator=O.IND_LEARNED,
                           mlp=(dims, p, lo, hi))
    a, fb = O.learned_alpha(cfg, ue)
    assert not fb
    # x_{k} > 0 (share 0.04/1.04 -> 1 + log10(.038)/6 = 0.76) -> 3/4; every other feature is -1 -> 1/2
    assert abs(a - 0.75) < 1e-12
    dims2, p2 = _selector_net(N, (k + 1) % N, 1e6, math.log(3.0) / 2, math.log(3.0) / 2)
    cfg.set_mlp(dims2, p2, lo, hi)
    assert abs(O.learned_alpha(cfg, ue)[0] - 0.5) < 1e-12


def test_learned_alpha_clips_like_the_indicator():
    N = 2
    ue = _euler2d_element_with_pressure(N, lambda X, Y: 1.0 + 0.1 * X)
    dims = [N, 2, 1]
    p = np.zeros(_npar(dims))
    lo, hi = -np.ones(N), np.ones(N)
    p[-1] = math.log(0.0005 / 0.9995)           # 5e-4 < alpha_min = 1e-3 -> 0
    cfg = O.RefConfig.make(O.EULER2D, N, 1, 1, blend=O.BLEND_MH, indicator=O.IND_LEARNED,
                           mlp=(dims, p, lo, hi), alpha_max=0.6)
    assert O.learned_alpha(cfg, ue)[0] == 0.0
    p[-1] = 5.0                                  # 0.993 > alpha_max = 0.6 -> 0.6
    cfg.set_mlp(dims, p, lo, hi)
    assert O.learned_alpha(cfg, ue)[0] == 0.6


def _quadrant_case(N=2, n=12, seed=3):
    u = W.euler2d_quadrants(seed, n, N)
    return u, n


def test_learned_step_with_constant_network_equals_constant_alpha():
    N = 2
    u, n = _quadrant_case(N)
    dims = [N, 4, 4, 1]
    p = np.zeros(_npar(dims))
    p[-1] = math.log(0.3 / 0.7)
    kw = dict(domain=(0.0, 1.0, 0.0, 1.0), bc=(O.OUTFLOW,) * 4, blend=O.BLEND_MH,
              flux_limiter=1, scaling=1)
    cl = O.RefConfig.make(O.EULER2D, N, n, n, indicator=O.IND_LEARNED, smooth_nbr=1,
                          mlp=(dims, p, -np.ones(N), np.ones(N)), **kw)
    cc = O.RefConfig.make(O.EULER2D, N, n, n, indicator=O.IND_CONST, alpha_const=0.3, **kw)
    dt = 0.5 * O.compute_dt(cl, u)
    ul, al, dl, _ = O.step(cl, u, dt)
    uc, ac, dc, _ = O.step(cc, u, dt)
    assert np.allclose(al, 0.3, atol=1e-15)
    assert np.max(np.abs(ul - uc)) < 1e-13


def test_learned_step_outside_box_equals_indicator_step():
    N = 3
    u, n = _quadrant_case(N)
    dims = [N, 4, 4, 1]
    p = np.random.default_rng(0).standard_normal(_npar(dims))
    kw = dict(domain=(0.0, 1.0, 0.0, 1.0), bc=(O.OUTFLOW,) * 4, blend=O.BLEND_MH,
              flux_limiter=1, scaling=1, smooth_nbr=1)
    cl = O.RefConfig.make(O.EULER2D, N, n, n, indicator=O.IND_LEARNED,
                          mlp=(dims, p, np.full(N, 2.0), np.full(N, 3.0)), **kw)
    cp = O.RefConfig.make(O.EULER2D, N, n, n, indicator=O.IND_PAPER, **kw)
    dt = 0.5 * O.compute_dt(cl, u)
    ul, al, _, _ = O.step(cl, u, dt)
    up, ap, _, _ = O.step(cp, u, dt)
    assert np.array_equal(al, ap)
    assert np.array_equal(ul, up)
