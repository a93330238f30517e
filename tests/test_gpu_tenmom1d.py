"""GPU parity of the one-dimensional ten-moment system with the source
(eq. tmp with x dependence only, eq. tenmom.source) and the two-rarefaction
test of Sec. 5.4.2 against the oracle."""
import numpy as np
import pytest

import oracle as O
from gpu_cases import rel_l1, rel_linf
from oracle_runs import cfl_for
from paper_2502_07517_amd import crkfr as C
from paper_2502_07517_amd import workloads as W

pytestmark = pytest.mark.gpu
LIM = dict(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
DOM = (0.0, 4.0, 0.0, 1.0)
SRC = W.TWO_RARE_SOURCE
COUNTERS = ("n_troubled", "n_flux_limited", "n_lo_inadmissible", "n_slope_limited", "n_hancock_fallback",
            "n_scaled", "n_mean_inadmissible")


def _pair(N, nx, *, lim=None, bc=(C.OUTFLOW,) * 4, dom=DOM, dtype=C.FP64, source=SRC):
    lim = lim or {}
    ref = O.RefConfig.make(C.TENMOM1D, N, nx, bc=bc, domain=dom, cfl=cfl_for(N), source=1 if source else 0,
                           src=source[:4] if source else (0, 0, 0, 0), src_lin=source[4:] if source else (0, 0),
                           **lim)
    gpu = C.Solver(C.TENMOM1D, N, nx, bc=bc, domain=dom, dtype=dtype, cfl=cfl_for(N))
    if lim:
        gpu.set_limiter(**lim)
    if source:
        gpu.set_source(1, *source)
    return ref, gpu


def _admissible(u):
    r = u[0]
    v1, v2 = u[1] / r, u[2] / r
    P11, P12, P22 = 2 * u[3] - r * v1 * v1, 2 * u[4] - r * v1 * v2, 2 * u[5] - r * v2 * v2
    return r.min() > 0 and P11.min() > 0 and (P11 * P22 - P12 ** 2).min() > 0


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_equilibrium_with_source_fp64(N):
    """Smooth: the rest state in the Gaussian potential, perturbed."""
    nx = 37
    ref, gpu = _pair(N, nx)
    u0 = W.tenmom1d_equilibrium(nx, N)
    u0[1] += 0.05 * np.sin(np.pi * W.node_coords_1d(nx, N, 0.0, 4.0))
    u = u0.copy()
    gpu.set_state(u0.copy())
    dt = O.compute_dt(ref, u0)
    for _ in range(10):
        u, _, _, st = O.step(ref, u, dt)
        assert st == 0
        gpu.step(dt)
    assert rel_linf(u, gpu.get_state().reshape(u.shape)) <= 1e-12


@pytest.mark.parametrize("N", [2, 3])
def test_two_rarefaction_single_steps_fp64(N):
    """The oracle's trajectory; every 11th step the GPU takes the same step
    from the oracle's state (limiter chain and source on)."""
    nx = 100
    ref, gpu = _pair(N, nx, lim=LIM)
    u, t, k, worst, acted = W.tenmom1d_two_rarefaction(nx, N), 0.0, 0, 0.0, 0
    while t < 0.1 - 1e-14:
        dt = min(O.compute_dt(ref, u), 0.1 - t)
        un, _, do, st = O.step(ref, u, dt)
        assert st == 0
        if k % 11 == 0:
            gpu.set_state(u.copy())
            gpu.step(dt)
            dg, _ = gpu.get_diag()
            e = rel_l1(un, gpu.get_state().reshape(un.shape))
            worst = max(worst, e)
            assert e <= 1e-12, (k, e)
            for key in COUNTERS:
                assert do[key] == dg[key], (k, key)
            acted += do["n_flux_limited"] + do["n_scaled"]
        u, t, k = un, t + dt, k + 1
    print(f"two rarefaction N={N}: worst single-step rel. L1 {worst:.2e}, limiter actions {acted}")
    assert acted > 0


def test_two_rarefaction_full_runs():
    """Device time steps to t = 0.1: 100 elements against the oracle's run
    (FP64), and the paper's 500 elements (N = 3): admissible at every node,
    density near vacuum."""
    N, nx = 3, 100
    ref, _ = _pair(N, nx, lim=LIM)
    u, t = W.tenmom1d_two_rarefaction(nx, N), 0.0
    while t < 0.1 - 1e-14:
        dt = min(O.compute_dt(ref, u), 0.1 - t)
        u, _, _, st = O.step(ref, u, dt)
        assert st == 0
        t += dt
    _, gpu = _pair(N, nx, lim=LIM)
    gpu.set_state(W.tenmom1d_two_rarefaction(nx, N))
    gpu.advance(0.1, 100000)
    d, rc = gpu.get_diag()
    assert rc == 0 and abs(d["t"] - 0.1) < 1e-14
    ug = gpu.get_state().reshape(u.shape)
    print(f"two rarefaction 100 elements: rel. L1 vs oracle {rel_l1(u, ug):.2e}")
    assert rel_l1(u, ug) <= 1e-12
    _, g5 = _pair(3, 500, lim=LIM)
    g5.set_state(W.tenmom1d_two_rarefaction(500, 3))
    g5.advance(0.1, 100000)
    d, rc = g5.get_diag()
    assert rc == 0 and abs(d["t"] - 0.1) < 1e-14 and d["n_mean_inadmissible"] == 0
    u5 = g5.get_state()
    assert _admissible(u5)
    assert u5[0].min() < 0.01


@pytest.mark.parametrize("N", [2, 3])
def test_walls_single_steps_fp64(N):
    nx = 24
    dom = (0.0, 1.0, 0.0, 1.0)
    src = (25.0, 200.0, 0.6, 0.0, 0.0, 0.0)
    ref, gpu = _pair(N, nx, lim=LIM, bc=(C.REFLECT,) * 4, dom=dom, source=src)
    u = W.tenmom1d_two_rarefaction(nx, N, dom=(0.0, 1.0), xs=0.41)
    u[1] *= 0.05
    for k in range(30):
        dt = O.compute_dt(ref, u)
        un, _, do, st = O.step(ref, u, dt)
        assert st == 0
        if k % 5 == 0:
            gpu.set_state(u.copy())
            gpu.step(dt)
            assert rel_l1(un, gpu.get_state().reshape(un.shape)) <= 1e-12
        u = un


def test_two_rarefaction_mp32_runs_admissible():
    """FP32 bulk arithmetic (FP64 means and roots) on the near-vacuum run:
    admissible in means, and close to the FP64 run in L1."""
    N, nx = 3, 200
    out = {}
    for dtype in (C.FP64, C.MP32):
        _, g = _pair(N, nx, lim=LIM, dtype=dtype)
        g.set_state(W.tenmom1d_two_rarefaction(nx, N))
        g.advance(0.1, 100000)
        d, rc = g.get_diag()
        assert rc == 0 and d["n_mean_inadmissible"] == 0
        out[dtype] = g.get_state()
    e = rel_l1(out[C.FP64], out[C.MP32])
    print(f"two rarefaction FP32 bulk vs FP64: rel. L1 {e:.2e}")
    assert e <= 1e-3


def test_batch_of_tenmom1d_members_equals_sequential():
    members = [(2, 60), (3, 100), (4, 41)]

    def make():
        out = []
        for N, nx in members:
            _, g = _pair(N, nx, lim=LIM)
            g.set_state(W.tenmom1d_two_rarefaction(nx, N))
            out.append(g)
        return out
    seq, bat = make(), make()
    for s in seq:
        for _ in range(6):
            s.step(0.0)
    b = C.Batch(bat)
    b.advance(6)
    b.sync()
    for s1, s2 in zip(seq, bat):
        assert np.array_equal(s1.get_state(), s2.get_state())
