"""Batched form: many uneven instances (grid sizes and degrees) advanced
together give exactly the results of advancing each instance on its own, in
the same arithmetic; the captured-graph replay and the autotuned persistent
grids change nothing."""
import numpy as np
import pytest

from paper_2502_07517_amd import crkfr as C
from paper_2502_07517_amd import workloads as W
from oracle_runs import cfl_for

pytestmark = pytest.mark.gpu


def _instances(dtype, lim):
    specs = W.batch_instances(11, 7, sides=(5, 23), degrees=(2, 3, 4))
    out = []
    for sp in specs:
        n, N = sp["n"], sp["N"]
        bc = (C.FARFIELD,) * 4
        s = C.Solver(C.EULER2D, N, n, n + 1, bc=bc, dtype=dtype, cfl=cfl_for(N))
        if lim:
            s.set_limiter(blend=C.BLEND_MH, flux_limiter=1, scaling=1)
        X, Y = W.node_coords_2d(n, n + 1, N, (0, 1, 0, 1))
        st = W.quadrant_states_euler(sp["seed"])
        rho, v1, v2, p = W._quadrant_fill(X, Y, 0.5 + 0.37 / n, 0.5 + 0.37 / (n + 1), st)
        u0 = W.euler2d_cons(rho, v1, v2, p)
        s.set_state(u0)
        out.append((s, u0))
    return out


@pytest.mark.parametrize("dtype", [C.FP64, C.MP32])
@pytest.mark.parametrize("lim", [0, 1])
def test_batch_equals_sequential(dtype, lim):
    seq = _instances(dtype, lim)
    bat = _instances(dtype, lim)
    steps = 6
    for s, _ in seq:
        for _ in range(steps):
            s.step(0.0)
    b = C.Batch([s for s, _ in bat])
    b.step()
    b.advance(steps - 2)     # graph replay of step pairs
    b.step()
    b.sync()
    for (s1, _), (s2, _) in zip(seq, bat):
        assert np.array_equal(s1.get_state(), s2.get_state())
        d1, _ = s1.get_diag()
        d2, _ = s2.get_diag()
        assert d1["steps"] == d2["steps"] == steps and d1["t"] == d2["t"]


def test_batch_autotune_keeps_results():
    a = _instances(C.MP32, 1)
    c = _instances(C.MP32, 1)
    ba = C.Batch([s for s, _ in a])
    grids = ba.autotune(2)
    assert len(grids) == ba.num_groups() >= 2
    bc = C.Batch([s for s, _ in c])
    ba.advance(4)
    bc.advance(4)
    ba.sync()
    bc.sync()
    for (s1, _), (s2, _) in zip(a, c):
        assert np.array_equal(s1.get_state(), s2.get_state())
