"""Small drivers around the oracle for the scheme-level pins (test helper)."""
import json
import os

import numpy as np

import oracle

_GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def cfl_table(kind="cfl"):
    with open(os.path.join(_GOLD, "cfl.json")) as f:
        d = json.load(f)
    return {(v["N"], v["stages"]): v[kind] for v in d.values() if kind in v}


def cfl_for(N, s=None, system=True):
    """CFL(N): the system value (all speed ratios) unless system=False (upwind)."""
    s = s if s is not None else min(N + 1, 4)
    return cfl_table("cfl_system" if system else "cfl")[(N, s)]


def run(cfg, u, t_end, max_steps=100000, dt_fixed=None):
    """Advance with the time-step rule (eq. time.step.2d), last step clipped."""
    t, n = 0.0, 0
    diags = []
    ghost = oracle.boundary_traces(cfg, u) if oracle.has_farfield(cfg) else None
    while t < t_end - 1e-14 and n < max_steps:
        dt = dt_fixed if dt_fixed is not None else oracle.compute_dt(cfg, u)
        dt = min(dt, t_end - t)
        u, _, d, st = oracle.step(cfg, u, dt, ghost=ghost)
        diags.append(d)
        t += dt
        n += 1
    return u, n, diags


def weights_2d(N):
    _, w = oracle.gl(N)
    return np.outer(w, w)


def l1_error_2d(u, uex, N, dx, dy, area):
    """L1 = sum_e dx dy sum_pq w_p w_q |u_h - u_ref| / area, per variable."""
    W2 = weights_2d(N)
    return (np.abs(u - uex) * W2).sum(axis=(1, 2, 3, 4)) * dx * dy / area


def l1_error_1d(u, uex, N, dx, length):
    _, w = oracle.gl(N)
    return (np.abs(u - uex) * w).sum(axis=(1, 2)) * dx / length
