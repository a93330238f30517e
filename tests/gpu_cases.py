"""Matching oracle / GPU runs for the parity tests (test helper)."""
import numpy as np

import oracle as O
from paper_2502_07517_amd import crkfr as C
from paper_2502_07517_amd import workloads as W
from oracle_runs import cfl_for


def make_pair(eq, N, nx, ny=1, *, bc=None, domain=(0.0, 1.0, 0.0, 1.0), dtype=C.FP64, blend=0,
              indicator=0, flux_limiter=0, scaling=0, alpha_const=0.0, source=None, smooth_nbr=1):
    bc = bc if bc is not None else (C.PERIODIC,) * 4
    system = eq != C.LINADV1D
    cfl = cfl_for(N, system=system)
    ref = O.RefConfig.make(eq, N, nx, ny, bc=bc, domain=domain, cfl=cfl, blend=blend, indicator=indicator,
                           flux_limiter=flux_limiter, scaling=scaling, alpha_const=alpha_const,
                           smooth_nbr=smooth_nbr, source=1 if source else 0,
                           src=source[:4] if source else (0, 0, 0, 0),
                           src_lin=source[4:] if source else (0, 0))
    gpu = C.Solver(eq, N, nx, ny, bc=bc, domain=domain, dtype=dtype, cfl=cfl)
    gpu.set_limiter(blend=blend, indicator=indicator, smooth_nbr=smooth_nbr, flux_limiter=flux_limiter,
                    scaling=scaling, alpha_const=alpha_const)
    if source:
        gpu.set_source(1, *source)
    return ref, gpu


def run_pair(ref, gpu, u0, steps, dt=None, alpha=None):
    """Advance both with the same fixed dt; returns (u_oracle, u_gpu, diags, dt)."""
    if dt is None:
        dt = O.compute_dt(ref, u0)
    ghost = O.boundary_traces(ref, u0) if O.has_farfield(ref) else None
    u = np.ascontiguousarray(u0, dtype=np.float64)
    gpu.set_state(u.copy())
    if alpha is not None:
        gpu.set_alpha(alpha)
    diags = []
    for _ in range(steps):
        u, a, d, st = O.step(ref, u, dt, alpha_given=alpha, ghost=ghost)
        gpu.step(dt)
        diags.append((d, gpu.get_diag()[0]))
    ug = gpu.get_state()
    return u, ug.reshape(u.shape), diags, dt


def rel_linf(a, b):
    return np.abs(a - b).max() / max(np.abs(a).max(), 1e-300)


def rel_l1(a, b):
    return np.abs(a - b).sum() / max(np.abs(a).sum(), 1e-300)
