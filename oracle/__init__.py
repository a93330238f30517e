"""Plain FP64 CPU oracle of one cRKFR step (Babbar & Chen, arXiv 2502.07517).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use it; the product path never does.  It shares no code with the
HIP library.  ``crkfr_oracle.c`` holds the arithmetic; this module is ctypes
marshalling plus the Fourier stability analysis in ``cfl.py``.
"""
from .oracle import (  # noqa: F401
    LINADV1D, EULER1D, EULER2D, TENMOM2D, BURGERS1D, TENMOM1D, PERIODIC, OUTFLOW, FARFIELD, REFLECT, INFLOW,
    DISS_D2, DISS_D1, DISS_DCSX, CENTRAL_EA, CENTRAL_AE, POINTS_GL, POINTS_GLL, step_crkfr_form,
    BLEND_OFF, BLEND_FO, BLEND_MH, IND_PAPER, IND_CONST, IND_GIVEN, IND_LEARNED,
    RefConfig, lib, build, gl, gll, nodes, diff_matrix, lagrange_at, legendre_orthonormal,
    tableau, flux, sigma, adm, nvar, nadm, local_crk, indicator_raw, indicator_features, learned_alpha,
    scale_element, compute_dt, lo_factor, flux_limit_face, mh_predict, step, means, mlp_forward, mlp_loss_grad,
    boundary_traces, has_farfield,
)
from .cfl import cfl_number, amplification_matrix  # noqa: F401
