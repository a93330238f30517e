"""Writes tests/golden/cfl.json: CFL(N) of the built scheme (GL points, Radau
correction, D2 dissipation, cRK of s stages) from the oracle's Fourier
analysis.  Calls only oracle/.  The paper does not print these numbers (it
refers to tables of earlier work for them, Sec. 5, eq. time.step.2d).

Two kinds per (N, s): "upwind" (dissipation speed = wave speed, a scalar
linear flux) and "system" (every ratio a/lambda in [0, 1], as for the fields
of a system under the Rusanov speed).  Tolerance on the spectral radius: 1e-12
for the linearly Lax-Wendroff equivalent pairs (N, s) = (1,2), (2,3), (3,4);
1e-5 for (4,4), whose amplification matrix has a weak growth below 5e-6 per
step up to a sharp knee.  For these pairs also the D1 values ("cfl_d1",
"cfl_system_d1"; eq. D1).  Further (N, s) pairs (the cRK stage count as an
option) with D2 and tolerance 1e-10.
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle.cfl import cfl_number, SYSTEM_RATIOS  # noqa: E402

PAIRS = [(1, 2, 1e-12), (2, 3, 1e-12), (3, 4, 1e-12), (4, 4, 1e-5)]
EXTRA = [(1, 3), (1, 4), (2, 2), (2, 4), (3, 2), (3, 3), (4, 2), (4, 3)]

if __name__ == "__main__":
    out = {}
    for N, s, tol in PAIRS:
        up = cfl_number(N, s, tol=tol, nk=2048, iters=48)
        sysv = cfl_number(N, s, tol=tol, nk=512, iters=40, ratios=SYSTEM_RATIOS)
        up1 = cfl_number(N, s, tol=tol, nk=2048, iters=48, d1=True)
        sys1 = cfl_number(N, s, tol=tol, nk=512, iters=40, ratios=SYSTEM_RATIOS, d1=True)
        out[f"{N},{s}"] = {"N": N, "stages": s, "tol": tol, "cfl": up, "cfl_system": sysv,
                           "cfl_d1": up1, "cfl_system_d1": sys1}
        print(N, s, up, sysv, up1, sys1, flush=True)
    for N, s in EXTRA:
        up = cfl_number(N, s, tol=1e-10, nk=1024, iters=44)
        sysv = cfl_number(N, s, tol=1e-10, nk=512, iters=40, ratios=SYSTEM_RATIOS)
        out[f"{N},{s}"] = {"N": N, "stages": s, "tol": 1e-10, "cfl": up, "cfl_system": sysv}
        print(N, s, up, sysv, flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfl.json"), "w") as f:
        json.dump(out, f, indent=1)
