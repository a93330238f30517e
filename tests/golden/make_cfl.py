"""Writes tests/golden/cfl.json: CFL(N) of the built scheme (Radau correction
with GL points, or g2 with GLL points; D2 dissipation; cRK of s stages) from
the oracle's Fourier analysis.  Calls only oracle/.  The paper does not print
these numbers (it refers to tables of earlier work for them, Sec. 5, eq.
time.step.2d).

Two kinds per (N, s): "upwind" (dissipation speed = wave speed, a scalar
linear flux) and "system" (every ratio a/lambda in [0, 1], as for the fields
of a system under the Rusanov speed).  Tolerance on the spectral radius: 1e-12
for the linearly Lax-Wendroff equivalent pairs (N, s) = (1,2), (2,3), (3,4);
1e-5 for (4,4), whose amplification matrix has a weak growth below 5e-6 per
step up to a sharp knee.  For these pairs also the D1 values ("cfl_d1",
"cfl_system_d1"; eq. D1) and the GLL/g2 values ("cfl_gll",
"cfl_system_gll").  Further (N, s) pairs (the cRK stage count as an option)
with D2 and tolerance 1e-10.  Existing entries are kept; only missing values
are computed.
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle.cfl import cfl_number, SYSTEM_RATIOS  # noqa: E402

PAIRS = [(1, 2, 1e-12), (2, 3, 1e-12), (3, 4, 1e-12), (4, 4, 1e-5)]
EXTRA = [(1, 3), (1, 4), (2, 2), (2, 4), (3, 2), (3, 3), (4, 2), (4, 3)]
PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfl.json")


def _kinds(tol):
    up = dict(tol=tol, nk=2048, iters=48)
    sy = dict(tol=tol, nk=512, iters=40, ratios=SYSTEM_RATIOS)
    return {"cfl": up, "cfl_system": sy,
            "cfl_d1": dict(up, d1=True), "cfl_system_d1": dict(sy, d1=True),
            "cfl_gll": dict(up, points=1), "cfl_system_gll": dict(sy, points=1)}


if __name__ == "__main__":
    out = json.load(open(PATH)) if os.path.exists(PATH) else {}
    for N, s, tol in PAIRS:
        e = out.setdefault(f"{N},{s}", {"N": N, "stages": s, "tol": tol})
        for kind, kw in _kinds(tol).items():
            if kind not in e:
                e[kind] = cfl_number(N, s, **kw)
                print(N, s, kind, e[kind], flush=True)
    for N, s in EXTRA:
        e = out.setdefault(f"{N},{s}", {"N": N, "stages": s, "tol": 1e-10})
        for kind, kw in (("cfl", dict(tol=1e-10, nk=1024, iters=44)),
                         ("cfl_system", dict(tol=1e-10, nk=512, iters=40, ratios=SYSTEM_RATIOS))):
            if kind not in e:
                e[kind] = cfl_number(N, s, **kw)
                print(N, s, kind, e[kind], flush=True)
    with open(PATH, "w") as f:
        json.dump(out, f, indent=1)
