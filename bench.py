"""Benchmark of one cRKFR step on one MI355X.

Workload: 2D Euler isentropic vortex on periodic [-5,5]^2, 512 x 512 elements,
N = 3 (16 Gauss-Legendre points per element, 4,194,304 DoF), cRK44, EA central
flux with D2 dissipation, limiter off (smooth problem), time step of eq.
time.step.2d computed on the device every step.  A "step" is one full
cRKFR step over the grid.  The state is resident in HBM before the timed
region starts.

Prints ONE JSON line: the plain FP64 path is `value`; the FP32-bulk path
(FP64 means and admissibility roots) is reported beside it with its
deviation from the FP64 result.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_DEG, N_EL = 3, 512
DOM = (-5.0, 5.0, -5.0, 5.0)
HBM_PEAK = 8.0e12
FP64_PEAK = 78.6e12


def kernel_bytes_per_node(M, N, dtype_bytes, dim=2):
    """Compulsory HBM bytes of k_local per solution point: read u, write the
    partial update and the face traces (F_EA, U, sigma per face point)."""
    nd = N + 1
    np_ = nd ** dim
    face_pts = 2 * dim * nd ** (dim - 1)
    trace_vals = face_pts * (2 * M + 1)
    return dtype_bytes * (2 * M + trace_vals / np_)


def run_gpu(dtype, steps, warmup, u0, cfl):
    import torch  # device memory and streams only
    from paper_2502_07517_amd import crkfr as C
    s = C.Solver(C.EULER2D, N_DEG, N_EL, N_EL, domain=DOM, dtype=dtype, cfl=cfl,
                 stream=torch.cuda.current_stream().cuda_stream)
    dev = torch.from_numpy(u0).to("cuda")
    s.set_state(dev)
    for _ in range(warmup):
        s.step(0.0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        s.step(0.0)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    d, rc = s.get_diag()
    out = s.get_state()
    # per-kernel device times with HIP events on the solver's stream
    s.set_timing(True)
    kt = np.zeros(4)
    nk = max(5, min(steps, 20))
    for _ in range(nk):
        s.step(0.0)
        kt += np.array(s.kernel_times())
    kt /= nk
    s.close()
    return {"ms_per_step": ms / steps, "wall_ms_per_step": 1e3 * wall / steps, "diag": d, "rc": rc,
            "state": out, "kernel_ms": kt.tolist()}


def cpu_baseline(u0, cfl, steps):
    import oracle as O
    cfg = O.RefConfig.make(O.EULER2D, N_DEG, N_EL, N_EL, domain=DOM, cfl=cfl)
    u = u0
    dt = O.compute_dt(cfg, u)
    t0 = time.perf_counter()
    for _ in range(steps):
        u, _, _, _ = O.step(cfg, u, dt)
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": N_EL * N_EL * (N_DEG + 1) ** 2 * steps / el, "unit": "DoF*steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{steps} FP64 oracle steps of the same 512x512 N=3 vortex (fixed dt), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["fp64", "mp32", "both"], default="both")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        a.fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copied 3 x 1 GiB", flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    from paper_2502_07517_amd import crkfr as C
    from paper_2502_07517_amd import workloads as W
    cfl = 0.1   # CFL(3) for systems: 2/((N+1)(N+2)); checked against the library's Fourier analysis
    lib_cfl = C.fourier_cfl(N_DEG, 0, 1, 1e-10)
    assert abs(lib_cfl - cfl) < 1e-6, lib_cfl
    u0 = np.ascontiguousarray(W.vortex2d(N_EL, N_DEG, 0.0, DOM))
    dof = N_EL * N_EL * (N_DEG + 1) ** 2
    res = {}
    if args.only in ("fp64", "both"):
        res["fp64"] = run_gpu(C.FP64, args.steps, args.warmup, u0, cfl)
        print(f"# fp64 {res['fp64']['ms_per_step']:.4f} ms/step kernels {res['fp64']['kernel_ms']}", flush=True)
    if args.only in ("mp32", "both"):
        res["mp32"] = run_gpu(C.MP32, args.steps, args.warmup, u0, cfl)
        print(f"# mp32 {res['mp32']['ms_per_step']:.4f} ms/step kernels {res['mp32']['kernel_ms']}", flush=True)

    main_key = "fp64" if "fp64" in res else "mp32"
    r = res[main_key]
    value = dof / (r["ms_per_step"] * 1e-3)
    M = 4
    rb = 8 if main_key == "fp64" else 4
    kb = kernel_bytes_per_node(M, N_DEG, rb) * dof
    k_ms = r["kernel_ms"][0]
    achieved = kb / (k_ms * 1e-3)
    line = {
        "metric": "DoF*steps/s, 2D Euler N=3 (cRKFR step)",
        "value": value,
        "unit": "DoF*steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if main_key == "fp64" else "f32 bulk + f64 means/roots",
        "data": "synthetic (isentropic vortex initial condition)",
        "config": {"workload": "2D Euler isentropic vortex, periodic [-5,5]^2, 512x512 elements, N=3, cRK44, "
                               "EA/D2 flux, limiter off, device dt (C_s=0.98, CFL=0.1)",
                   "elements": N_EL * N_EL, "dof": dof, "N": N_DEG},
        "roofline": {"bound": "hbm", "kernel": "k_local", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": None,
                     "algorithmic_bytes_per_launch": kb, "avg_ms": k_ms},
        "kernel_ms": {"local": r["kernel_ms"][0], "face_x": r["kernel_ms"][1], "face_y": r["kernel_ms"][2],
                      "update": r["kernel_ms"][3]},
        "step_effective_GBps_at_64B_per_dof": 64 * dof / (r["ms_per_step"] * 1e-3) / 1e9,
    }
    if "fp64" in res and "mp32" in res:
        a, b = res["fp64"]["state"], res["mp32"]["state"]
        line["mp32"] = {"value": dof / (res["mp32"]["ms_per_step"] * 1e-3),
                        "ms_per_step": res["mp32"]["ms_per_step"],
                        "rel_l1_vs_fp64": float(np.abs(a - b).sum() / np.abs(a).sum()),
                        "kernel_ms": res["mp32"]["kernel_ms"]}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(u0, cfl, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
