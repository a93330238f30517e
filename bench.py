"""Benchmark of the cRKFR step on one MI355X.

Headline (`value`): the plain FP64 step of the 2D Euler isentropic vortex on
periodic [-5,5]^2, 512 x 512 elements, N = 3 (4,194,304 DoF), cRK44, EA
central flux with D2 dissipation, limiter off, the time step of eq.
time.step.2d computed on the device (C_s = 0.98, CFL(3) = 0.1); DoF*steps/s
over K graph-replayed steps after W warm-up steps, the state resident in
HBM.  This is the paper's arithmetic (FP64) on its 2D Euler N = 3 workload.

Beside it (extra keys):
  equal_occupancy_512  FP64 and FP32 bulk (FP64 means and admissibility
                       roots) at 512^2, limiter off and with the limiter chain
                       (MUSCL-Hancock blending, flux limiter, scaling);
  matched_l1           the FP32-bulk + learned-indicator + batched path
                       against plain FP64 at matched density L1 error on the
                       vortex sweep (limiter chain on, t = 2), DoF*steps/s of
                       each path interpolated in log-log at each L1 target;
  sweep_batch          the sweep's grids advanced together as one batch
                       (plus copies to fill the GPU), per-instance L1;
  c5_uneven_batch      256 uneven 4-quadrant instances (sides 64-512,
                       N = 2..4, FP32 bulk + learned indicator);
  roofline             the dominant kernel of the headline step against the
                       8 TB/s HBM peak at the algorithmic 64 B per DoF-step;
  cpu_baseline         the FP64 oracle on the host cores on a bounded sample
                       of the headline workload (all cores; one core beside).

Prints ONE JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_DEG = 3
DOM = (-5.0, 5.0, -5.0, 5.0)
CFL3 = 0.1          # CFL(3) for systems, 2/((N+1)(N+2)); checked against the library's Fourier analysis
HBM_PEAK = 8.0e12
FP64_VALU_PEAK = 78.6e12
# algorithmic HBM bytes per DoF and step: one read of u^n and one write of
# u^{n+1} (FP64: 2 x 4 variables x 8 B; FP32 bulk: 2 x 4 x 4 B + the FP64
# means read and written once per element of 16 points)
ALG_BYTES = {"fp64": 64.0, "mp32": 32.0 + 64.0 / 16.0}
# algorithmic flops per DoF and step of the high-order step (four stages of
# fluxes, local derivatives and stage updates, time averages, EA traces and
# face fluxes, volume term, numerical flux and correction; divides and square
# roots counted as one)
ALG_FLOPS = 800.0
TARGETS = (1e-4, 1e-5, 1e-6)
SWEEP = "12,16,24,32,48,64,96,128"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "vortex_512sq_n3_fp64_hbm_traffic.md")


KERNEL_SOURCES = ("crkfr_kernels.hpp", "crkfr_physics.hpp", "crkfr_launch.hpp", "crkfr_eq_euler2d.hip")


def kernel_sources_digest():
    """SHA-256 over the sources of the 2D Euler step's kernels and their
    launch shapes (file names and contents, in this order)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2502_07517_amd", "csrc")
    for fn in KERNEL_SOURCES:
        h.update(fn.encode())
        with open(os.path.join(d, fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes of the headline step from the committed counter summary, if
    it was taken on the current kernel sources (else None): per launch of the
    dominant kernel, and per whole step."""
    import re
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"sources_sha256: (\w+)", txt)
    k = re.search(r"dominant_kernel_bytes_per_launch: (\d+)", txt)
    s = re.search(r"step_bytes: (\d+)", txt)
    if not (m and k and s) or m.group(1) != kernel_sources_digest():
        return None
    return {"kernel": int(k.group(1)), "step": int(s.group(1))}


def gl_weights(N):
    _, w = np.polynomial.legendre.leggauss(N + 1)
    return 0.5 * w


def density_l1(state, n, t):
    """L1 = sum_e dx dy sum_pq w_p w_q |rho_h - rho_exact| / area."""
    from paper_2502_07517_amd import workloads as W
    X, Y = W.node_coords_2d(n, n, N_DEG, DOM)
    rho_ex = W.vortex_prim(X, Y, t, DOM)[0]
    w = gl_weights(N_DEG)
    W2 = np.outer(w, w)
    return float((np.abs(state[0] - rho_ex) * W2).sum() / (n * n))


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _limited(s, C, indicator, net=None):
    s.set_limiter(blend=C.BLEND_MH, indicator=indicator, flux_limiter=1, scaling=1)
    if net is not None:
        s.set_mlp(net)


# ---------------------------------------------------------------- the 512^2 single-instance step
def run_c3(dtype, steps, warmup, limited=False, path=None):
    """The 512^2 vortex step: graph-replayed steps for the rate, then the
    same number of eagerly enqueued steps with HIP events between the
    kernels on the solver's stream for the per-kernel times."""
    import torch
    from paper_2502_07517_amd import crkfr as C
    from paper_2502_07517_amd import workloads as W
    n = 512
    s = C.Solver(C.EULER2D, N_DEG, n, n, domain=DOM, dtype=dtype, cfl=CFL3,
                 stream=torch.cuda.current_stream().cuda_stream)
    if limited:
        _limited(s, C, C.IND_PAPER)
    if path is not None:
        s.set_path(path)
    s.set_state(torch.from_numpy(np.ascontiguousarray(W.vortex2d(n, N_DEG, 0.0, DOM))).to("cuda"))
    s.advance(0.0, warmup)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    s.advance(0.0, steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    s.set_timing(True)
    kt = np.zeros(4)
    for _ in range(steps):
        s.step(0.0)
        kt += np.array(s.kernel_times())
    kt /= steps
    s.set_timing(False)
    d, rc = s.get_diag()
    if rc != 0:
        raise RuntimeError(f"512^2 step ({dtype}, limited={limited}) failed: {d}")
    out = s.get_state()
    used = s.path_in_use()
    s.close()
    return {"ms_per_step": ms, "dofsteps_per_s": n * n * (N_DEG + 1) ** 2 / (ms * 1e-3),
            "kernel_ms": kt.tolist(), "state": out, "n_troubled_last": int(d["n_troubled"]),
            "path": ["split", "tile", "face_update", "checker"][used]}


# ---------------------------------------------------------------- learned indicator for 2D Euler
def train_network_for(N, seed=0):
    """A network for degree N from three 4-quadrant runs (32^2) and four
    element-pattern states (64^2), 40 epochs (the batch of uneven members)."""
    import torch
    from paper_2502_07517_amd import crkfr as C
    from paper_2502_07517_amd import learned as LI
    from paper_2502_07517_amd import workloads as W
    ff = (C.FARFIELD,) * 4
    runs = []
    for sd in range(3):
        s = C.Solver(C.EULER2D, N, 32, 32, bc=ff)
        s.set_limiter(blend=C.BLEND_MH, indicator=C.IND_PAPER, flux_limiter=1, scaling=1)
        s.set_state(W.euler2d_quadrants(sd, 32, N))
        runs.append(s)
    X1, y1 = LI.collect_pairs(runs, steps=80, every=2)
    ps = C.Solver(C.EULER2D, N, 64, 64, bc=ff)
    X2, y2 = LI.pairs_of_states(ps, [W.element_patterns_2d(500 + i, 64, 64, N) for i in range(4)])
    net, _ = LI.train_indicator(torch.cat([X1, X2]), torch.cat([y1, y2]), epochs=40, batch=2048, seed=seed + N)
    return net


def train_network(seed=0):
    """Training pairs from the method itself: snapshots of four 4-quadrant
    Riemann runs (64^2, smoothness indicator) and eight states of
    single-element patterns; trained with the library's GPU kernels."""
    import torch
    from paper_2502_07517_amd import crkfr as C
    from paper_2502_07517_amd import learned as LI
    from paper_2502_07517_amd import workloads as W
    t0 = time.perf_counter()
    ff = (C.FARFIELD,) * 4
    runs = []
    for sd in range(4):
        s = C.Solver(C.EULER2D, N_DEG, 64, 64, bc=ff, cfl=CFL3)
        s.set_limiter(blend=C.BLEND_MH, indicator=C.IND_PAPER, flux_limiter=1, scaling=1)
        s.set_state(W.euler2d_quadrants(sd, 64, N_DEG))
        runs.append(s)
    X1, y1 = LI.collect_pairs(runs, steps=150, every=3)
    ps = C.Solver(C.EULER2D, N_DEG, 128, 128, bc=ff, cfl=CFL3)
    X2, y2 = LI.pairs_of_states(ps, [W.element_patterns_2d(1000 + i, 128, 128, N_DEG) for i in range(8)])
    X, y = torch.cat([X1, X2]), torch.cat([y1, y2])
    net, hist = LI.train_indicator(X, y, epochs=60, batch=4096, lr=3e-3, seed=seed)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    held = []
    for sd in range(100, 102):
        s = C.Solver(C.EULER2D, N_DEG, 64, 64, bc=ff, cfl=CFL3)
        s.set_limiter(blend=C.BLEND_MH, indicator=C.IND_PAPER, flux_limiter=1, scaling=1)
        s.set_state(W.euler2d_quadrants(sd, 64, N_DEG))
        held.append(s)
    Xh, yh = LI.collect_pairs(held, steps=150, every=3)
    agree, mad = LI.agreement(net, Xh, yh)
    return net, {"rows": int(X.shape[0]), "epochs": 60, "final_loss": float(hist[-1]), "train_s": train_s,
                 "heldout_agreement": agree, "heldout_mean_abs_alpha_diff": mad}


# ---------------------------------------------------------------- the matched-L1 sweep
def run_plain(n, t_end, steps, warmup):
    """Plain FP64, one instance, smoothness indicator and limiter chain."""
    import torch
    from paper_2502_07517_amd import crkfr as C
    from paper_2502_07517_amd import workloads as W
    st = torch.cuda.current_stream().cuda_stream
    s = C.Solver(C.EULER2D, N_DEG, n, n, domain=DOM, dtype=C.FP64, cfl=CFL3, stream=st)
    _limited(s, C, C.IND_PAPER)
    s.set_state(torch.from_numpy(np.ascontiguousarray(W.vortex2d(n, N_DEG, 0.0, DOM))).to("cuda"))
    s.advance(t_end, warmup)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    s.advance(t_end, steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    s.advance(t_end, 10 ** 9)
    d, rc = s.get_diag()
    if rc != 0 or abs(d["t"] - t_end) > 1e-12:
        raise RuntimeError(f"plain run n={n} did not reach t_end: rc={rc} diag={d}")
    l1 = density_l1(s.get_state(), n, t_end)
    dof = n * n * (N_DEG + 1) ** 2
    s.close()
    return {"n": n, "copies": 1, "dof": dof, "ms_per_step": ms, "dofsteps_per_s": dof / (ms * 1e-3),
            "l1": l1, "steps_to_t_end": int(d["steps"])}


def _vortex_solver(C, n, net, st, dtype=None, indicator=None):
    import torch
    from paper_2502_07517_amd import workloads as W
    ind = C.IND_LEARNED if indicator is None else indicator
    s = C.Solver(C.EULER2D, N_DEG, n, n, domain=DOM, dtype=C.MP32 if dtype is None else dtype, cfl=CFL3,
                 stream=st)
    _limited(s, C, ind, net if ind == C.IND_LEARNED else None)
    s.set_state(torch.from_numpy(np.ascontiguousarray(W.vortex2d(n, N_DEG, 0.0, DOM))).to("cuda"))
    return s


def _run_batch_to(b, solvers, t_end, steps, warmup):
    """Timed steps of a batch, then the rest of the run to t_end."""
    import torch
    b.set_t_end(t_end)
    b.autotune(3)
    b.advance(warmup)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    b.advance(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    while True:
        b.advance(64)
        b.sync()
        done = True
        for s in solvers:
            d, rc = s.get_diag()
            if rc != 0:
                raise RuntimeError(f"batched run: {d}")
            done = done and d["t"] >= t_end
        if done:
            break
    return ms


def run_optimized(n, t_end, steps, warmup, net, fill_dof):
    """FP32 bulk + learned indicator + copies of the n^2 vortex batched to
    about fill_dof DoF."""
    import torch
    from paper_2502_07517_amd import crkfr as C
    st = torch.cuda.current_stream().cuda_stream
    dof1 = n * n * (N_DEG + 1) ** 2
    copies = max(1, int(round(fill_dof / dof1)))
    solvers = [_vortex_solver(C, n, net, st) for _ in range(copies)]
    b = C.Batch(solvers, stream=st)
    ms = _run_batch_to(b, solvers[:1] + solvers[-1:], t_end, steps, warmup)
    l1 = density_l1(solvers[0].get_state(), n, t_end)
    l1_last = density_l1(solvers[-1].get_state(), n, t_end)
    b.close()
    for s in solvers:
        s.close()
    return {"n": n, "copies": copies, "dof": dof1 * copies, "ms_per_step": ms,
            "dofsteps_per_s": dof1 * copies / (ms * 1e-3), "l1": l1, "l1_last_copy": l1_last}


def run_sweep_batch(sweep, t_end, steps, warmup, net, fill_dof):
    """The sweep's grids advanced together in one batch (FP32 bulk + learned
    indicator), repeated to about fill_dof DoF; aggregate DoF*steps/s while
    every member advances, and each grid's L1 at t_end."""
    import torch
    from paper_2502_07517_amd import crkfr as C
    st = torch.cuda.current_stream().cuda_stream
    set_dof = sum(n * n * (N_DEG + 1) ** 2 for n in sweep)
    reps = max(1, int(round(fill_dof / set_dof)))
    members = [(n, _vortex_solver(C, n, net, st)) for _ in range(reps) for n in sweep]
    solvers = [s for _, s in members]
    b = C.Batch(solvers, stream=st)
    ms = _run_batch_to(b, solvers, t_end, min(steps, 30), warmup)
    l1 = {str(n): density_l1(s.get_state(), n, t_end) for n, s in members[:len(sweep)]}
    b.close()
    for s in solvers:
        s.close()
    return {"grids": sweep, "repeats": reps, "instances": len(solvers), "dof": set_dof * reps,
            "ms_per_step": ms, "dofsteps_per_s": set_dof * reps / (ms * 1e-3),
            "timed_steps": min(steps, 30), "l1_first_set": l1}


def loglog_at(rows, target):
    """DoF*steps/s at an L1 target, interpolated linearly in (log L1, log
    rate) between the two consecutive sweep grids whose errors bracket it;
    None when no pair brackets it."""
    rows = sorted(rows, key=lambda r: r["n"])
    for a, b in zip(rows, rows[1:]):
        if a["l1"] >= target >= b["l1"] and a["l1"] > b["l1"]:
            f = (math.log(target) - math.log(a["l1"])) / (math.log(b["l1"]) - math.log(a["l1"]))
            lr = math.log(a["dofsteps_per_s"]) + f * (math.log(b["dofsteps_per_s"]) - math.log(a["dofsteps_per_s"]))
            return {"dofsteps_per_s": math.exp(lr), "between": [a["n"], b["n"]]}
    return None


def run_c5(nets, steps, warmup):
    """The batch of 256 uneven 2D Euler 4-quadrant instances (sides 64-512,
    N = 2, 3, 4; 4.3e8 DoF), FP32 bulk + learned indicator, autotuned,
    captured two-step graph replay; aggregate DoF*steps/s."""
    import torch
    from paper_2502_07517_amd import crkfr as C
    from paper_2502_07517_amd import workloads as W
    st = torch.cuda.current_stream().cuda_stream
    specs = W.batch_instances(2026, 256, sides=(64, 512), degrees=(2, 3, 4))
    solvers, dof = [], 0
    for sp in specs:
        n, N = sp["n"], sp["N"]
        s = C.Solver(C.EULER2D, N, n, n, bc=(C.FARFIELD,) * 4, dtype=C.MP32, stream=st)
        _limited(s, C, C.IND_LEARNED, nets[N])
        s.set_state(torch.from_numpy(np.ascontiguousarray(W.euler2d_quadrants(sp["seed"] % 1000, n, N))).to("cuda"))
        solvers.append(s)
        dof += n * n * (N + 1) ** 2
    b = C.Batch(solvers, stream=st)
    grids = b.autotune(2)
    b.advance(warmup)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    b.advance(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    b.set_timing(True)
    acc = np.zeros(4)
    for _ in range(4):
        b.advance(1)
        acc += np.array(b.phase_times())
    b.set_timing(False)
    b.sync()
    bad = sum(1 for s in solvers if s.get_diag()[1] != 0)
    b.close()
    for s in solvers:
        s.close()
    return {"instances": len(specs), "dof": dof, "ms_per_step": ms, "dofsteps_per_s": dof / (ms * 1e-3),
            "phase_ms": (acc / 4).tolist(), "grids": grids, "members_with_errors": bad,
            "steps": steps + warmup + 4}


# ---------------------------------------------------------------- CPU oracle baseline
def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds=12.0):
    """The FP64 oracle on the headline workload (512^2 vortex, N = 3,
    limiter off, fixed dt), steps until `seconds` have passed: first on
    every host thread OpenMP gives it, then on one."""
    import ctypes
    import oracle as O
    from paper_2502_07517_amd import workloads as W
    n = 512
    cfg = O.RefConfig.make(O.EULER2D, N_DEG, n, n, domain=DOM, cfl=CFL3)
    u0 = W.vortex2d(n, N_DEG, 0.0, DOM)
    dt = O.compute_dt(cfg, u0)
    dof = n * n * (N_DEG + 1) ** 2
    O.lib()
    gomp = ctypes.CDLL("libgomp.so.1")
    all_threads = int(gomp.omp_get_max_threads())
    res = {}
    for key, threads in (("all", all_threads), ("one", 1)):
        gomp.omp_set_num_threads(threads)
        u = u0
        t0 = time.perf_counter()
        k = 0
        while True:
            u, _, _, _ = O.step(cfg, u, dt)
            k += 1
            if time.perf_counter() - t0 > seconds:
                break
        el = time.perf_counter() - t0
        res[key] = {"value": dof * k / el, "threads": threads, "steps": k, "seconds": el}
    gomp.omp_set_num_threads(all_threads)
    return {"value": res["all"]["value"], "unit": "DoF*steps/s", "cores": all_threads, "kind": "oracle",
            "sample": f"{res['all']['steps']} FP64 oracle steps of the headline workload (512^2 vortex, N=3, "
                      f"limiter off, fixed dt) on {all_threads} threads in {res['all']['seconds']:.1f} s",
            "single_thread": res["one"], "cpu_model": cpu_model()}


PHASES = ("local", "x faces", "y faces", "update")
# the four timed intervals of a step on each kernel path, and the fraction of
# the DoF each kernel carries the whole step for (the units of its
# algorithmic bytes): the checkerboard step's colour-1 kernel takes its half
# of the elements from u^n to u^{n+1}
PATH_KERNELS = {
    "split": (("k_local", 1.0), ("k_face x", 1.0), ("k_face y", 1.0), ("k_update", 1.0)),
    "tile": (("k_tile", 1.0), ("k_tile_face x", 1.0), ("k_tile_face y", 1.0), ("k_update (tile edges)", 1.0)),
    "face_update": (("k_local", 1.0), ("-", 0.0), ("-", 0.0), ("k_update (faces fused)", 1.0)),
    "checker": (("k_cb_local (colour 0)", 0.5), ("k_cb_white (colour 1: local, faces, update)", 0.5),
                ("-", 0.0), ("k_cb_update (colour 0)", 0.5)),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--t-end", type=float, default=2.0)
    ap.add_argument("--sweep", default=SWEEP)
    ap.add_argument("--fill-dof", type=float, default=4.2e6)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="seconds per CPU-baseline leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the 256-instance uneven batch")
    ap.add_argument("--part", choices=["all", "c3", "c3head", "c3lim", "sweep", "c5"], default="all",
                    help="c3: only the 512^2 step on each kernel path; c3head: only the headline path "
                         "(counter runs); c3lim: only the 512^2 steps with the limiter chain; sweep: only the "
                         "matched-L1 sweep; c5: only the uneven batch (profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver has no multi-GPU path, run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
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

    from paper_2502_07517_amd import crkfr as C
    lib_cfl = C.fourier_cfl(N_DEG, 0, 1, 1e-10)
    assert abs(lib_cfl - CFL3) < 1e-6, lib_cfl
    sweep = [int(v) for v in args.sweep.split(",")]
    dof512 = 512 * 512 * (N_DEG + 1) ** 2

    def c3_row(r):
        return {k: v for k, v in r.items() if k != "state"}

    if args.part == "c3lim":
        out = {}
        for k, dt in (("fp64_limited", C.FP64), ("mp32_limited", C.MP32)):
            for name, pth in (("", None), ("_split", C.PATH_SPLIT), ("_face_update", C.PATH_FACE_UPDATE)):
                r = c3_row(run_c3(dt, args.steps, args.warmup, limited=True, path=pth))
                out[k + name] = r
                print(f"# 512^2 {k}{name} ({r['path']}): {r['ms_per_step']:.4f} ms/step, kernels (ms) "
                      f"{np.round(r['kernel_ms'], 4).tolist()}", flush=True)
        print(json.dumps({"part": "c3lim", "equal_occupancy_512": out}), flush=True)
        return
    if args.part == "c3head":
        r = run_c3(C.FP64, args.steps, args.warmup)
        print(f"# 512^2 FP64 limiter off ({r['path']}): {r['ms_per_step']:.4f} ms/step, kernels (ms) "
              f"{np.round(r['kernel_ms'], 4).tolist()}", flush=True)
        return
    if args.part == "c5":
        nets = {3: train_network()[0]}
        nets.update({N: train_network_for(N) for N in (2, 4)})
        print(json.dumps({"part": "c5", "c5": run_c5(nets, args.steps, args.warmup)}), flush=True)
        return
    if args.part == "sweep":
        net, train = train_network()
        plain = [run_plain(n, args.t_end, 20, 2) for n in sweep]
        opt = [run_optimized(n, args.t_end, 20, 2, net, args.fill_dof) for n in sweep]
        print(json.dumps({"part": "sweep", "plain": plain, "optimized": opt}), flush=True)
        return

    # ---- headline: the plain FP64 512^2 step, limiter off
    head = run_c3(C.FP64, args.steps, args.warmup)
    print(f"# 512^2 FP64 limiter off ({head['path']}): {head['ms_per_step']:.4f} ms/step, kernels (ms) "
          f"{np.round(head['kernel_ms'], 4).tolist()}", flush=True)
    kms = head["kernel_ms"]
    dom = int(np.argmax(kms))
    k_ms = kms[dom]
    kname, share = PATH_KERNELS[head["path"]][dom]
    alg_step = ALG_BYTES["fp64"] * dof512
    alg = alg_step * share            # the DoF this launch takes through the whole step
    traffic = recorded_traffic()
    roofline = {"bound": "hbm", "kernel": kname, "achieved": alg / (k_ms * 1e-3) / 1e9,
                "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": alg / (k_ms * 1e-3) / HBM_PEAK,
                "traffic": None if traffic is None else traffic["kernel"],
                "algorithmic_bytes_per_launch": alg, "dof_per_launch": dof512 * share, "avg_ms": k_ms,
                "alu": {"peak_tflops": FP64_VALU_PEAK / 1e12,
                        "achieved_tflops": ALG_FLOPS * dof512 * share / (k_ms * 1e-3) / 1e12,
                        "frac": ALG_FLOPS * dof512 * share / (k_ms * 1e-3) / FP64_VALU_PEAK},
                "whole_step": {"hbm_frac": alg_step / (head["ms_per_step"] * 1e-3) / HBM_PEAK,
                               "alu_frac": ALG_FLOPS * dof512 / (head["ms_per_step"] * 1e-3) / FP64_VALU_PEAK,
                               "measured_bytes": None if traffic is None else traffic["step"],
                               "measured_over_algorithmic": None if traffic is None else traffic["step"] / alg_step}}
    line = {
        "metric": "DoF·steps/s, 2D Euler N=3: FP32/learned/batched vs plain FP64 at matched L1",
        "value": head["dofsteps_per_s"],
        "unit": "DoF*steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: isentropic vortex initial condition sampled at the Gauss-Legendre points",
        "config": {"workload": "2D Euler isentropic vortex, periodic [-5,5]^2, 512x512 elements, N=3 "
                               "(4,194,304 DoF), cRK44, EA central flux with D2 dissipation, limiter off, FP64, "
                               "device time step (C_s 0.98, CFL 0.1), graph-replayed steps",
                   "elements": 512 * 512, "dof": dof512, "N": N_DEG, "kernel_path": head["path"]},
        "kernel_ms": {n: t for (n, _), t in zip(PATH_KERNELS[head["path"]], kms) if n != "-"},
        "roofline": roofline,
    }
    # the other kernel paths of the same step (crkfr_set_path), for comparison
    line["other_paths_512"] = {}
    for name, pth in (("split", C.PATH_SPLIT), ("tile", C.PATH_TILE), ("face_update", C.PATH_FACE_UPDATE),
                      ("checker", C.PATH_CHECKER)):
        if name == head["path"]:
            continue
        r = run_c3(C.FP64, args.steps, args.warmup, path=pth)
        row = {k: v for k, v in r.items() if k != "state"}
        row["rel_linf_vs_headline"] = float(np.abs(r["state"] - head["state"]).max() / np.abs(head["state"]).max())
        line["other_paths_512"][name] = row
        print(f"# 512^2 FP64 {name}: {r['ms_per_step']:.4f} ms/step, kernels (ms) "
              f"{np.round(r['kernel_ms'], 4).tolist()}", flush=True)
    if args.part == "c3":
        print(json.dumps(line), flush=True)
        return

    # ---- equal occupancy at 512^2: FP64 vs FP32 bulk, limiter off and on
    eq = {"fp64": c3_row(head)}
    mp = run_c3(C.MP32, args.steps, args.warmup)
    eq["mp32"] = c3_row(mp)
    eq["mp32"]["rel_l1_vs_fp64"] = float(np.abs(mp["state"] - head["state"]).sum() / np.abs(head["state"]).sum())
    for key, dt in (("fp64_limited", C.FP64), ("mp32_limited", C.MP32)):
        eq[key] = c3_row(run_c3(dt, args.steps, args.warmup, limited=True))
    for k, v in eq.items():
        print(f"# 512^2 {k}: {v['ms_per_step']:.4f} ms/step", flush=True)
    line["equal_occupancy_512"] = eq

    # ---- matched L1: FP32 bulk + learned + batched vs plain FP64
    net, train = train_network()
    print(f"# learned indicator: {train}", flush=True)
    plain, opt = [], []
    for n in sweep:
        plain.append(run_plain(n, args.t_end, 20, 2))
        opt.append(run_optimized(n, args.t_end, 20, 2, net, args.fill_dof))
        print(f"# sweep n={n}: plain {plain[-1]['dofsteps_per_s']:.3e} L1 {plain[-1]['l1']:.3e} | optimized "
              f"x{opt[-1]['copies']} {opt[-1]['dofsteps_per_s']:.3e} L1 {opt[-1]['l1']:.3e}", flush=True)
    per_target = {}
    for tau in TARGETS:
        p, o = loglog_at(plain, tau), loglog_at(opt, tau)
        per_target[f"{tau:g}"] = {"plain_fp64": p, "fp32_learned_batched": o,
                                  "speedup": None if (p is None or o is None)
                                  else o["dofsteps_per_s"] / p["dofsteps_per_s"]}
    line["matched_l1"] = {"targets": per_target,
                          "fp32_bulk_l1_floor": min(r["l1"] for r in opt),
                          "note": "speed-up at a target mostly measures batching small grids: compare "
                                  "equal_occupancy_512 for the arithmetic alone"}
    line["sweep"] = {"plain": plain, "optimized": opt}
    line["sweep_batch"] = run_sweep_batch([n for n in sweep if n >= 32], args.t_end, args.steps, 2, net,
                                          args.fill_dof)
    line["learned_indicator"] = dict(train, note="against the smoothness indicator it gains no accuracy (density "
                                     "L1 within 1.1x either way on held-out runs) and costs the network on top of "
                                     "the same modal energies, about 12 % of the limited local phase")
    if not args.no_c5:
        nets = {3: net}
        nets.update({N: train_network_for(N) for N in (2, 4)})
        c5 = run_c5(nets, 20, 2)
        print(f"# c5 batch: {c5['instances']} instances, {c5['dof']:.3e} DoF, {c5['dofsteps_per_s']:.3e} "
              f"DoF*steps/s, phases {np.round(c5['phase_ms'], 3).tolist()}", flush=True)
        line["c5_uneven_batch"] = c5
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
