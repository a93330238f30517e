"""Benchmark of the cRKFR step on one MI355X: FP32-bulk + learned indicator +
batched versus plain FP64, at matched L1 error.

Workload (2D Euler N=3): the isentropic vortex on periodic [-5,5]^2 (beta 5,
Mach 0.5, 45 degrees, gamma 1.4), cRK44, EA central flux with D2
dissipation, the limiter chain active (MUSCL-Hancock subcell blending, flux
limiter, scaling limiter), time step of eq. time.step.2d computed on the
device (C_s = 0.98, CFL(3) = 0.1), run to t = 2 on n x n grids for n in a
sweep.  Two paths run each grid:

  plain      FP64, one instance, the smoothness indicator;
  optimized  FP32 bulk with FP64 means and admissibility roots, the learned
             indicator (a network trained on the GPU beforehand on blending
             coefficients the method produces), and copies of the instance
             advanced together as one batch (graph-replayed steps) filling
             the GPU to about 4.2M DoF.

Both report DoF*steps/s over K timed steps after W warm-up steps (state in
HBM), and the density L1 error against the exact solution at t = 2.  For an
L1 target the matched grid of each path is the smallest sweep grid whose
error meets it; `value` is the optimized path's throughput on its matched
grid for L1 = 1e-5, with the plain path's throughput on its own matched grid
beside it.  The single-instance 512^2 step (limiter off) is reported too,
with its kernel times.

Prints ONE JSON line.
"""
import argparse
import json
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
TARGETS = (1e-4, 1e-5, 1e-6)
HEADLINE_TARGET = 1e-5


def local_bytes_per_node(M, N, real_bytes, lim, mp, dim=2):
    """Algorithmic HBM bytes of the local kernel per solution point: read the
    state (MP32: deviations + the element's FP64 means), write the partial
    update and the face traces (F_EA, U, sigma per face point; with limiting
    also the predicted subcell face value and the adjacent subface flux), and
    with limiting the element's blending coefficient (FP64)."""
    nd = N + 1
    np_ = nd ** dim
    face_pts = 2 * dim * nd ** (dim - 1)
    comps = 4 * M + 1 if lim else 2 * M + 1
    b = real_bytes * (2 * M + face_pts * comps / np_)
    if mp:
        b += 8 * M / np_
    if lim:
        b += 8 / np_
    return b


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_batch_local_mp32_limited_vortex_32sq_x256_hbm_traffic.md")


def kernel_sources_digest():
    """SHA-256 over the HIP sources (file names and contents, sorted)."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2502_07517_amd", "csrc")
    for fn in sorted(os.listdir(d)):
        h.update(fn.encode())
        with open(os.path.join(d, fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(grid, copies):
    """HBM bytes per launch of the batched local phase from the committed
    counter summary, if it was taken on the current kernel sources and the
    same batch (else None)."""
    import re
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"sources_sha256: (\w+)", txt)
    t = re.search(r"traffic_bytes_per_launch: (\d+)", txt)
    w = re.search(r"batch: (\d+) x (\d+)\^2", txt)
    if not (m and t and w) or m.group(1) != kernel_sources_digest():
        return None
    if int(w.group(1)) != copies or int(w.group(2)) != grid:
        return None
    return int(t.group(1))


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


# ---------------------------------------------------------------- the 512^2 single-instance step
def run_c3(dtype, steps, warmup, limited=False):
    import torch
    from paper_2502_07517_amd import crkfr as C
    from paper_2502_07517_amd import workloads as W
    n = 512
    s = C.Solver(C.EULER2D, N_DEG, n, n, domain=DOM, dtype=dtype, cfl=CFL3,
                 stream=torch.cuda.current_stream().cuda_stream)
    if limited:
        _limited(s, C, C.IND_PAPER)
    s.set_state(torch.from_numpy(np.ascontiguousarray(W.vortex2d(n, N_DEG, 0.0, DOM))).to("cuda"))
    for _ in range(warmup):
        s.step(0.0)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for _ in range(steps):
        s.step(0.0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    s.set_timing(True)
    kt = np.zeros(4)
    nk = max(5, min(steps, 20))
    for _ in range(nk):
        s.step(0.0)
        kt += np.array(s.kernel_times())
    kt /= nk
    out = s.get_state()
    s.close()
    return {"ms_per_step": ms, "kernel_ms": kt.tolist(), "state": out}


# ---------------------------------------------------------------- learned indicator for 2D Euler N=3
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
    # held-out quadrant runs
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


# ---------------------------------------------------------------- the sweep
def _limited(s, C, indicator, net=None):
    s.set_limiter(blend=C.BLEND_MH, indicator=indicator, flux_limiter=1, scaling=1)
    if net is not None:
        s.set_mlp(net)


def run_plain(n, t_end, steps, warmup):
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
            "l1": l1, "steps_to_t_end": int(d["steps"]), "n_troubled_last": int(d["n_troubled"])}


def run_optimized(n, t_end, steps, warmup, net, fill_dof, phase_timing=True, dtype=None, indicator=None):
    """Batched copies of the n^2 vortex; by default FP32 bulk + the learned
    indicator (other arithmetic / indicator for the speed-up decomposition)."""
    import torch
    from paper_2502_07517_amd import crkfr as C
    from paper_2502_07517_amd import workloads as W
    st = torch.cuda.current_stream().cuda_stream
    dof1 = n * n * (N_DEG + 1) ** 2
    copies = max(1, int(round(fill_dof / dof1)))
    u0 = torch.from_numpy(np.ascontiguousarray(W.vortex2d(n, N_DEG, 0.0, DOM))).to("cuda")
    solvers = []
    for _ in range(copies):
        dt_ = C.MP32 if dtype is None else dtype
        ind = C.IND_LEARNED if indicator is None else indicator
        s = C.Solver(C.EULER2D, N_DEG, n, n, domain=DOM, dtype=dt_, cfl=CFL3, stream=st)
        _limited(s, C, ind, net if ind == C.IND_LEARNED else None)
        s.set_state(u0)
        solvers.append(s)
    b = C.Batch(solvers, stream=st)
    b.set_t_end(t_end)
    grids = b.autotune(3)
    b.advance(warmup)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    b.advance(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    phase = None
    if phase_timing:
        # per-phase device times with HIP events on the batch stream, same steps
        b.set_timing(True)
        acc = np.zeros(4)
        k = 10
        for _ in range(k):
            b.advance(1)
            acc += np.array(b.phase_times())
        b.set_timing(False)
        phase = (acc / k).tolist()
    while True:
        b.advance(64)
        b.sync()
        d, rc = solvers[0].get_diag()
        if rc != 0:
            raise RuntimeError(f"optimized run n={n}: {d}")
        if d["t"] >= t_end:
            break
    d_last, rc_last = solvers[-1].get_diag()
    l1 = density_l1(solvers[0].get_state(), n, t_end)
    l1_last = density_l1(solvers[-1].get_state(), n, t_end)
    b.close()
    for s in solvers:
        s.close()
    return {"n": n, "copies": copies, "dof": dof1 * copies, "ms_per_step": ms,
            "dofsteps_per_s": dof1 * copies / (ms * 1e-3), "l1": l1, "l1_last_copy": l1_last,
            "phase_ms": phase, "grids": grids, "n_learned_fallback_last": int(d["n_learned_fallback"]),
            "n_troubled_last": int(d["n_troubled"])}


def matched(rows, target):
    """Smallest sweep grid whose L1 meets the target (None if none does)."""
    ok = [r for r in rows if r["l1"] <= target]
    return min(ok, key=lambda r: r["n"]) if ok else None


# ---------------------------------------------------------------- CPU oracle baseline
def cpu_baseline(n, t_end, max_steps):
    import oracle as O
    from paper_2502_07517_amd import workloads as W
    cfg = O.RefConfig.make(O.EULER2D, N_DEG, n, n, domain=DOM, cfl=CFL3, blend=O.BLEND_MH,
                           indicator=O.IND_PAPER, flux_limiter=1, scaling=1)
    u = W.vortex2d(n, N_DEG, 0.0, DOM)
    dt = O.compute_dt(cfg, u)
    t0 = time.perf_counter()
    k = 0
    while k < max_steps:
        u, _, _, _ = O.step(cfg, u, dt)
        k += 1
        if time.perf_counter() - t0 > 15.0:
            break
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    dof = n * n * (N_DEG + 1) ** 2
    return {"value": dof * k / el, "unit": "DoF*steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} FP64 oracle steps of the same vortex at {n}x{n}, N=3, limiter chain on "
                      f"(fixed dt), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--t-end", type=float, default=2.0)
    ap.add_argument("--sweep", default="8,12,16,24,32,48,64,96,128,192,256")
    ap.add_argument("--fill-dof", type=float, default=4.2e6)
    ap.add_argument("--cpu-steps", type=int, default=1000000,
                    help="cap on the oracle's steps (the CPU leg also stops after 15 s)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the 256-instance uneven batch")
    ap.add_argument("--part", choices=["all", "sweep", "c3", "optimized", "c5"], default="all",
                    help="c3: only the 512^2 single-instance step; optimized: only the optimized path "
                         "on the --sweep grids; c5: only the 256-instance uneven batch (profiling)")
    ap.add_argument("--c3-limiter", action="store_true",
                    help="also run the 512^2 step with the limiter chain (smoothness indicator)")
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
        print("bench.py measures one GPU: the solver has no multi-GPU path, run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2502_07517_amd import crkfr as C
    lib_cfl = C.fourier_cfl(N_DEG, 0, 1, 1e-10)
    assert abs(lib_cfl - CFL3) < 1e-6, lib_cfl
    sweep = [int(v) for v in args.sweep.split(",")]
    line = {}

    if args.part == "c5":
        nets = {3: train_network()[0]}
        nets.update({N: train_network_for(N) for N in (2, 4)})
        print(json.dumps({"part": "c5", "c5": run_c5(nets, args.steps, args.warmup)}), flush=True)
        return

    c3 = {}
    if args.part in ("all", "c3"):
        for key, dt in (("fp64", C.FP64), ("mp32", C.MP32)):
            c3[key] = run_c3(dt, args.steps, args.warmup)
            if args.c3_limiter:
                c3[key + "_limited"] = run_c3(dt, args.steps, args.warmup, limited=True)
            print(f"# c3 512^2 {key}: {c3[key]['ms_per_step']:.4f} ms/step kernels "
                  f"{np.round(c3[key]['kernel_ms'], 4).tolist()}", flush=True)

    plain, opt, train = [], [], None
    if args.part in ("all", "sweep", "optimized"):
        net, train = train_network()
        print(f"# learned indicator: {train}", flush=True)
        for n in sweep:
            if args.part != "optimized":
                plain.append(run_plain(n, args.t_end, args.steps, args.warmup))
                r = plain[-1]
                print(f"# plain n={n}: {r['dofsteps_per_s']:.3e} DoF*steps/s  L1 {r['l1']:.3e}  "
                      f"steps {r['steps_to_t_end']}", flush=True)
            opt.append(run_optimized(n, args.t_end, args.steps, args.warmup, net, args.fill_dof))
            r = opt[-1]
            print(f"# optimized n={n} x{r['copies']}: {r['dofsteps_per_s']:.3e} DoF*steps/s  L1 {r['l1']:.3e}  "
                  f"phases {np.round(r['phase_ms'], 4).tolist()}", flush=True)

    if args.part in ("c3", "optimized"):
        print(json.dumps({"part": args.part, "c3": {k: {kk: vv for kk, vv in v.items() if kk != "state"}
                                                  for k, v in c3.items()}, "optimized": opt}), flush=True)
        return

    c5 = None
    if args.part == "all" and not args.no_c5:
        nets = {3: net}
        nets.update({N: train_network_for(N) for N in (2, 4)})
        c5 = run_c5(nets, 20, 2)
        print(f"# c5 batch: {c5['instances']} instances, {c5['dof']:.3e} DoF, {c5['dofsteps_per_s']:.3e} DoF*steps/s, "
              f"phases {np.round(c5['phase_ms'], 3).tolist()}", flush=True)

    # decomposition of the speed-up on the headline grid: batching alone
    # (FP64, smoothness indicator), then FP32 bulk (smoothness indicator)
    decomposition = None
    ro0 = matched(opt, HEADLINE_TARGET)
    if ro0 is not None and plain:
        rb64 = run_optimized(ro0["n"], args.t_end, args.steps, args.warmup, None, args.fill_dof,
                             phase_timing=False, dtype=C.FP64, indicator=C.IND_PAPER)
        rb32 = run_optimized(ro0["n"], args.t_end, args.steps, args.warmup, None, args.fill_dof,
                             phase_timing=False, dtype=C.MP32, indicator=C.IND_PAPER)
        rp0 = [r for r in plain if r["n"] == ro0["n"]][0]
        decomposition = {
            "grid": ro0["n"],
            "plain_fp64_single": rp0["dofsteps_per_s"],
            "fp64_batched_indicator": rb64["dofsteps_per_s"],
            "fp32_bulk_batched_indicator": rb32["dofsteps_per_s"],
            "fp32_bulk_batched_learned": ro0["dofsteps_per_s"],
            "l1": {"plain_fp64_single": rp0["l1"], "fp64_batched_indicator": rb64["l1"],
                   "fp32_bulk_batched_indicator": rb32["l1"], "fp32_bulk_batched_learned": ro0["l1"]}}
        print(f"# decomposition n={ro0['n']}: {decomposition}", flush=True)

    dof512 = 512 * 512 * (N_DEG + 1) ** 2
    per_target = {}
    for tau in TARGETS:
        rp, ro = matched(plain, tau), matched(opt, tau)
        per_target[f"{tau:g}"] = {
            "plain": None if rp is None else {"n": rp["n"], "dofsteps_per_s": rp["dofsteps_per_s"], "l1": rp["l1"]},
            "optimized": None if ro is None else {"n": ro["n"], "copies": ro["copies"],
                                                  "dofsteps_per_s": ro["dofsteps_per_s"], "l1": ro["l1"]},
            "speedup": None if (rp is None or ro is None) else ro["dofsteps_per_s"] / rp["dofsteps_per_s"]}
    head = per_target[f"{HEADLINE_TARGET:g}"]
    ro = matched(opt, HEADLINE_TARGET)
    rp = matched(plain, HEADLINE_TARGET)
    if ro is None:
        raise RuntimeError("no sweep grid meets the headline L1 target")
    # roofline of the dominant kernel of the timed optimized run: the batched local phase
    M = 4
    lb = local_bytes_per_node(M, N_DEG, 4, lim=True, mp=True) * ro["dof"]
    lms = ro["phase_ms"][0]
    achieved = lb / (lms * 1e-3)
    line = {
        "metric": "DoF*steps/s, 2D Euler N=3: FP32/learned/batched vs plain FP64 at matched L1",
        "value": ro["dofsteps_per_s"],
        "unit": "DoF*steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ro["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 bulk + f64 means/roots",
        "data": "synthetic (isentropic vortex initial condition; learned indicator trained on synthetic "
                "Riemann runs and element patterns)",
        "config": {"workload": f"2D Euler isentropic vortex, periodic [-5,5]^2, N=3, cRK44, EA/D2, limiter chain "
                               f"on, t_end={args.t_end}, n^2 sweep {sweep}; value = FP32-bulk + learned indicator "
                               f"+ batched copies on the grid matching density L1 <= {HEADLINE_TARGET:g}",
                   "matched_grid": ro["n"], "copies": ro["copies"], "dof": ro["dof"], "N": N_DEG},
        "plain_fp64_at_target": None if rp is None else {"n": rp["n"], "dofsteps_per_s": rp["dofsteps_per_s"],
                                                          "ms_per_step": rp["ms_per_step"], "l1": rp["l1"]},
        "speedup_vs_plain_fp64": head["speedup"],
        "speedup_decomposition": decomposition,
        "matched_l1": per_target,
        "roofline": {"bound": "hbm", "kernel": "k_batch local phase (MP32, limiter chain)",
                     "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK, "traffic": recorded_traffic(ro["n"], ro["copies"]),
                     "algorithmic_bytes_per_launch": lb, "avg_ms": lms},
        "learned_indicator": train,
        "c5_uneven_batch": c5,
        "sweep": {"plain": plain, "optimized": opt},
    }
    if c3:
        kb = local_bytes_per_node(M, N_DEG, 8, lim=False, mp=False) * dof512
        k_ms = c3["fp64"]["kernel_ms"][0]
        a, b_ = c3["fp64"]["state"], c3["mp32"]["state"]
        line["c3_512"] = {
            "fp64": {"dofsteps_per_s": dof512 / (c3["fp64"]["ms_per_step"] * 1e-3),
                     "ms_per_step": c3["fp64"]["ms_per_step"], "kernel_ms": c3["fp64"]["kernel_ms"]},
            "mp32": {"dofsteps_per_s": dof512 / (c3["mp32"]["ms_per_step"] * 1e-3),
                     "ms_per_step": c3["mp32"]["ms_per_step"], "kernel_ms": c3["mp32"]["kernel_ms"],
                     "rel_l1_vs_fp64": float(np.abs(a - b_).sum() / np.abs(a).sum())},
            "roofline_k_local_fp64": {"bound": "hbm", "achieved": kb / (k_ms * 1e-3) / 1e9,
                                      "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                                      "frac": kb / (k_ms * 1e-3) / HBM_PEAK, "algorithmic_bytes_per_launch": kb,
                                      "avg_ms": k_ms},
            "limiter": "off"}
        for key in ("fp64_limited", "mp32_limited"):
            if key in c3:
                line["c3_512"][key] = {"dofsteps_per_s": dof512 / (c3[key]["ms_per_step"] * 1e-3),
                                       "ms_per_step": c3[key]["ms_per_step"], "kernel_ms": c3[key]["kernel_ms"]}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(rp["n"] if rp else 64, args.t_end, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
