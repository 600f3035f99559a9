"""Benchmark: NFFT-accelerated Sinkhorn iterations per second on one MI355X.

Workload (default): the 2-D Gaussian-mixture problem, n = nt = 1e6 points,
Dirichlet weights, squared Euclidean cost, eps = 0.01, N = 512, m = 8,
sigma = 2, FP32 grids/FFT with FP64 scalings and reductions.  One step is
one Sinkhorn iteration (alpha update then alpha_t update, each one full fast
summation plus the fused scaling update), replayed from a captured hipGraph
with every input resident in HBM.

Prints one JSON line with the throughput, the roofline figure of the dominant
kernel (device times from HIP events on the solver's stream) and the FP64
oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Sources whose change invalidates the measured HBM traffic of the hot kernels.
TRAFFIC_SOURCES = ("paper_2201_07524_amd/csrc/nufft_kernels.hip", "paper_2201_07524_amd/csrc/plan_kernels.hip",
                   "paper_2201_07524_amd/csrc/common.h", "paper_2201_07524_amd/csrc/kernels.h")
CALIB_COPY_BYTES = 256 << 20


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_bytes(info, d, which):
    """Algorithmic HBM bytes per launch: points (FP32 tile-local coordinates,
    FP64 weights / marginals / scalings) and grid values, each moved once."""
    n_s = 0.5 * (info["n"] + info["nt"])   # spread and interp alternate between the clouds
    G = info["grid_cells"]
    gb = info["grid_value_bytes"]
    cb = 4 * d if gb == 4 else 8 * d
    if which == "spread":
        return n_s * (cb + 8) + G * gb
    if which == "fft":
        return 4 * G * gb
    return G * gb + n_s * (cb + 24)


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_<kernel>_gmm2d_1e6_fp32.md: FETCH_SIZE + WRITE_SIZE,
    each scaled by the same counter's reading for a plain copy of known size),
    or None when that summary is missing or the kernel sources changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_gmm2d_1e6_fp32.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                vals[k.strip("`")] = v.strip().strip("`")
    if vals.get("source_sha256") != source_digest():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_util(kernel):
    """VALU and LDS busy fractions of `kernel` from the committed counter
    summary (profiles/util_<kernel>_gmm2d_1e6_fp32.md: rocprofv3's VALUBusy
    and LdsUtil derived metrics), or (None, None) when it is missing or the
    kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"util_{kernel}_gmm2d_1e6_fp32.md")
    if not os.path.exists(path):
        return None, None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].strip().split(": ", 1)
                vals[k.strip("`")] = v.strip().strip("`")
    if vals.get("source_sha256") != source_digest():
        return None, None
    try:
        return float(vals["valu_frac"]), float(vals["lds_frac"])
    except (KeyError, ValueError):
        return None, None


def cpu_baseline(cfg, budget_rows=8192):
    """Oracle (FP64 matrix-free direct sums in C/OpenMP) timed on a bounded
    sample: one kernel product K v over all sources for `budget_rows` sampled
    targets, scaled to the two full products of one iteration (extrapolated)."""
    import numpy as np
    from oracle import direct

    direct.load()
    n, nt = cfg["x"].shape[0], cfg["y"].shape[0]
    rows = np.random.default_rng(5).choice(nt, size=min(budget_rows, nt), replace=False)
    w = np.ones(n)
    t0 = time.perf_counter()
    direct.kv(cfg["y"], cfg["x"], w, cfg["r"], cfg["eps"], rows=rows)
    dt = time.perf_counter() - t0
    pairs_sample = len(rows) * n
    pairs_iter = 2.0 * n * nt
    sec_per_iter = dt * pairs_iter / pairs_sample
    return dict(value=1.0 / sec_per_iter, unit="iter/s", cores=direct.num_threads(), kind="oracle",
                sample=f"one FP64 kernel product on {len(rows)} sampled targets x {n} sources "
                       f"({dt:.1f} s), scaled to 2 full products per iteration")


def plain_1d_leg(nfs, workloads, torch, T):
    """The latency-bound workload: d = 1, n = nt = 2048 points uniform on
    [-1/4, 1/4], eps = 0.05, N = 256, m = 8, FP64, its 200 iterations.  GPU:
    plan and ms per iteration (graph replay).  CPU: the oracle's dense FP64
    Algorithm 1 for the same 200 iterations, on all host cores and on one."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import sinkhorn_dense as sd
    cfg = workloads.plain_1d()
    prm = nfs.Params(d=1, eps=cfg["eps"], N=cfg["N"], m=cfg["m"], precision="fp64")
    x, p, y, pt = T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = nfs.Solver(prm, x, p, y, pt)
    torch.cuda.synchronize()
    plan = time.perf_counter() - t0
    s.iterate(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(cfg["iters"])
    torch.cuda.synchronize()
    t_it = (time.perf_counter() - t0) / cfg["iters"]
    s.close()
    out = {"n": 2048, "iters": cfg["iters"], "plan_ms": plan * 1e3, "ms_per_iteration": t_it * 1e3,
           "solve_ms": (plan + cfg["iters"] * t_it) * 1e3}
    # all cores: the threads this process may use (the machine's CPU share; OMP_NUM_THREADS when set)
    all_threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    for name, threads in (("oracle_all_cores", all_threads), ("oracle_one_core", 1)):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            sd.solve(cfg["x"], cfg["p"], cfg["y"], cfg["pt"], 2, cfg["eps"], cfg["iters"])
            out[name + "_s"] = time.perf_counter() - t0
    out["oracle_threads_all"] = all_threads
    return out


def batched_leg(nfs, workloads, torch, T, iters=10, sample_every=16):
    """The batched form: 512 independent 2-D mixture problems (sizes log-uniform
    in [1e3, 2e5], eps uniform in [0.005, 0.05], N = 256, m = 6, FP32), all
    advanced by one captured iteration; compared with plain single-problem
    solvers run one after another (every `sample_every`-th problem, scaled to
    the whole batch).  Then one complete solve of `iters` iterations with
    automatic FP64 promotion of the problems FP32 grids cannot resolve (wall
    time including plan, FP32 batch and the FP64 re-solves)."""
    import numpy as np
    cfg = workloads.batched_2d()
    probs = cfg["problems"]
    prm = nfs.Params(d=2, eps=1.0, N=cfg["N"], m=cfg["m"], precision="fp32")
    xs = [T(p["x"]) for p in probs]
    ps = [T(p["p"]) for p in probs]
    ys = [T(p["y"]) for p in probs]
    pts = [T(p["pt"]) for p in probs]
    eps = [p["eps"] for p in probs]
    s = nfs.BatchSolver(prm, xs, ps, ys, pts, eps)  # loads the code objects
    s.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = nfs.BatchSolver(prm, xs, ps, ys, pts, eps)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    s.iterate(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(iters)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / iters
    res = s.finish(check=False)
    nonpos = sum(1 for r in res if r.n_nonpos > 0)
    s.close()
    del s
    t_plain = 0.0
    sample = list(range(0, len(probs), sample_every))
    for b in sample:
        sp = nfs.Params(d=2, eps=eps[b], N=cfg["N"], m=cfg["m"], precision="fp32")
        one = nfs.Solver(sp, xs[b], ps[b], ys[b], pts[b])
        one.iterate(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one.iterate(iters)
        torch.cuda.synchronize()
        t_plain += (time.perf_counter() - t0) / iters
        one.close()
    t_plain *= len(probs) / len(sample)
    npts = sum(p["x"].shape[0] + p["y"].shape[0] for p in probs)
    # one-shot solve with automatic promotion: problems whose FP32 sums hit
    # t <= 0 or a dynamic range above 1e5 again as one FP64 batch, and those
    # beyond FP64's range in the centred form
    aprm = nfs.Params(d=2, eps=1.0, N=cfg["N"], m=cfg["m"], precision="auto")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ares = nfs.batch_sinkhorn(aprm, xs, ps, ys, pts, eps, iters, check=False)
    torch.cuda.synchronize()
    t_auto = time.perf_counter() - t0
    return {"problems": len(probs), "points": npts, "plan_ms": t_plan * 1e3, "ms_per_iteration": t_batch * 1e3,
            "problem_iterations_per_s": len(probs) / t_batch,
            "plain_sequential_ms_per_iteration_est": t_plain * 1e3,
            "speedup_vs_plain": t_plain / t_batch,
            "problems_with_nonpositive_sums_fp32": nonpos,
            "auto_solve_ms": t_auto * 1e3, "auto_iterations": iters,
            "auto_promoted_to_fp64": sum(1 for r in ares if r.precision_used == "fp64"),
            "auto_centred": sum(1 for r in ares if r.centred),
            "auto_nonpositive_after_promotion": sum(1 for r in ares if r.n_nonpos > 0)}


def grad_leg(nfs, workloads, torch, T, iters=5):
    """The differentiated form: 3-D mixtures, n = nt = 1e6, eps = 0.01, N = 128,
    m = 8, FP32; time of one forward iteration vs one envelope gradient in
    positions and weights of both clouds, on the solver's own plan
    (nfs_solver_grad), and vs the one-shot entry point that plans again."""
    cfg = workloads.gmm_3d()
    prm = nfs.Params(d=3, eps=cfg["eps"], N=cfg["N"], m=cfg["m"], precision="fp32")
    x, p, y, pt = T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"])
    s = nfs.Solver(prm, x, p, y, pt)
    s.iterate(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(iters)
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / iters
    res = s.finish(check=False)
    s.grad(True, True, False, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.grad(True, True, False, False)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    t0 = time.perf_counter()
    s.grad(True, True, True, True)
    torch.cuda.synchronize()
    t_grad4 = time.perf_counter() - t0
    s.close()
    nfs.sinkhorn_grad(prm, x, p, y, pt, res.alpha, res.alpha_t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nfs.sinkhorn_grad(prm, x, p, y, pt, res.alpha, res.alpha_t)
    torch.cuda.synchronize()
    t_once = time.perf_counter() - t0
    return {"forward_ms_per_iteration": t_fwd * 1e3, "gradient_x_mu_ms": t_grad * 1e3,
            "gradient_over_forward_iteration": t_grad / t_fwd, "gradient_x_mu_y_nu_ms": t_grad4 * 1e3,
            "one_shot_gradient_ms_incl_plan": t_once * 1e3, "cpu_oracle": cpu_baseline(cfg, budget_rows=2048)}


def log_leg(nfs, prm, x, p, y, pt, torch, iters=20):
    """The log-domain form (Algorithm 4) on the benchmarked 2-D mixture
    workload: ms per iteration of the potentials solve, same parameters."""
    from dataclasses import replace
    lp = replace(prm, flags=prm.flags | nfs.FLAG_LOG_DOMAIN)
    s = nfs.Solver(lp, x, p, y, pt)
    s.iterate(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(iters)
    torch.cuda.synchronize()
    t_it = (time.perf_counter() - t0) / iters
    stage_ms, _ = s.profile(5)
    res = s.finish(check=False)
    s.close()
    return {"ms_per_iteration": t_it * 1e3, "iterations": iters + 2 + 5, "cost": res.cost,
            "n_nonpos": res.n_nonpos,
            "stage_ms": dict(zip(("spread_incl_weights", "fft", "interp", "iteration"), stage_ms))}


def ball_shell_leg(nfs, workloads, torch, T, iters=3, rho=1):
    """The Euclidean-cost form (r = 1, with the near field): ball against
    shell, 4e6 points per cloud, eps = 0.02, N = 128, m = 6, FP32; ms per
    iteration and per-stage device times.  rho: the exponent of the distance
    (a real rho goes through the sampled-kernel tables)."""
    cfg = dict(workloads.ball_shell_3d(), r=rho)
    prm = nfs.Params(d=3, r=rho, eps=cfg["eps"], N=cfg["N"], m=cfg["m"], precision="fp32")
    t0 = time.perf_counter()
    s = nfs.Solver(prm, T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"]))
    torch.cuda.synchronize()
    plan = time.perf_counter() - t0
    s.iterate(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(iters)
    torch.cuda.synchronize()
    t_it = (time.perf_counter() - t0) / iters
    stage_ms, _ = s.profile(1)
    res = s.finish(check=False)
    s.close()
    return {"points": int(cfg["x"].shape[0]), "ms_per_iteration": t_it * 1e3, "plan_ms": plan * 1e3,
            "stage_ms": dict(zip(("spread", "fft", "interp", "iteration", "near_field"), stage_ms)),
            "near_field_share": 2.0 * stage_ms[4] / stage_ms[3], "cost": res.cost, "n_nonpos": res.n_nonpos,
            "cpu_oracle": cpu_baseline(cfg, budget_rows=512)}


def paper_shapes_leg(nfs, workloads, torch, T, iters=10):
    """The paper's standing workload shapes, FP64 grids, N = 64, m = 8,
    eps = 0.05 (lambda = 20), r = 2: two images on one k x k pixel grid
    (k = 32 ... 512) and uniform samples on [0,1]^2 (n = 1e3 ... 1e7).  Plan
    time and ms per iteration; solve_100_s = plan + 100 iterations."""
    out = {}
    cases = [("grid%d" % k, lambda k=k: workloads.pixel_grid_pair(k)) for k in (32, 64, 128, 256, 512)]
    cases += [("uniform%d" % n, lambda n=n: workloads.uniform_square(n)) for n in (10**3, 10**4, 10**5, 10**6, 10**7)]
    for name, make in cases:
        cfg = make()
        prm = nfs.Params(d=2, eps=cfg["eps"], N=64, m=8, precision="fp64")
        x, p, y, pt = T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = nfs.Solver(prm, x, p, y, pt)
        torch.cuda.synchronize()
        plan = time.perf_counter() - t0
        s.iterate(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(iters)
        torch.cuda.synchronize()
        t_it = (time.perf_counter() - t0) / iters
        res = s.finish(check=False)
        s.close()
        out[name] = {"n": int(cfg["x"].shape[0]), "plan_ms": plan * 1e3, "ms_per_iteration": t_it * 1e3,
                     "solve_100_s": plan + 100 * t_it, "marg_err": res.marg_err, "n_nonpos": res.n_nonpos}
        del x, p, y, pt, s
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-iters", type=int, default=10)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--flags", type=int, default=0, help="nfs_params.flags (library variants)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--no-legs", action="store_true", help="skip the log-domain, batched, gradient, ball/shell and paper-shape legs")
    ap.add_argument("--only-leg", choices=("batched", "gradient", "ball_shell", "ball_shell_rho", "paper_shapes",
                                           "plain_1d"),
                    help="run one secondary leg alone and print its JSON (for profiling)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with one device copy of 256 MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: every box here has a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2201_07524_amd import nfs, workloads

    if args.only_leg:
        dev = torch.device("cuda:0")
        T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
        leg = {"batched": batched_leg, "gradient": grad_leg, "ball_shell": ball_shell_leg,
               "ball_shell_rho": lambda *a: ball_shell_leg(*a, rho=1.5),
               "paper_shapes": paper_shapes_leg, "plain_1d": plain_1d_leg}[args.only_leg]
        print(json.dumps({args.only_leg: leg(nfs, workloads, torch, T)}), flush=True)
        return

    log("bench: generating the 2-D mixture workload")
    cfg = workloads.gmm_2d(args.n)
    dev = torch.device("cuda:0")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    x, p, y, pt = T(cfg["x"]), T(cfg["p"]), T(cfg["y"]), T(cfg["pt"])
    prm = nfs.Params(d=2, eps=cfg["eps"], N=cfg["N"], m=cfg["m"], sigma=cfg["sigma"], precision="fp32",
                     flags=args.flags, tile=args.tile, chunk=args.chunk)
    torch.cuda.synchronize()
    log("bench: planning")
    # the first plan of the process also loads the library's code objects;
    # the plan figure is the second one
    t0 = time.perf_counter()
    solver = nfs.Solver(prm, x, p, y, pt)
    torch.cuda.synchronize()
    plan_first_s = time.perf_counter() - t0
    solver.close()
    t0 = time.perf_counter()
    solver = nfs.Solver(prm, x, p, y, pt)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    log(f"bench: plan {plan_s * 1e3:.1f} ms (first call {plan_first_s * 1e3:.1f} ms); warmup {args.warmup} iterations")
    solver.iterate(args.warmup)
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} iterations")
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    solver.iterate(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_total = ev0.elapsed_time(ev1)
    ms_per_step = ms_total / args.steps
    value = args.steps / (ms_total / 1e3)
    log(f"bench: {ms_per_step:.4f} ms/iteration (wall {wall * 1e3 / args.steps:.4f} ms)")

    res = solver.finish(check=False)
    log(f"bench: cost={res.cost:.9e} marg_err={res.marg_err:.3e} nonpos={res.n_nonpos}")

    stage_ms, info = solver.profile(args.profile_iters)
    names = ("spread", "fft", "interp")
    dom = int(np.argmax(stage_ms[:3]))
    d = 2
    achieved = {k: kernel_bytes(info, d, k) / (stage_ms[i] * 1e-3) / 1e9 for i, k in enumerate(names)}
    log("bench: stage ms/launch " + ", ".join(f"{k}={stage_ms[i]:.4f}" for i, k in enumerate(names))
        + f", iteration={stage_ms[3]:.4f}")
    log("bench: algorithmic GB/s " + ", ".join(f"{k}={v:.1f}" for k, v in achieved.items()))
    fast_pts = 2.0 * (info["n"] + info["nt"]) * value

    out = {
        "metric": "Sinkhorn iters/s at n=m=1e6 d=2",
        "value": value,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2-D Gaussian mixtures, n=nt={args.n}, Dirichlet weights, |x-y|^2, "
                               f"eps=0.01, N=512, m=8, sigma=2, FP32 grids + FP64 scalings",
                   "n": args.n, "d": 2, "N": 512, "m": 8, "eps": 0.01},
        "fastsum_points_per_s": fast_pts,
        "plan_ms": plan_s * 1e3,
        "plan_ms_first_call": plan_first_s * 1e3,
        "stage_ms": dict(zip(names + ("iteration",), stage_ms)),
        "stage_gbs": achieved,
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved[names[dom]],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved[names[dom]] / HBM_PEAK_GBS, "traffic": measured_traffic(names[dom]),
                     "algorithmic_bytes": kernel_bytes(info, d, names[dom]),
                     "valu_frac": measured_util(names[dom])[0], "lds_frac": measured_util(names[dom])[1]},
    }
    solver.close()
    del solver
    if not args.no_legs:
        log("bench: FP64-grid figure for the same workload")
        from dataclasses import replace
        s64 = nfs.Solver(replace(prm, precision="fp64"), x, p, y, pt)
        s64.iterate(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s64.iterate(20)
        torch.cuda.synchronize()
        out["fp64_grids_ms_per_iteration"] = (time.perf_counter() - t0) / 20 * 1e3
        s64.close()
        del s64
        log("bench: 1-D latency-bound leg")
        out["plain_1d"] = plain_1d_leg(nfs, workloads, torch, T)
        log("bench: plain 1-D " + json.dumps(out["plain_1d"]))
        log("bench: log-domain leg")
        out["log_domain"] = log_leg(nfs, prm, x, p, y, pt, torch)
        out["log_domain"]["over_scaling_iteration"] = out["log_domain"]["ms_per_iteration"] / ms_per_step
        log("bench: log-domain " + json.dumps(out["log_domain"]))
        log("bench: batched leg")
        out["batched"] = batched_leg(nfs, workloads, torch, T)
        log("bench: batched " + json.dumps(out["batched"]))
        torch.cuda.empty_cache()
        log("bench: gradient leg")
        out["gradient"] = grad_leg(nfs, workloads, torch, T)
        log("bench: gradient " + json.dumps(out["gradient"]))
        torch.cuda.empty_cache()
        log("bench: ball/shell (r = 1) leg")
        out["ball_shell_r1"] = ball_shell_leg(nfs, workloads, torch, T)
        log("bench: ball/shell " + json.dumps(out["ball_shell_r1"]))
        torch.cuda.empty_cache()
        log("bench: ball/shell (real rho = 1.5) leg")
        out["ball_shell_rho1.5"] = ball_shell_leg(nfs, workloads, torch, T, rho=1.5)
        log("bench: ball/shell rho " + json.dumps(out["ball_shell_rho1.5"]))
        torch.cuda.empty_cache()
        log("bench: paper-shaped workloads leg")
        out["paper_shapes"] = paper_shapes_leg(nfs, workloads, torch, T)
        log("bench: paper shapes " + json.dumps(out["paper_shapes"]))
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(cfg)
    if args.calib_copy:
        src = torch.full((CALIB_COPY_BYTES // 4,), 1.0, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: calibration copy of {CALIB_COPY_BYTES} bytes")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
