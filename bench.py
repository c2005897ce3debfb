"""Benchmark: Matérn Gaussian log-likelihood evaluations per second at
n = 512,000 on one MI355X (FP64 H path), with p50/p99 latency, the roofline
fraction of the dominant kernel and the dense CPU oracle as baseline.

One step = one likelihood evaluation for a new theta: re-assembly of C~
(dense leaves + ACA + recompression), H-Cholesky with the forward solve
L~ v = z fused into the sweep, log-determinant and quadratic form.  The trees
and the plan are built once per location set, outside the timed region.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 512000]
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

PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (= FP64 matrix) peak
PEAK_HBM_TBS = 8.0           # MI355X HBM3E bandwidth


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_full, theta, sizes=(1000, 2000, 4000)):
    """Dense FP64 oracle (NumPy/SciPy assembly of Eq. (3) entries, LAPACK
    dpotrf and triangular solve, Eq. (1)) timed on the host at a few sizes of
    the same workload, each phase fitted to its own cost law -- assembly
    a n^2 (one Matérn evaluation per entry), factorisation and solve b n^3 --
    and extrapolated to n_full (the dense matrix there does not fit in
    memory)."""
    from oracle import dense
    import workloads

    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max(int(i.get("num_threads", 0)) for i in threadpool_info()) or None
    except Exception:
        pass
    rows = []
    for n_s in sizes:
        locs, xi = workloads.uniform(n_s, seed=0)
        t0 = time.perf_counter()
        C = dense.cov_matrix(locs, *theta)
        t1 = time.perf_counter()
        L = dense.cholesky_lapack(C)
        v = dense.forward_solve_lapack(L, xi)
        _ = dense.logdet_from_factor(L) + float(v @ v)
        t2 = time.perf_counter()
        rows.append((n_s, t1 - t0, t2 - t1))
        del C, L
    ns = np.array([r[0] for r in rows], dtype=np.float64)
    ta = np.array([r[1] for r in rows])
    tc = np.array([r[2] for r in rows])
    # least squares through the origin on the two cost laws
    a = float(np.sum(ta * ns ** 2) / np.sum(ns ** 4))
    b = float(np.sum(tc * ns ** 3) / np.sum(ns ** 6))
    t_full = a * n_full ** 2 + b * n_full ** 3
    samp = ", ".join(f"n={r[0]}: assembly {r[1]:.2f} s + Cholesky/solve {r[2]:.2f} s" for r in rows)
    return {"value": 1.0 / t_full, "unit": "evals/s", "cores": threads or os.cpu_count(), "kind": "oracle",
            "cpu_model": _cpu_model(), "extrapolated": True,
            "sample": f"dense FP64 oracle of the same workload timed at {samp}; fitted assembly "
                      f"{a:.3e} s x n^2 and Cholesky+solve {b:.3e} s x n^3, extrapolated to n={n_full}: "
                      f"{a * n_full ** 2:.3e} s + {b * n_full ** 3:.3e} s per evaluation (the dense matrix at "
                      f"n={n_full} would need {8 * n_full**2 / 1e12:.1f} TB)"}


def serving(args, hcov, workloads):
    """Serving stream: requests of n log-uniform in [1k, 64k], uniform
    locations, theta uniform in the stated boxes, z = xi (FP64, eps 1e-8,
    leaf 64, eta 2, nugget 1e-4).  A request whose factorisation cannot reach
    the accuracy within the rank capacity (HCOV_ERANK) or loses positive
    definiteness (HCOV_ENOTSPD) fails alone and is counted, not retried: the
    smoothest, worst-conditioned kernels of the box (nu near 2.5 with large
    ell), where the truncation errors of the Schur complements are amplified
    by the condition number.  Three runs of the same requests: the plain
    path one at a time in arrival order (FIFO), the server with every request
    queued at once (capacity), and the server under Poisson arrivals at 0.8 x
    its own capacity (latency under load)."""
    eps, leaf, eta, nug = 1e-8, 64, 2.0, 1e-4
    reqs = workloads.serving_stream(count=args.requests, seed=0, rate=1.0)
    inputs = [workloads.request_inputs(r) for r in reqs]
    thetas = [(r["sigma2"], r["ell"], r["nu"], nug) for r in reqs]
    # warm-up (kernel attributes, allocator pools)
    w = hcov.HCov(inputs[0][0], thetas[0], eps=eps, leaf=leaf, eta=eta)
    w.loglik(inputs[0][1])
    w.close()
    progress("warm-up done")

    def run(slots, arrivals):
        S = hcov.Server(slots=slots)
        t0 = time.perf_counter()
        tickets = []
        for (locs, z), th, a in zip(inputs, thetas, arrivals):
            dt = t0 + a - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            tickets.append(S.submit(z, th, locs=locs, eps=eps, leaf=leaf, eta=eta))
            if len(tickets) % 64 == 0 and arrivals[-1] > 0.0:
                progress(f"{len(tickets)}/{len(arrivals)} requests submitted")
        res = []
        for i, t in enumerate(tickets):
            res.append(S.wait(t))
            if (i + 1) % 32 == 0:
                progress(f"{slots} slot(s): {i + 1}/{len(tickets)} requests done")
        wall = time.perf_counter() - t0
        S.close()
        bad = [r["status"] for r in res if r["status"] != 0]
        assert all(b in (hcov.ERANK, hcov.ENOTSPD) for b in bad), bad
        lat = np.array([r["latency_ms"] for r in res])
        return wall, lat, res

    zero = [0.0] * len(reqs)
    t_fifo, lat_fifo, res_fifo = run(1, zero)
    progress(f"FIFO plain path: {len(reqs) / t_fifo:.2f} evals/s")
    t_cap, lat_cap, res_cap = run(args.slots, zero)
    progress(f"server capacity ({args.slots} slots): {len(reqs) / t_cap:.2f} evals/s")
    rate = 0.8 * len(reqs) / t_cap
    gaps = np.random.default_rng(1).exponential(1.0 / rate, size=len(reqs))
    arr = list(np.cumsum(gaps) - gaps[0])
    t_open, lat_open, res_open = run(args.slots, arr)
    progress(f"server open loop at {rate:.2f} req/s done")
    same = all((a["status"], a["loglik"], a["logdet"], a["quad"]) == (b["status"], b["loglik"], b["logdet"], b["quad"])
               == (c["status"], c["loglik"], c["logdet"], c["quad"]) for a, b, c in zip(res_fifo, res_cap, res_open))
    failed = [i for i, r in enumerate(res_cap) if r["status"] != 0]
    pct = lambda a, q: float(np.percentile(a, q))
    return {
        "metric": "serving: loglik evals/sec over a request stream (n log-uniform 1k-64k); p50/p99 latency",
        "value": len(reqs) / t_cap, "unit": "evals/s", "n_gpus": 1, "steps": len(reqs), "warmup": 1,
        "ms_per_step": 1e3 * t_cap / len(reqs), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serving stream of {len(reqs)} requests, n log-uniform [1000, 64000], uniform "
                               f"[0,1]^2 locations, sigma2 U[0.5,2], ell U[0.02,0.3], nu U[0.3,2.5], nugget {nug}, "
                               f"eps {eps}, leaf {leaf}, eta {eta}, z = xi", "slots": args.slots},
        "fifo_plain_path": {"evals_per_s": len(reqs) / t_fifo, "p50_ms": pct(lat_fifo, 50),
                            "p99_ms": pct(lat_fifo, 99)},
        "capacity": {"evals_per_s": len(reqs) / t_cap, "p50_ms": pct(lat_cap, 50), "p99_ms": pct(lat_cap, 99)},
        "open_loop": {"arrival_rate_per_s": rate, "evals_per_s": len(reqs) / t_open, "p50_ms": pct(lat_open, 50),
                      "p99_ms": pct(lat_open, 99)},
        "results_identical_across_runs": bool(same),
        "failed": {"count": len(failed),
                   "erank": sum(res_cap[i]["status"] == hcov.ERANK for i in failed),
                   "enotspd": sum(res_cap[i]["status"] == hcov.ENOTSPD for i in failed),
                   "theta": [[round(v, 4) for v in thetas[i][:3]] for i in failed],
                   "n": [int(len(inputs[i][1])) for i in failed]},
    }


def fit128k(args, hcov, workloads):
    """Maximum-likelihood fit on the jittered-grid workload: n = 128,000,
    sigma2 1, ell 0.05, nu 1.5, nugget 1e-5, leaf 64, eta 2.  The accuracy eps
    is the first of 1e-10, 1e-9, 1e-8 whose factorisation at the truth keeps
    every low-rank block within the rank capacity of 64 (this smooth kernel's
    Cholesky factor needs more at some accuracies); z = L~ xi is drawn from that
    factorisation and Nelder-Mead runs at the same eps from truth x
    (1.2, 0.8, 1.1) for a fixed number of evaluations, inside the library.
    Evaluations that exceed the capacity count as +inf for the search."""
    n, truth, nug, leaf, eta = 128000, (1.0, 0.05, 1.5), 1e-5, 64, 2.0
    locs, xi = workloads.jitter_grid(n, 358, seed=0)
    t0 = time.perf_counter()
    z, eps_draw = None, None
    for e in (1e-10, 1e-9, 1e-8):
        S = hcov.HCov(locs, (*truth, nug), eps=e, leaf=leaf, eta=eta)
        try:
            S.cholesky()
            z = S.sample(xi[S.perm()])   # external order
            eps_draw = e
            break
        except hcov.HcovError as err:
            if err.code != hcov.ERANK:
                raise
            progress(f"eps {e}: {err}")
        finally:
            S.close()
    assert z is not None, "no drawing factorisation fits the rank capacity"
    progress(f"observations drawn at eps {eps_draw} in {time.perf_counter() - t0:.1f} s")
    t1 = time.perf_counter()
    theta0 = np.array(truth) * np.array([1.2, 0.8, 1.1])
    H = hcov.HCov(locs, (*theta0, nug), eps=eps_draw, leaf=leaf, eta=eta)
    t_build = time.perf_counter() - t1
    t2 = time.perf_counter()
    th, ll, ne, hist = H.fit(z, theta0, nug, max_evals=args.evals)
    t_fit = time.perf_counter() - t2
    H.close()
    failed = sum(not np.isfinite(f) for _, f in hist)
    return {
        "metric": "Nelder-Mead fit: loglik evaluations/sec inside the simplex search (n = 128k jittered grid)",
        "value": ne / t_fit, "unit": "evals/s", "n_gpus": 1, "steps": ne, "warmup": 0,
        "ms_per_step": 1e3 * t_fit / ne, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "jittered 358x358 grid, n 128000, sigma2 1, ell 0.05, nu 1.5, nugget 1e-5, leaf 64, "
                               f"eta 2, eps {eps_draw}, z = L~xi at the same eps, start truth x (1.2, 0.8, 1.1)"},
        "theta_hat": [float(x) for x in th], "loglik_hat": ll, "evaluations": ne,
        "failed_evaluations": failed, "build_s": t_build,
        "fit_s": t_fit,
    }


def paramid_bench(args, hcov, workloads):
    """Parameter identification (Sec. 5.1, Fig. 9): Z0 = L~ xi at n0 uniform
    locations from theta* = (sigma2 1, ell 0.0864, nu 0.5), nugget 1e-4
    (eps 1e-7, leaf 128); replicate subsets of n points, each fitted by
    Nelder-Mead from theta* x (1.2, 0.8, 1.1) (eps 1e-7, leaf 64)."""
    from paper_1709_08625_amd import paramid
    sizes = [int(x) for x in args.sizes.split(",")]
    t0 = time.perf_counter()
    locs0, xi0 = workloads.uniform(args.n0, seed=0)
    z0 = paramid.draw_field(locs0, xi0)
    t_draw = time.perf_counter() - t0
    progress(f"Z0 drawn at n0={args.n0} in {t_draw:.1f} s")
    start = tuple(np.array(paramid.TRUTH) * np.array([1.2, 0.8, 1.1]))
    t1 = time.perf_counter()
    fits = paramid.identify(locs0, z0, sizes, args.replicates, start, max_evals=args.evals, progress=progress)
    t_fit = time.perf_counter() - t1
    evals = sum(f["evals"] for f in fits)
    return {
        "metric": "parameter identification: likelihood evaluations/sec over replicate Nelder-Mead fits",
        "value": evals / t_fit, "unit": "evals/s", "n_gpus": 1, "steps": len(fits), "warmup": 0,
        "ms_per_step": 1e3 * t_fit / max(len(fits), 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Z0 = L~xi at n0={args.n0} uniform locations, theta* = (sigma2 1, ell 0.0864, "
                               f"nu 0.5), nugget 1e-4; {args.replicates} replicates per n in {sizes}, "
                               f"{args.evals} evaluations per fit"},
        "truth": {"sigma2": paramid.TRUTH[0], "ell": paramid.TRUTH[1], "nu": paramid.TRUTH[2]},
        "draw_s": t_draw, "fit_s": t_fit, "evaluations": evals,
        "summary": paramid.summarise(fits), "fits": fits,
    }


def large2m(args, hcov, workloads):
    """The large instance: n = 2,000,000 locations (70% uniform in [0,1]^2,
    30% from 20 Gaussian clusters of sd 0.01), sigma2 1, ell 0.1, nu 0.5,
    nugget 1e-4, eps 1e-6, leaf 128, eta 2; z = L~ xi drawn at the truth;
    the library's Nelder-Mead (hcov_nm_minimize, the initial steps of
    hcov_fit) over (sigma2, ell, nu) from truth x (1.2, 0.8, 1.1) for --evals
    evaluations, each re-assembling and factorising C~ for its theta."""
    n, truth, nug, leaf, eta, eps = args.n if args.n != 512000 else 2000000, (1.0, 0.1, 0.5), 1e-4, 128, 2.0, 1e-6
    locs, xi = workloads.mixture(n, seed=0)
    opts = {"precision": hcov.MIXED if args.precision == "mixed" else hcov.FP64}
    if args.rank_cap:
        opts["initial_rank_cap"] = args.rank_cap
    t0 = time.perf_counter()
    H = hcov.HCov(locs, (*truth, nug), eps=eps, leaf=leaf, eta=eta, opts=opts)
    t_build = time.perf_counter() - t0
    progress(f"trees, plan and assembly at n={n}: {t_build:.1f} s")
    t1 = time.perf_counter()
    H.cholesky()
    z = H.sample(xi[H.perm()])
    t_draw = time.perf_counter() - t1
    progress(f"z = L~xi drawn in {t_draw:.1f} s")
    theta0 = np.array(truth) * np.array([1.2, 0.8, 1.1])
    hist_all = []
    t2 = time.perf_counter()

    def negll(x):
        # -L~ of Eq. (1) at theta = x (outside the domain or not positive
        # definite: +inf, as in hcov_fit); one progress line per evaluation
        if min(x) <= 0.0:
            v = float("inf")
        else:
            try:
                H.set_theta((float(x[0]), float(x[1]), float(x[2]), nug))
                v = -H.loglik(z)[0]
            except hcov.HcovError:
                v = float("inf")
        hist_all.append(([float(a) for a in x], v))
        progress(f"evaluation {len(hist_all)}: theta ({x[0]:.4f}, {x[1]:.4f}, {x[2]:.4f}) -loglik {v:.6e} "
                 f"({time.perf_counter() - t2:.0f} s)")
        return v

    th, fbest, done = hcov.nm_minimize(negll, theta0, np.array([0.01, 0.04, 0.02]), max_evals=args.evals,
                                       size_tol=1e-5)[:3]
    t_fit = time.perf_counter() - t2
    theta = np.asarray(th, dtype=np.float64)
    st = H.stats()
    H.close()
    return {
        "metric": "large instance: loglik evaluations/sec inside Nelder-Mead (n = 2M mixture)",
        "value": done / t_fit, "unit": "evals/s", "n_gpus": 1, "steps": done, "warmup": 0,
        "ms_per_step": 1e3 * t_fit / done, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32-accumulated low-rank products, f64 storage",
        "data": "synthetic",
        "config": {"workload": f"n {n}: 70% uniform [0,1]^2 + 30% from 20 Gaussian clusters (sd 0.01), sigma2 1, "
                               f"ell 0.1, nu 0.5, nugget 1e-4, eps {eps}, leaf {leaf}, eta {eta}, z = L~xi at the "
                               f"truth, Nelder-Mead from truth x (1.2, 0.8, 1.1), {args.evals} evaluations",
                   "precision": args.precision},
        "build_s": t_build, "draw_s": t_draw, "fit_s": t_fit, "evaluations": done,
        "theta_hat": [float(x) for x in theta], "loglik_hat": -float(fbest), "history": hist_all,
        "structure": {"device_GB": st["bytes_device"] / 1e9, "factor_GB": st["bytes_factor"] / 1e9,
                      "max_rank": st["max_rank_seen"], "mean_rank": st["mean_rank"],
                      "lr_blocks": st["n_lr_blocks"], "dense_blocks": st["n_dense_blocks"],
                      "initial_rank_cap": args.rank_cap, "lowrank_GB": st["bytes_lowrank"] / 1e9,
                      "replans": st["n_replans"]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the planner's GEMM kernel choice (default: both GEMM kernels are timed on the "
                         "first factorisation, outside the timed steps, and each launch keeps the faster)")
    ap.add_argument("--rank-cap", type=int, default=32,
                    help="initial room of every low-rank block's U and V (0: max_rank 64 everywhere); blocks "
                         "that need more grow, with a plan rebuild, during the first evaluations")
    ap.add_argument("--profile-kind", default="gemm")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch the sweep stage by stage instead of replaying captured graph segments")
    ap.add_argument("--workload", default="loglik512k", choices=["loglik512k", "serving", "fit128k", "paramid", "large2m"])
    ap.add_argument("--n0", type=int, default=2000000, help="paramid: size of the field Z0")
    ap.add_argument("--sizes", default="2000,4000,8000,16000", help="paramid: subset sizes")
    ap.add_argument("--replicates", type=int, default=5, help="paramid: fits per subset size")
    ap.add_argument("--evals", type=int, default=30)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--requests", type=int, default=96)
    ap.add_argument("--slots", type=int, default=6)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(requests shard across GPUs as independent contexts)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_1709_08625_amd import hcov

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    if args.workload == "serving":
        print(json.dumps(serving(args, hcov, workloads)))
        return
    if args.workload == "fit128k":
        print(json.dumps(fit128k(args, hcov, workloads)))
        return
    if args.workload == "paramid":
        print(json.dumps(paramid_bench(args, hcov, workloads)))
        return
    if args.workload == "large2m":
        print(json.dumps(large2m(args, hcov, workloads)))
        return
    n = args.n
    theta0 = (1.0, 0.08, 0.8, 1e-4)
    eps, leaf, eta = 1e-7, 128, 2.0
    locs, xi = workloads.uniform(n, seed=0)
    stream = torch.cuda.current_stream().cuda_stream
    t_build = time.perf_counter()
    opts = {"precision": hcov.MIXED if args.precision == "mixed" else hcov.FP64}
    if args.no_graphs:
        opts["use_graphs"] = 0
    if args.autotune:
        opts["autotune"] = 1
    if args.rank_cap:
        opts["initial_rank_cap"] = args.rank_cap
    H = hcov.HCov(locs, theta0, eps=eps, leaf=leaf, eta=eta, stream=stream, opts=opts)
    t_build = time.perf_counter() - t_build
    progress(f"trees, plan and first assembly at n={n}: {t_build:.1f} s")
    # synthetic observations: a sample Z = L~ xi of the field at theta0
    H.cholesky()
    perm = H.perm()
    z = H.sample(xi[perm])
    thetas = workloads.theta_perturbations(theta0[:3], args.warmup + args.steps, rel=0.10, seed=0)
    thetas = [(float(a), float(b), float(c), theta0[3]) for a, b, c in thetas]
    z_dev = torch.from_numpy(z).to("cuda")
    progress("synthetic observations drawn")

    def step(th):
        H.set_theta(th)
        return H.loglik(z_dev)

    for i in range(args.warmup):
        step(thetas[i])
        progress(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    lat = []
    lls = []
    replans0 = H.stats()["n_replans"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        s0 = time.perf_counter()
        lls.append(step(thetas[args.warmup + i])[0])
        lat.append(time.perf_counter() - s0)
        progress(f"timed step {i + 1}/{args.steps}: {lat[-1]:.3f} s")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    st = H.stats()
    # roofline of the dominant kernel: one more evaluation at the last timed
    # theta with its launches bracketed by HIP events (the timed steps replay
    # the captured sweep, which carries no per-launch events; a kernel's
    # duration does not depend on how its launch was submitted)
    H.profile_begin(args.profile_kind)
    step(thetas[-1])
    torch.cuda.synchronize()
    launches, kern_ms, kern_flops, kern_bytes = H.profile_end()
    progress("roofline evaluation done")
    H.close()

    avg_us = 1e3 * kern_ms / max(launches, 1)
    fl_launch = kern_flops / max(launches, 1)
    by_launch = kern_bytes / max(launches, 1)
    tflops = fl_launch / (avg_us * 1e-6) / 1e12 if launches else 0.0
    gbs = by_launch / (avg_us * 1e-6) / 1e9 if launches else 0.0
    # the bound that applies: a launch whose algorithmic intensity is below
    # the FP64 ridge (78.6 TFLOP/s / 8 TB/s = 9.8 flop/B) is HBM bound
    intensity = fl_launch / by_launch if by_launch > 0 else float("inf")
    hbm_bound = intensity < PEAK_FP64_TFLOPS / PEAK_HBM_TBS
    rec = {
        "metric": "loglik evals/sec at n=512k (H-Cholesky+logdet+solve); p50/p99 latency",
        "value": args.steps / total,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": f"matern-loglik n={n} uniform[0,1]^2 seed 0, theta=(sigma2 1, ell 0.08, nu 0.8, "
                        f"nugget 1e-4) +-10% per step, leaf {leaf}, eta {eta}, eps {eps}, "
                        f"{'FP64' if args.precision == 'fp64' else 'mixed-precision'} H path",
            "n": n, "leaf": leaf, "eta": eta, "eps": eps, "precision": args.precision,
        },
        "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)), "p99": 1e3 * float(np.percentile(lat, 99)),
                       "mean": 1e3 * float(np.mean(lat))},
        "phases_ms_last": {"assemble": st["ms_assemble"], "factor_and_solve": st["ms_factor"],
                           "tree_build_once": 1e3 * t_build},
        "structure": {"depth": st["depth"], "lr_blocks": st["n_lr_blocks"], "dense_blocks": st["n_dense_blocks"],
                      "mean_rank": st["mean_rank"], "max_rank": st["max_rank_seen"],
                      "factor_GB": st["bytes_factor"] / 1e9, "device_GB": st["bytes_device"] / 1e9,
                      "launches_per_factorisation": st["n_launches_factor"],
                      "sketch_retries": st["n_sketch_retries"],
                      "mean_sketch_width": st["mean_sketch_width"],
                      "gemm_launches_grouped": st["n_gemm_grouped"], "autotune": bool(args.autotune),
                      "gemm_tflop_per_factorisation": st["gemm_flops_factor"] / 1e12,
                      "gemm_gb_per_factorisation": st["gemm_bytes_factor"] / 1e9,
                      "autotune_switched": st["n_autotune_switched"],
                      "initial_rank_cap": args.rank_cap, "lowrank_GB": st["bytes_lowrank"] / 1e9,
                      "replans": st["n_replans"], "replans_timed": st["n_replans"] - replans0},
        # FP64 tiles of k_gemm run on the matrix cores (dense FP64 MFMA peak);
        # its products are thin (k = ranks 10-40), so their algorithmic
        # intensity sits below the ridge and HBM bandwidth is the bound
        "roofline": {"bound": "hbm" if hbm_bound else "mfma", "kernel": "k_gemm + k_gemm_wide" if args.profile_kind == "gemm" else f"k_{args.profile_kind}",
                     "achieved": gbs if hbm_bound else tflops,
                     "peak": 1e3 * PEAK_HBM_TBS if hbm_bound else PEAK_FP64_TFLOPS,
                     "unit": "GB/s" if hbm_bound else "TFLOP/s",
                     "frac": gbs / (1e3 * PEAK_HBM_TBS) if hbm_bound else tflops / PEAK_FP64_TFLOPS,
                     "traffic": None, "launches": launches, "avg_launch_us": avg_us,
                     "algorithmic_flops_per_launch": fl_launch, "algorithmic_bytes_per_launch": by_launch,
                     "intensity_flop_per_byte": intensity, "achieved_tflops": tflops,
                     "frac_of_fp64_mfma": tflops / PEAK_FP64_TFLOPS, "achieved_gbs": gbs,
                     "frac_of_hbm": gbs / (1e3 * PEAK_HBM_TBS)},
        "loglik_last": lls[-1],
    }
    if not args.no_cpu:
        progress("timing the CPU oracle on a bounded sample")
        rec["cpu_baseline"] = cpu_baseline(n, theta0)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
