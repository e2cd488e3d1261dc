"""Benchmark of the PDNQP hot path on one MI355X.

A step is one outer iteration of PDNQP (Algorithm "practical outer
iteration"): forming the inner QP, the inner rAPDHG iterations with their
sparse products, acceptance tests, averaging and periodic KKT/restart
checks, then the multiplier, residual, penalty, tolerance and centre
updates.  The timed region is one pdnqp_solve call limited to K outer
iterations (it includes the solver's own set-up: scaling, Lanczos, initial
penalties), on problem data already resident in HBM.

value = accepted inner PDHG iterations per second over the timed region.
Extra fields: per-kernel HIP-event timings of the per-trial kernels and the
roofline of the dominant one, the time to reach 1e-4 KKT on the same
instance, and the FP64 CPU oracle's rate on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload large]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "inner PDHG iters/s & time-to-1e-4 KKT at n≈1M; SpMV HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0

# Memory-side bytes per launch from the two rocprofv3 counter passes
# (FETCH_SIZE, WRITE_SIZE) on the large workload, scaled by the same counters
# on a plain 8 MB copy kernel (profiles/traffic_trial_kernels_large.md).
# Valid only for the device code they were taken on: the hash covers the
# kernel helpers and the kernels of the inner iteration, not the host-side
# launch wrappers.
PMC_TRAFFIC = {"source_sha256_prefix": "0f8df680da5b4c87", "workload": "large",
               "bytes": {"f32": {"xtrial": 48.0e6, "qa_spmv": 213.0e6, "at_spmv": 81.2e6,
                                 "decide": 0.1e6},
                         "f64": {"xtrial": 95.9e6, "qa_panels": 242.9e6, "qa_rows": 78.1e6,
                                 "at_spmv": 204.2e6, "decide": 0.1e6}}}


def _kernel_source_sha():
    """sha256 prefix of the inner-iteration device code: the device helpers
    header plus the kernel section (anonymous namespace) of pdnqp_iter.hip."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2609_19557_amd", "csrc")
    helpers = open(os.path.join(csrc, "pdnqp_device.hpp"), "rb").read()
    it = open(os.path.join(csrc, "pdnqp_iter.hip"), "rb").read()
    beg = it.index(b"\nnamespace {\n")
    end = it.index(b"\n}  // namespace\n", beg)
    return hashlib.sha256(helpers + it[beg:end]).hexdigest()[:16]


def _describe(prob):
    return (f"random indefinite sparse QP n={prob['n']:,} m={prob['m']:,} "
            f"(half equalities), nnz(Q)={prob['Q'].nnz:,}, nnz(A)={prob['A'].nnz:,}, box [0,1]")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, n_inner):
    """FP64 CPU oracle on a bounded sample of the same instance: one outer
    step whose inner solve runs exactly ``n_inner`` accepted iterations
    (checks after every 64; the initial inner tolerance is set to 1e-12 so
    that the stopping test does not end the sample early -- the cost of an
    iteration does not depend on it).  The rate counts only the time spent inside the
    oracle's inner solver (its set-up -- scaling, Lanczos, inner-QP
    formation -- is excluded).  The oracle runs on one core: every BLAS/
    OpenMP thread pool is limited to one thread for the whole leg (scipy's
    sparse products are single-threaded)."""
    from threadpoolctl import threadpool_limits

    from oracle import pdnqp_oracle as O
    spent = [0.0]
    orig = O.inner_solve

    def timed(*a, **k):
        t = time.perf_counter()
        r = orig(*a, **k)
        spent[0] += time.perf_counter() - t
        return r

    O.inner_solve = timed
    try:
        with threadpool_limits(limits=1):
            st = O.Settings(max_outer=1, max_inner=n_inner, delta0=1e-12)
            t0 = time.perf_counter()
            r = O.solve(prob, st)
            total = time.perf_counter() - t0
    finally:
        O.inner_solve = orig
    rate = r.counters.accepted / max(1e-9, spent[0])
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count()
    return {"value": round(rate, 3), "unit": "inner iters/s", "cores": 1, "kind": "oracle",
            "host_cpu": _cpu_model(), "host_nproc": os.cpu_count(), "host_cpus_available": avail,
            "sample": (f"one outer step of the same n={prob['n']:,} instance with the inner "
                       f"solve run for {r.counters.accepted} accepted iterations "
                       f"({r.counters.accepted // 64} stopping/restart checks); "
                       f"{spent[0]:.1f} s inside the inner solver ({total:.1f} s with the "
                       f"oracle's set-up); numpy/scipy FP64 on one thread")}


def gather_bound(P, prob, dom, precision):
    """Random-gather ceiling of the sparse products (pdnqp_probe_gather):
    gathers per second for vectors of 1-64 MB in the element size of the
    run, and what the dominant kernel's gathers cost at the rate measured
    for its own gathered vector (x, n elements).  The per-trial product
    kernels gather x[col] (Q without its diagonal, and A) or y[row] (A');
    their speed is set by this rate, not by the matrix stream's bytes."""
    import numpy as np
    eb = 8 if precision == "fp64" else 4
    table = []
    for mb in (1, 2, 4, 8, 16, 64):
        rate, _ = P.probe_gather((mb << 20) // eb, eb, 8_000_000, reps=10, seed=1)
        table.append({"vector_MB": mb, "gathers_per_s": round(rate / 1e9, 2)})
    Q = prob["Q"]
    diag = int(np.count_nonzero(Q.diagonal()))
    per_launch = {"qa_spmv": (Q.nnz - diag) + prob["A"].nnz,
                  "qa_panels": (Q.nnz - diag) + prob["A"].nnz, "at_spmv": prob["A"].nnz}
    out = {"unit": "G gathers/s", "elem_bytes": eb, "probe": table}
    g = per_launch.get(dom["name"])
    if g is not None:
        vec = prob["m"] if dom["name"] == "at_spmv" else prob["n"]
        panels = 2 if dom["name"] == "qa_panels" else 1
        rate, _ = P.probe_gather(vec, eb, g, reps=10, seed=2, panels=panels)
        out.update({"kernel": dom["name"], "gathers_per_launch": g,
                    "gathered_vector_MB": round(vec * eb / 2 ** 20, 2), "panels": panels,
                    "probe_rate_at_that_size": round(rate / 1e9, 2),
                    "gather_time_us": round(g / rate * 1e6, 2),
                    "kernel_avg_us": dom["avg_us"],
                    "gather_frac": round((g / rate * 1e6) / dom["avg_us"], 4)})
    return out


def batch_leg(P, qpgen, args):
    """Batched workload: ``count`` uneven instances (n_i ~ U{200..20000},
    m_i = n_i // 2, k_R = 5, k_A = 4) solved to 1e-4 in one persistent
    launch (FP32 bulk, FP64 reductions), each under a time limit; the
    workgroup size comes from the autotuner.  Baseline: a sample of the same
    instances solved one after another by the FP64 single-instance path."""
    import numpy as np
    probs = qpgen.batch(args.seed, args.batch_count)
    kw = dict(time_limit_s=args.batch_limit, outer_scaling=P.SCALE_RUIZ_QA)
    solvers = [P.Solver.from_problem(p, precision=P.FP32, **kw) for p in probs]
    cfg, tune_ms = P.batch_autotune(solvers, probe_inner=64)
    t0 = time.perf_counter()
    out = P.solve_batch(solvers, 1e-4, 1e-4)
    wall = time.perf_counter() - t0
    rep = P.batch_report(len(probs))
    done = rep.pop("done_ms")
    status = np.array([o[2]["status"] for o in out])
    solve_s = np.array([o[2]["solve_s"] for o in out])
    inner = np.array([o[2]["inner_accepted"] for o in out])
    ok = status == P.SOLVED
    for s in solvers:
        s.close()
    idx = np.linspace(0, len(probs) - 1, args.batch_seq_sample).astype(int) \
        if args.batch_seq_sample > 0 else np.zeros(0, dtype=int)
    seq = []
    for i in idx:
        s = P.Solver.from_problem(probs[i], precision=P.FP64, **kw)
        t1 = time.perf_counter()
        _, _, inf = s.solve(1e-4, 1e-4)
        seq.append((time.perf_counter() - t1, inf["status"] == P.SOLVED))
        s.close()
    seq_t = np.array([t for t, _ in seq]) if seq else np.zeros(1)
    return {
        "workload": (f"{len(probs)} instances, n_i ~ U{{200..20000}} (sum n {sum(p['n'] for p in probs):,}), "
                     f"m_i = n_i // 2, k_R = 5, k_A = 4, seed {args.seed}"),
        "precision": "fp32 bulk, fp64 reductions", "tol": 1e-4, "outer_scaling": "ruiz_qa",
        "time_limit_per_instance_s": args.batch_limit,
        "block": rep["block"], "waves": rep["waves"], "grid": rep["grid"],
        "lds_bytes": rep["lds_bytes"], "staged": rep["staged"],
        "autotune_ms": {f"{b}x{w}": round(x, 1) for (b, w), x in zip(P.BATCH_CONFIGS, tune_ms)},
        "wall_s": round(wall, 3), "kernel_ms": round(rep["kernel_ms"], 1),
        "solved": int(ok.sum()),
        "done_ms_p50": round(float(np.percentile(done, 50)), 1),
        "done_ms_p99": round(float(np.percentile(done, 99)), 1),
        "solve_s_p50": round(float(np.percentile(solve_s, 50)), 3),
        "solve_s_p99": round(float(np.percentile(solve_s, 99)), 3),
        "solved_solve_s_p50": round(float(np.percentile(solve_s[ok], 50)), 3) if ok.any() else None,
        "inner_iters_per_s_aggregate": round(float(inner.sum()) / max(1e-9, wall), 1),
        "sequential_fp64_sample": ({"instances": len(seq), "mean_s": round(float(seq_t.mean()), 3),
                                    "solved": int(sum(ok_ for _, ok_ in seq)),
                                    "estimate_all_s": round(float(seq_t.mean()) * len(probs), 1)}
                                   if seq else None),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-tol", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=256)
    ap.add_argument("--tol-time-limit", type=float, default=90.0)
    ap.add_argument("--tol", type=float, default=1e-4,
                    help="eps_abs = eps_rel of the time-to-tolerance solve")
    ap.add_argument("--tol-settings", default="{}",
                    help="JSON object of further pdnqp_settings fields for the time-to-tolerance "
                         "solve, e.g. '{\"anderson_mem\": 5}'")
    ap.add_argument("--tol-verbose", action="store_true",
                    help="the time-to-tolerance solve prints one line per outer step to stderr "
                         "(the library's settings.verbose)")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                    help="fp64 (the paper's arithmetic, default); fp32: FP32 matrix values and "
                         "inner vectors with FP64 reductions, FP64 outer update and final check "
                         "(the FP32-bulk extension, also timed as the other-precision leg)")
    ap.add_argument("--stream-grid", type=int, default=0,
                    help="settings.stream_grid of the timed solves (0 automatic)")
    ap.add_argument("--col-panels", type=int, default=0, choices=[0, 1, 2],
                    help="settings.col_panels of the timed solves: 0 automatic (two column "
                         "panels when x exceeds one XCD's L2), 1 never, 2 always")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched workload (512 uneven instances, one persistent launch)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-limit", type=float, default=30.0,
                    help="time limit per instance of the batched workload (s)")
    ap.add_argument("--batch-seq-sample", type=int, default=8,
                    help="instances of the batch solved one after another in FP64 as baseline "
                         "(0: none)")
    ap.add_argument("--no-other-precision", action="store_true",
                    help="skip timing the other precision on the same instance")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2609_19557_amd as P
    import qpgen

    torch.cuda.set_device(0)
    prob = qpgen.workload(args.workload, args.seed)
    print(f"[bench] instance: {_describe(prob)}", file=sys.stderr, flush=True)

    # warm-up (separate handle, same data)
    sw = P.Solver.from_problem(prob, use_torch=True, max_outer=max(1, args.warmup),
                               precision=P.FP32 if args.precision == "fp32" else P.FP64,
                               col_panels=args.col_panels,
                               stream_grid=args.stream_grid)
    sw.solve(1e-4, 1e-4)
    sw.close()
    print("[bench] warm-up done", file=sys.stderr, flush=True)

    prec = P.FP32 if args.precision == "fp32" else P.FP64
    s = P.Solver.from_problem(prob, use_torch=True, max_outer=args.steps, profile=32,
                              precision=prec, col_panels=args.col_panels,
                              stream_grid=args.stream_grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, lam, info = s.solve(1e-4, 1e-4)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps_done = int(info["outer_iters"])
    ks = s.kernel_stats()
    print(f"[bench] timed: {steps_done} outer steps, {info['inner_accepted']} accepted inner "
          f"iterations, {wall:.3f} s", file=sys.stderr, flush=True)

    kernels = []
    for k in ks:
        if k["launches"] == 0:  # the separate decision launch when it is fused
            continue
        gbs = k["bytes_per_launch"] / (k["avg_us"] * 1e-6) / 1e9 if k["avg_us"] > 0 else 0.0
        kernels.append({"name": k["name"], "launches": k["launches"],
                        "avg_us": round(k["avg_us"], 3), "total_ms": round(k["total_ms"], 3),
                        "bytes_per_launch": k["bytes_per_launch"], "GBps": round(gbs, 1)})
    dom = max(kernels, key=lambda k: k["total_ms"])
    traffic = None
    if (_kernel_source_sha() == PMC_TRAFFIC["source_sha256_prefix"] and
            args.workload == PMC_TRAFFIC["workload"]):
        traffic = PMC_TRAFFIC["bytes"]["f32" if args.precision == "fp32" else "f64"].get(dom["name"])
    roofline = {"bound": "hbm", "kernel": dom["name"], "achieved": dom["GBps"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dom["GBps"] / HBM_PEAK_GBS, 4), "traffic": traffic}
    trial_us = sum(k["avg_us"] for k in kernels)
    trial_bytes = sum(k["bytes_per_launch"] for k in kernels)

    # practical stream peak, measured while the GPU is still busy from the timed
    # solve: a plain device copy of known size (512 MB read, 512 MB written)
    a = torch.empty(64 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * a.numel() * 8 * 20 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    roofline["copy_GBps"] = round(copy_gbs, 1)
    roofline["frac_of_copy"] = round(dom["GBps"] / copy_gbs, 4)
    roofline["gather_bound"] = gather_bound(P, prob, dom, args.precision)

    ttt = None
    if not args.no_time_to_tol:
        tkw = dict(outer_scaling=P.SCALE_RUIZ_QA, time_limit_s=args.tol_time_limit,
                   precision=prec, col_panels=args.col_panels, stream_grid=args.stream_grid,
                   verbose=1 if args.tol_verbose else 0)
        tkw.update(json.loads(args.tol_settings))
        st = P.Solver.from_problem(prob, use_torch=True, **tkw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, _, inf2 = st.solve(args.tol, args.tol)
        torch.cuda.synchronize()
        ttt = {"tol": args.tol, "settings": json.loads(args.tol_settings),
               "seconds": round(time.perf_counter() - t1, 3),
               "status": inf2["status_name"],
               "outer_iters": inf2["outer_iters"], "inner_accepted": inf2["inner_accepted"],
               "outer_scaling": {P.SCALE_RUIZ_A: "ruiz_a", P.SCALE_NONE: "none",
                                 P.SCALE_RUIZ_QA: "ruiz_qa"}[tkw["outer_scaling"]],
               "r_p": inf2["r_p"], "r_d": inf2["r_d"],
               "s_p": inf2["s_p"], "s_d": inf2["s_d"],
               "inner_iters_per_s": round(inf2["inner_accepted"] / max(1e-9, inf2["solve_s"]), 1)}
        st.close()
        print(f"[bench] time-to-{args.tol:g}: {ttt}", file=sys.stderr, flush=True)

    other = None
    if not args.no_other_precision:
        oprec = P.FP64 if args.precision == "fp32" else P.FP32
        so = P.Solver.from_problem(prob, use_torch=True, max_outer=args.steps, profile=32,
                                   precision=oprec, col_panels=args.col_panels,
                                   stream_grid=args.stream_grid)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        _, _, io = so.solve(1e-4, 1e-4)
        torch.cuda.synchronize()
        wo = time.perf_counter() - t2
        other = {"precision": "fp64" if oprec == P.FP64 else "fp32 bulk, fp64 reductions",
                 "value": round(io["inner_accepted"] / wo, 2), "unit": "inner iters/s",
                 "steps": io["outer_iters"], "inner_accepted": io["inner_accepted"],
                 "kernels": [{"name": k["name"], "avg_us": round(k["avg_us"], 3),
                              "GBps": round(k["bytes_per_launch"] / (k["avg_us"] * 1e-6) / 1e9, 1)
                              if k["avg_us"] > 0 else 0.0} for k in so.kernel_stats()
                             if k["launches"] > 0]}
        so.close()
        print(f"[bench] other precision: {other}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(prob, args.cpu_iters)
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)

    batch = None
    if not args.no_batch:
        batch = batch_leg(P, qpgen, args)
        print(f"[bench] batch: {batch}", file=sys.stderr, flush=True)

    value = info["inner_accepted"] / wall
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "inner iters/s",
        "n_gpus": 1,
        "steps": steps_done,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * wall / max(1, steps_done), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {_describe(prob)}", "seed": args.seed,
                   "outer_scaling": "ruiz_a (paper)", "step": "one outer iteration",
                   "precision": ("fp32 bulk (matrix values, inner vectors), fp64 reductions, "
                                 "fp64 outer update and final check" if args.precision == "fp32"
                                 else "fp64"),
                   "inner_accepted": info["inner_accepted"], "inner_trials": info["inner_trials"],
                   "setup_s": round(info["setup_s"], 4)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_tol": ttt,
        "other_precision": other,
        "batch": batch,
        "trial": {"us_per_trial_kernels": round(trial_us, 3),
                  "bytes_per_trial": trial_bytes,
                  "GBps_per_trial": round(trial_bytes / (trial_us * 1e-6) / 1e9, 1)
                  if trial_us > 0 else None},
        "kernels": kernels,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
