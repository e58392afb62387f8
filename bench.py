"""Benchmark: deflated, multigrid-approximated CSLP + FGMRES solve of the B-spline
Helmholtz system on one MI355X.

One step = one complete solve to ||f - A u|| <= 1e-7 ||f|| (every kernel of
the hot path: operator applies, V-cycles, transfers, deflation, Arnoldi/MGS,
Givens, updates) on a right-hand side already resident in HBM.  The metric is
DoF-iterations per second: N x (outer FGMRES iterations) / solve time.

Prints ONE JSON line.  `value` is the plain FP64 form.  Extra fields:
`roofline` for the kernel class that takes the most device time in the solve
(timed live with HIP events on the library's stream inside the timed region),
`mixed_learned` (the same workload solved with the FP32 V-cycle and the learned
fine-level smoother, the network trained on the GPU beforehand on other
problems of the same grid; training time reported, not timed), and
`cpu_baseline` (the CPU oracle timed on the host, same workload, one thread).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from paper_2010_10232_amd import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
# rocprofv3 traffic summaries (written by paper_2010_10232_amd.profiling) per kernel class
TRAFFIC_PREFIX = {1: "fine_op", 2: "einv", 3: "arnoldi"}
CLASS_NAMES = {1: "finest-level operator (stencil) kernel", 2: "exact E^-1 solve (direct deflation level)",
               3: "outer Arnoldi MGS kernel"}

WORKLOADS = {
    # MP 2-A mesh of the paper's table (k = 100, p = 3, 160 x 160 elements): the default
    "mp2a_k100_p3_160": dict(dim=2, p=3, n_el=160, k=100.0, x0=(0.5, 0.5), opts=dict()),
    # MP 1-B: 1D, k = 50, p = 2, 80 elements, two-level deflation
    "mp1b_k50_p2_80": dict(dim=1, p=2, n_el=80, k=50.0, x0=(0.5,), opts=dict(defl_mode=1)),
    # three-layer wedge, k0 = 150, p = 3, 480 x 480 elements, FP64 or mixed
    # (direct deflation level up to 65536 unknowns: level 1, k h <= 1.25 there)
    "wedge_k150_p3_480": dict(dim=2, p=3, n_el=480, wedge=150.0, x0=(0.5, 0.95),
                              opts=dict(defl_direct_max=65536)),
    # Gaussian random field k = 300 (1 + 0.3 g), p = 4, 960 x 960 elements
    # (direct deflation level 2, 58,564 unknowns)
    "grf_k300_p4_960": dict(dim=2, p=4, n_el=960, grf=300.0, x0=(0.5, 0.5), opts=dict(defl_direct_max=65536)),
    # 64 independent constant-k problems, k ~ U[50, 400], n_el = ceil(k / 0.625),
    # p ~ U{2, 3, 4}, random interior sources; FP32 V-cycle, FP64 Krylov and deflation
    "batch64_k50_400": dict(batch=64, seed=0, opts=dict(precision=1, maxit=400)),
}


def measure_copy_gbs(mib=1024, reps=5):
    """Achieved bandwidth of a plain 1 GiB device-to-device copy (read + write bytes / time), the
    practical ceiling next to the 8 TB/s vendor peak."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 8 / (best * 1e-3) / 1e9


def k_field(w):
    if "wedge" in w:
        return W.wedge_k(w["n_el"], w["wedge"])
    if "grf" in w:
        return W.grf_k(w["n_el"], kbar=w["grf"], seed=0)
    return None


def cpu_baseline(w, seconds_cap=30.0):
    """The CPU oracle on the same workload (one thread), solve only (setup excluded)."""
    from threadpoolctl import threadpool_limits

    from oracle import helmholtz as hz
    from oracle import solver as osv
    with threadpool_limits(limits=1):
        ke = k_field(w)
        op = hz.Problem(w["dim"], w["p"], w["n_el"], w.get("k", 1.0), k_elem=ke)
        s = osv.Solver(op, osv.Options(**w["opts"]))
        f = hz.point_source_rhs(op, w["x0"])
        t0 = time.perf_counter()
        u, info = s.solve(f)
        dt = time.perf_counter() - t0
    N = s.levels[0].N
    return {"value": N * info.iters / dt, "unit": "DoF-iter/s", "cores": 1, "kind": "oracle",
            "sample": f"one full solve of the same workload ({info.iters} iterations, {dt:.1f} s, setup excluded)",
            "iters": info.iters}


def learned_specs(w, n_problems=2, seed=11):
    """Training problems for the learned smoother: the workload's grid and degree with other
    random fields (seeds other than the test field's, kbar scaled by U[0.7, 1]), other wedge
    scales (k0 scaled by U[0.8, 1]), or, for constant k, other source positions; never the
    test problem itself."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_problems):
        x0 = tuple(float(v) for v in rng.uniform(0.3, 0.7, size=w["dim"]))
        sp = dict(dim=w["dim"], p=w["p"], n_el=w["n_el"], x0=x0)
        if "grf" in w:
            sp["k_elem"] = W.grf_k(w["n_el"], kbar=w["grf"] * float(rng.uniform(0.7, 1.0)), seed=1000 + i)
        elif "wedge" in w:
            sp["k_elem"] = W.wedge_k(w["n_el"], w["wedge"] * float(rng.uniform(0.8, 1.0)))
        else:
            sp["k"] = w["k"]
        specs.append(sp)
    return specs


def run_learned(args, w, prob, f, plain_ms):
    """Mixed form (FP32 V-cycle) with the learned fine-level smoother, trained on the GPU from
    scratch on learned_specs(w); the timed solves are those of the test problem."""
    import torch

    from paper_2010_10232_amd import binding as B
    from paper_2010_10232_amd import learned as L
    t0 = time.perf_counter()
    data = L.capture(learned_specs(w), per_problem=30, maxit=40,
                     solver_opts=dict(precision=1, **w["opts"]),
                     log=lambda m: print(m, file=sys.stderr, flush=True))
    net = B.Cnn(seed=1)
    net.set_params(net.get_params() * 0.1)
    l0, l1, t_train = L.train(net, data, steps=900, lr=3e-4)
    samples = int(sum(d[2].shape[0] for d in data))
    del data
    torch.cuda.empty_cache()
    t_prep = time.perf_counter() - t0
    print(f"[bench] learned smoother: loss {l0:.3f} -> {l1:.3f}, training {t_train:.1f} s", file=sys.stderr,
          flush=True)
    solver = B.Solver(prob, precision=1, **w["opts"])
    solver.set_smoother(net)
    u = torch.empty_like(f)
    for _ in range(max(args.warmup, 1)):
        solver.solve(f, u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [solver.solve(f, u)[1] for _ in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    return {"form": "mixed (FP32 V-cycle) + learned fine-level smoother",
            "value": prob.N * sum(i["iters"] for i in infos) / dt, "unit": "DoF-iter/s",
            "ms_per_step": ms, "iters_per_solve": infos[0]["iters"],
            "relres_true": infos[-1]["relres_true"], "converged": all(i["converged"] == 1 for i in infos),
            "speedup_vs_plain": plain_ms / ms,
            "training": {"problems": len(learned_specs(w)), "samples": samples, "steps": 900, "lr": 3e-4,
                         "loss_before": l0, "loss_after": l1, "train_s": round(t_train, 2),
                         "capture_and_train_s": round(t_prep, 2),
                         "recipe": "same grid and degree, other fields / sources (bench.learned_specs)"}}


def batch_member_opts(d, base):
    """Deflation per batch member: two-level with the exact E^-1 on level 1 (constant k: fast
    diagonalisation, affordable at every member size)."""
    o = dict(base)
    o.update(defl_mode=1)
    return o


def run_batched(args, w):
    """64-problem lockstep batch: one step = one hh_solve_batched of the whole batch."""
    import torch

    from paper_2010_10232_amd import binding as B
    draws = W.batch_draws(n=w["batch"], seed=w["seed"])
    t0 = time.perf_counter()
    probs, solvers = [], []
    for i, d in enumerate(draws):
        probs.append(B.Problem(2, d["p"], d["n_el"], k=d["k"]))
        solvers.append(B.Solver(probs[-1], **batch_member_opts(d, w["opts"])))
        print(f"[bench] setup {i + 1}/{len(draws)}: p={d['p']} n_el={d['n_el']} N={probs[-1].N} "
              f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    fs = [pr.point_source(d["x0"]) for pr, d in zip(probs, draws)]
    us = [torch.empty_like(f) for f in fs]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    for _ in range(args.warmup):
        _, infos = B.solve_batched(solvers, fs, us)
        print(f"[bench] warm-up batch: iterations {[i['iters'] for i in infos]}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    work = 0
    for k in range(args.steps):
        _, infos = B.solve_batched(solvers, fs, us)
        work += sum(pr.N * inf["iters"] for pr, inf in zip(probs, infos))
        print(f"[bench] timed batch {k + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same problems one after another (single-solve path) for comparison
    t1 = time.perf_counter()
    for s_, f_, u_ in zip(solvers, fs, us):
        s_.solve(f_, u_)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    out = {
        "metric": "DoF-iterations/s of the deflated MG-CSLP FGMRES solve to 1e-7 relative residual",
        "value": work / dt, "unit": "DoF-iter/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": args.workload, "problems": len(probs),
                   "N_total": int(sum(pr.N for pr in probs)),
                   "N_range": [int(min(pr.N for pr in probs)), int(max(pr.N for pr in probs))],
                   "iters_range": [min(i["iters"] for i in infos), max(i["iters"] for i in infos)],
                   "converged": int(sum(i["converged"] == 1 for i in infos)),
                   "setup_s": round(t_setup, 2), "sequential_single_solves_ms": round(t_seq * 1e3, 2)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(draws, w["opts"])
    print(json.dumps(out), flush=True)


def cpu_baseline_batch(draws, opts, budget_s=20.0):
    """The oracle on the smallest problems of the batch until about budget_s of solve time."""
    from threadpoolctl import threadpool_limits

    from oracle import helmholtz as hz
    from oracle import solver as osv
    order = sorted(range(len(draws)), key=lambda i: draws[i]["n_el"] * draws[i]["p"])
    o = {k: v for k, v in opts.items() if k != "precision"}
    work, spent, done = 0, 0.0, 0
    with threadpool_limits(limits=1):
        for i in order:
            d = draws[i]
            op = hz.Problem(2, d["p"], d["n_el"], d["k"])
            s = osv.Solver(op, osv.Options(**batch_member_opts(d, o)))
            f = hz.point_source_rhs(op, d["x0"])
            t0 = time.perf_counter()
            _, info = s.solve(f)
            spent += time.perf_counter() - t0
            work += s.levels[0].N * info.iters
            done += 1
            if spent >= budget_s:
                break
    return {"value": work / spent, "unit": "DoF-iter/s", "cores": 1, "kind": "oracle",
            "sample": f"the {done} smallest problems of the batch solved one by one in FP64 "
                      f"({spent:.1f} s of solve time, setup excluded)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mp2a_k100_p3_160", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", type=int, default=0, help="0 FP64, 1 FP32 V-cycle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the mixed + learned-smoother form (trained on the GPU before its timing)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="run one plain device copy of this many MiB first (PMC traffic calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2010_10232_amd import binding as B
    torch.cuda.set_device(0)
    if "batch" in WORKLOADS[args.workload]:
        return run_batched(args, WORKLOADS[args.workload])
    if args.calibrate_copy_mb:
        n = args.calibrate_copy_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # a counter run keeps the calibration copy the largest copy of the process
    copy_gbs = None if args.calibrate_copy_mb else measure_copy_gbs()
    w = WORKLOADS[args.workload]
    ke = k_field(w)
    t0 = time.perf_counter()
    prob = B.Problem(w["dim"], w["p"], w["n_el"], k=w.get("k"), k_elem=ke)
    solver = B.Solver(prob, precision=args.precision, **w["opts"])
    f = prob.point_source(w["x0"])
    u = torch.empty_like(f)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    N = prob.N
    print(f"[bench] {args.workload}: N = {N}, setup {t_setup:.2f} s", file=sys.stderr, flush=True)

    for i in range(args.warmup):
        _, inf = solver.solve(f, u)
        print(f"[bench] warm-up solve {i + 1}/{args.warmup}: {inf['iters']} iterations, "
              f"relres {inf['relres_true']:.2e}", file=sys.stderr, flush=True)
    # dominant kernel class: the one with the most device time in one solve
    per_class = {}
    for cls in (1, 2, 3):
        solver.set_kernel_timing(cls)
        _, inf = solver.solve(f, u)
        per_class[cls] = inf["op_ms_total"]
        print(f"[bench] kernel class {cls}: {per_class[cls]:.3f} ms per solve", file=sys.stderr, flush=True)
    dom = max(per_class, key=per_class.get)
    solver.set_kernel_timing(dom)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, k_ms, k_n, k_bytes = [], 0.0, 0, 0.0
    infos = []
    for i in range(args.steps):
        _, inf = solver.solve(f, u)
        infos.append(inf)
        if N >= 200000:
            print(f"[bench] timed solve {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for inf in infos:
        iters.append(inf["iters"])
        k_ms += inf["op_ms_total"]
        k_n += inf["op_launches"]
        k_bytes += inf["op_bytes_per_launch"] * inf["op_launches"]
    solver.set_kernel_timing(0)
    ms_per_step = dt * 1e3 / args.steps
    value = N * sum(iters) / dt
    achieved = (k_bytes / (k_ms * 1e-3)) / 1e9 if k_ms > 0 else None
    from paper_2010_10232_amd import profiling
    tr = profiling.read_summary(os.path.join(ROOT, "profiles",
                                             f"{TRAFFIC_PREFIX[dom]}_{args.workload}_traffic.md"))
    traffic = tr[0] if tr else None
    out = {
        "metric": "DoF-iterations/s of the deflated MG-CSLP FGMRES solve to 1e-7 relative residual",
        "value": value,
        "unit": "DoF-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "dim": w["dim"], "p": w["p"], "n_el": w["n_el"],
                   "N": N, "precision": "fp64" if args.precision == 0 else "mixed (fp32 V-cycle)",
                   "iters_per_solve": iters[0], "relres_true": infos[-1]["relres_true"],
                   "setup_s": round(t_setup, 3), "solve_ms": ms_per_step},
        "roofline": {"bound": "hbm", "kernel": CLASS_NAMES[dom],
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                     "copy_GBps_measured": round(copy_gbs, 1) if copy_gbs else None,
                     "launches": k_n, "avg_us": (k_ms * 1e3 / k_n) if k_n else None,
                     "bytes_per_launch": (k_bytes / k_n) if k_n else None,
                     "class_ms_per_solve": {CLASS_NAMES[c]: round(v, 4) for c, v in per_class.items()}},
    }
    if not args.no_learned and args.precision == 0:
        try:
            out["mixed_learned"] = run_learned(args, w, prob, f, ms_per_step)
        except Exception as e:  # reported, not hidden: the plain result above stands
            out["mixed_learned"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
