"""Writes the oracle's reference values for the full-size workloads.

Calls only the CPU oracle (`oracle/`) and the seeded input generators.  For each
workload the oracle solves A u = f with the same options the library is run
with, at tol 1e-7 (the method's stopping rule, section 4.3; the GPU must take
the same number of iterations and match within 1e-10) and at tol 1e-10 (the
reference for the mixed-precision forms, which must match within 1e-6).  The
solutions are too large to keep whole, so each file keeps a seeded sample of
entries (plus the largest one) and the norms of the whole vectors:

    tests/golden/full_<workload>.npz

Run from the repository root (about an hour of CPU for all of them):

    python tests/golden/make_full_size.py [workload ...]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import helmholtz as hz  # noqa: E402
from oracle import solver as osv  # noqa: E402
from paper_2010_10232_amd import workloads as W  # noqa: E402

N_SAMPLES = 16384
# options of the library that select an implementation, not the method: the oracle has none of them
GPU_ONLY = ("defl_direct_solver", "autotune", "ortho", "time_kernels", "defl_refine")


def _batch_member(rank):
    """The rank-th largest problem of the 64-problem batch (k ~ U[50, 400], seed 0)."""
    draws = W.batch_draws(n=64, seed=0)
    order = sorted(range(len(draws)), key=lambda i: -(draws[i]["n_el"] + draws[i]["p"] - 2))
    d = draws[order[rank]]
    return dict(dim=2, p=d["p"], n_el=d["n_el"], k=d["k"], x0=d["x0"], opts=dict(defl_mode=1), member=order[rank])


WORKLOADS = {
    "wedge_k150_p2_480": dict(dim=2, p=2, n_el=480, wedge=150.0, x0=(0.5, 0.95),
                              opts=dict(defl_direct_max=65536, defl_refine=0)),
    "wedge_k150_p3_480": dict(dim=2, p=3, n_el=480, wedge=150.0, x0=(0.5, 0.95),
                              opts=dict(defl_direct_max=65536, defl_refine=0)),
    "wedge_k150_p4_480": dict(dim=2, p=4, n_el=480, wedge=150.0, x0=(0.5, 0.95),
                              opts=dict(defl_direct_max=65536, defl_refine=0)),
    "grf_k300_p4_960": dict(dim=2, p=4, n_el=960, grf=300.0, x0=(0.5, 0.5),
                            opts=dict(defl_direct_max=65536, defl_inner_its=(2, 4, 2, 1, 1, 1, 1, 1), mg_min_elems=30,
                                      defl_refine=0)),
    "batch64_largest": _batch_member(0),
    "batch64_second": _batch_member(1),
}


def k_field(w):
    if "wedge" in w:
        return W.wedge_k(w["n_el"], w["wedge"])
    if "grf" in w:
        return W.grf_k(w["n_el"], kbar=w["grf"], seed=0)
    return None


def make(name, out_dir):
    w = WORKLOADS[name]
    t0 = time.time()
    op = hz.Problem(w["dim"], w["p"], w["n_el"], w.get("k", 1.0), k_elem=k_field(w))
    f = hz.point_source_rhs(op, w["x0"])
    rec = {}
    for tol, tag in ((1e-7, ""), (1e-10, "_tol1e10")):
        s = osv.Solver(op, osv.Options(tol=tol, **{k: v for k, v in w["opts"].items() if k not in GPU_ONLY}))
        t1 = time.time()
        u, info = s.solve(f)
        print(f"[{name}] tol {tol:g}: {info.iters} iterations, relres {info.relres_true:.3e}, "
              f"setup {t1 - t0:.0f} s, solve {time.time() - t1:.0f} s", flush=True)
        N = u.shape[0]
        rng = np.random.default_rng(2024)
        idx = np.unique(np.concatenate([rng.choice(N, size=min(N_SAMPLES, N), replace=False),
                                        [int(np.argmax(np.abs(u)))]])).astype(np.int64)
        rec["iters" + tag] = info.iters
        rec["restarts" + tag] = info.restarts
        rec["relres" + tag] = info.relres_true
        rec["norm2" + tag] = float(np.linalg.norm(u))
        rec["maxabs" + tag] = float(np.max(np.abs(u)))
        rec["idx" + tag] = idx
        rec["val" + tag] = u[idx]
        t0 = time.time()
    rec["N"] = op_N = int(f.shape[0])
    assert op_N == rec["idx"].max() + 1 or rec["idx"].max() < op_N
    path = os.path.join(out_dir, f"full_{name}.npz")
    np.savez(path, **rec)
    print(f"[{name}] wrote {path}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(WORKLOADS)
    for n in names:
        make(n, os.path.dirname(os.path.abspath(__file__)))
