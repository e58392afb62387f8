"""Training of the learned fine-level smoother on the GPU.

Training data are the inputs of the finest-level V-cycle captured while the
plain method (damped Jacobi smoother) solves a set of training problems:
seeded Gaussian-random-field wave numbers k = kbar (1 + 0.3 g) with kbar drawn
so that k spans [100, 500], on grids that resolve k_max with k_max h = 0.625
(at most 640 elements per side).  The network sees k^2 h^2 as an input, so it
is applied unchanged on grids of other sizes and resolutions.  The network (forward, backward and Adam) runs in the
library; this module only schedules problems, samples and steps.
"""
import math
import time

import numpy as np

from . import binding as B
from . import workloads as W


def training_specs(n_problems=4, p=4, kh_max=0.625, kbar_range=(100.0 / 0.7, 500.0 / 1.3), seed=7,
                   max_n_el=640):
    """Seeded training problems: (p, n_el, k_elem, source) with k in [100, 500].

    Each grid resolves its largest wave number at k_max h = kh_max; n_el is
    capped at max_n_el, the kbar draw shrunk accordingly.
    """
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_problems):
        kbar = float(rng.uniform(*kbar_range))
        n_el = int(math.ceil(1.3 * kbar / kh_max))
        if n_el > max_n_el:
            n_el = max_n_el
            kbar = kh_max * n_el / 1.3
        ke = W.grf_k(n_el, kbar=kbar, seed=int(rng.integers(1 << 30)))
        x0 = tuple(float(v) for v in rng.uniform(0.2, 0.8, size=2))
        specs.append(dict(p=p, n_el=n_el, kbar=kbar, k_elem=ke, x0=x0))
    return specs


def field_specs(n_el, p, n_problems=2, kbar_range=(100.0 / 0.7, 500.0 / 1.3), seed=11):
    """Training problems on the application's own grid: seeded random fields
    k = kbar (1 + 0.3 g) with kbar ~ U[kbar_range] (k within [100, 500]), field
    seeds 1000 + i (the workloads' own field is seed 0) and sources ~ U(0.3, 0.7)^2."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_problems):
        kbar = float(rng.uniform(*kbar_range))
        x0 = tuple(float(v) for v in rng.uniform(0.3, 0.7, size=2))
        specs.append(dict(p=p, n_el=n_el, kbar=kbar, k_elem=W.grf_k(n_el, kbar=kbar, seed=1000 + i), x0=x0))
    return specs


def capture(specs, per_problem=24, maxit=60, solver_opts=None, log=None):
    """Plain solves of the training problems; returns [(problem, solver, samples)]
    with samples a device tensor [n, N] of finest-level V-cycle inputs.  A spec
    holds p, n_el, x0 and either k_elem (per element) or k (constant); dim
    defaults to 2."""
    import torch
    out = []
    for s in specs:
        prob = B.Problem(s.get("dim", 2), s["p"], s["n_el"], k=s.get("k", 1.0), k_elem=s.get("k_elem"))
        sol = B.Solver(prob, maxit=maxit, **(solver_opts or {}))
        f = prob.point_source(s["x0"])
        buf = torch.zeros((per_problem, prob.N), dtype=torch.complex128, device="cuda")
        sol.capture(buf, per_problem)
        sol.solve(f)
        sol.capture(None, 0)
        n = sol.captured()
        out.append((prob, sol, buf[:n]))
        if log:
            log(f"[train] captured {n} samples on a {s['n_el']}-element p={s['p']} problem")
    return out


def train(net, data, steps=800, lr=3e-4, seed=0, log=None, out_weights=None):
    """Adam steps over the (problem, sample) pairs in a seeded order, in the library
    (hh_cnn_train); returns (mean loss before, mean loss after, seconds)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    l0, l1 = net.train([sol for _, sol, _ in data], [smp.contiguous() for _, _, smp in data], steps=steps, lr=lr,
                       seed=seed, out_weights=out_weights)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if log:
        log(f"[train] {steps} steps in {dt:.1f} s (mean loss over the samples included)")
    return l0, l1, dt


def trained_smoother(specs=None, steps=800, lr=3e-4, init_scale=0.05, seed=1, log=None, **capture_kw):
    """A network trained from scratch on the given (default: seeded) training problems."""
    net = B.Cnn(seed=seed)
    net.set_params(net.get_params() * (init_scale / 0.5))
    data = capture(specs or training_specs(), log=log, **capture_kw)
    l0, l1, dt = train(net, data, steps=steps, lr=lr, log=log)
    info = dict(loss_before=l0, loss_after=l1, train_s=dt, steps=steps,
                samples=int(sum(d[2].shape[0] for d in data)), problems=len(data))
    del data
    return net, info
