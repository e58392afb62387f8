"""Batched solves (uneven sizes and degrees, concurrent host workers on a stream pool) against
single solves and the oracle."""
import sys

import numpy as np
import pytest

from oracle import helmholtz as hz
from oracle import solver as osv
from paper_2010_10232_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _batch_problems(n=6, seed=3):
    # a scaled-down version of the batch draws: k in [12, 48], n_el = ceil(k / 0.625)
    return W.batch_draws(n=n, seed=seed, k_lo=12.0, k_hi=48.0)


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_equals_single(precision):
    import torch
    from paper_2010_10232_amd import binding as B
    draws = _batch_problems()
    opts = dict(precision=precision, defl_direct_max=400)
    probs = [B.Problem(2, d["p"], d["n_el"], k=d["k"]) for d in draws]
    solvers = [B.Solver(pr, **opts) for pr in probs]
    fs = [pr.point_source(d["x0"]) for pr, d in zip(probs, draws)]
    _say(f"[batched precision={precision}] sizes", [pr.N for pr in probs], "p", [d["p"] for d in draws])
    us, infos = B.solve_batched(solvers, fs)
    torch.cuda.synchronize()
    for i, (s, f, u, info) in enumerate(zip(solvers, fs, us, infos)):
        _say(f"[batched precision={precision}] problem {i}: single solve")
        u1, info1 = s.solve(f)
        assert info["status"] == 0 and info["converged"] == 1
        assert info["iters"] == info1["iters"], (i, info["iters"], info1["iters"])
        d = (torch.linalg.norm(u - u1) / torch.linalg.norm(u1)).item()
        assert d <= 1e-10, (i, d)


def test_batched_matches_oracle():
    import torch
    from paper_2010_10232_amd import binding as B
    draws = _batch_problems(n=4, seed=11)
    opts = dict(defl_direct_max=400)
    probs = [B.Problem(2, d["p"], d["n_el"], k=d["k"]) for d in draws]
    solvers = [B.Solver(pr, **opts) for pr in probs]
    fs = [pr.point_source(d["x0"]) for pr, d in zip(probs, draws)]
    _say("[batched vs oracle] gpu")
    us, infos = B.solve_batched(solvers, fs)
    for i, d in enumerate(draws):
        _say(f"[batched vs oracle] problem {i} oracle p={d['p']} n_el={d['n_el']}")
        op = hz.Problem(2, d["p"], d["n_el"], d["k"])
        osol = osv.Solver(op, osv.Options(**opts))
        u_ref, info_ref = osol.solve(hz.point_source_rhs(op, d["x0"]))
        assert infos[i]["iters"] == info_ref.iters
        e = np.linalg.norm(us[i].cpu().numpy() - u_ref) / np.linalg.norm(u_ref)
        assert e <= 1e-10, (i, e)


def test_batched_rejects_duplicates():
    from paper_2010_10232_amd import binding as B
    pr = B.Problem(2, 2, 16, k=10.0)
    s = B.Solver(pr)
    f = pr.point_source((0.5, 0.5))
    with pytest.raises(B.HHError):
        B.solve_batched([s, s], [f, f.clone()])


def test_batched_repeated_calls_match_single():
    """A short restart (several cycles per solve) and three batched calls with
    eager single solves (timing switched on and off) between them: every call
    reproduces the single solves (same iterations and restarts, solutions to
    1e-10)."""
    import torch
    from paper_2010_10232_amd import binding as B
    draws = _batch_problems(n=5, seed=21)
    opts = dict(defl_direct_max=400, restart=6, maxit=120)
    probs = [B.Problem(2, d["p"], d["n_el"], k=d["k"]) for d in draws]
    solvers = [B.Solver(pr, **opts) for pr in probs]
    fs = [pr.point_source(d["x0"]) for pr, d in zip(probs, draws)]
    ref = [s.solve(f) for s, f in zip(solvers, fs)]
    assert max(r[1]["restarts"] for r in ref) >= 1
    for call in range(3):
        _say(f"[repeated batches] batched call {call + 1}")
        us, infos = B.solve_batched(solvers, fs)
        torch.cuda.synchronize()
        for i, (u, info) in enumerate(zip(us, infos)):
            u1, info1 = ref[i]
            assert info["status"] in (0, 1) and info["restarts"] == info1["restarts"]
            assert info["iters"] == info1["iters"], (call, i)
            d = (torch.linalg.norm(u - u1) / torch.linalg.norm(u1)).item()
            assert d <= 1e-10, (call, i, d)
        solvers[call].set_kernel_timing(3)
        solvers[call].solve(fs[call])
        solvers[call].set_kernel_timing(0)


def test_batched_with_graph_solvers():
    """Solvers set up with step graphs (and already replaying them) inside a
    batch: the batch launches their steps one by one, so its results equal a
    batch of the same solvers without graphs bit for bit; single solves after
    the batch replay the graphs again and reproduce the single solves before
    it."""
    import torch
    from paper_2010_10232_amd import binding as B
    draws = _batch_problems(n=5, seed=31)
    opts = dict(defl_direct_max=400)
    probs = [B.Problem(2, d["p"], d["n_el"], k=d["k"]) for d in draws]
    fs = [pr.point_source(d["x0"]) for pr, d in zip(probs, draws)]
    plain = [B.Solver(pr, **opts) for pr in probs]
    graphed = [B.Solver(pr, use_graph=1, **opts) for pr in probs]
    _say("[batched graph solvers] single solves with graphs")
    before = [s.solve(f) for s, f in zip(graphed, fs)]
    _say("[batched graph solvers] batch of plain solvers")
    u0, i0 = B.solve_batched(plain, fs)
    _say("[batched graph solvers] batch of graph solvers")
    u1, i1 = B.solve_batched(graphed, fs)
    torch.cuda.synchronize()
    for i in range(len(draws)):
        assert i1[i]["status"] == 0 and i1[i]["iters"] == i0[i]["iters"], i
        assert torch.equal(u1[i], u0[i]), i
    _say("[batched graph solvers] single solves with graphs after the batch")
    for i, (s, f) in enumerate(zip(graphed, fs)):
        u, info = s.solve(f)
        assert info["iters"] == before[i][1]["iters"], i
        assert torch.equal(u, before[i][0]), i
