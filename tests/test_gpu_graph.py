"""Step graphs (use_graph = 1): every outer Arnoldi step captured once per step index
into a HIP graph and replayed.  A graphed solve must be the same work as the
launched one: identical iterates, bit for bit, with the same iteration count and
residual history, on every replay (several solves in a row with other
right-hand sides and eager work between them), including inner deflation
levels, the substructured E^-1, the FP32 V-cycle and the learned smoother (the
graphs are re-captured when the smoother changes)."""
import sys

import numpy as np
import pytest

from paper_2010_10232_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "mp2a_k100_p3_160": dict(dim=2, p=3, n_el=160, k=100.0, x0s=((0.5, 0.5), (0.3, 0.7)), opts=dict()),
    # multilevel deflation: inner FGMRES steps on levels 1..2 inside every graphed step
    "2d_p3_multi": dict(dim=2, p=3, n_el=24, k=15.0, x0s=((0.5, 0.5), (0.2, 0.4)),
                        opts=dict(defl_direct_max=100, defl_kh_max=0)),
    # variable k, substructured E^-1 with its tile products and level residuals
    "2d_wedge_p3_sub": dict(dim=2, p=3, n_el=128, wedge=30.0, x0s=((0.5, 0.95), (0.5, 0.5)), opts=dict(defl_mode=1)),
    "1d_p2_k50": dict(dim=1, p=2, n_el=80, k=50.0, x0s=((0.5,), (0.21,)), opts=dict(defl_mode=1)),
    "2d_p4_mixed": dict(dim=2, p=4, n_el=40, k=25.0, x0s=((0.5, 0.5), (0.7, 0.3)), opts=dict(precision=1)),
}


def _problem(c):
    from paper_2010_10232_amd import binding as B
    ke = W.wedge_k(c["n_el"], c["wedge"]) if "wedge" in c else None
    return B.Problem(c["dim"], c["p"], c["n_el"], k=c.get("k"), k_elem=ke)


@pytest.mark.parametrize("name", list(CASES))
def test_graphed_steps_equal_launched_steps(name):
    import torch
    from paper_2010_10232_amd import binding as B
    c = CASES[name]
    prob = _problem(c)
    eager = B.Solver(prob, **c["opts"])
    graph = B.Solver(prob, use_graph=1, **c["opts"])
    fs = [prob.point_source(x0) for x0 in c["x0s"]]
    for rep, f in enumerate(fs + fs[:1] + fs[1:]):
        _say(f"[graph {name}] solve {rep}")
        ue, ie = eager.solve(f)
        he = eager.history()
        ug, ig = graph.solve(f)
        hg = graph.history()
        assert ie["converged"] == 1 and ig["converged"] == 1
        assert ie["iters"] == ig["iters"] and ie["restarts"] == ig["restarts"]
        assert torch.equal(ue, ug), float((ue - ug).abs().max())
        assert np.array_equal(he, hg)
        assert ig["model_bytes"] == ie["model_bytes"]
        # eager work between replays
        torch.cuda.synchronize()
        (f * 2.0).sum().item()


def test_graphs_recaptured_when_the_smoother_changes():
    import torch
    from paper_2010_10232_amd import binding as B
    prob = B.Problem(2, 3, 64, k=40.0)
    net = B.Cnn(seed=5)
    net.set_params(net.get_params() * 0.05)
    f = prob.point_source((0.5, 0.5))
    eager = B.Solver(prob, precision=1)
    graph = B.Solver(prob, precision=1, use_graph=1)
    for smoother in (None, net, None):
        eager.set_smoother(smoother)
        graph.set_smoother(smoother)
        _say(f"[graph smoother] {'learned' if smoother else 'jacobi'}")
        ue, ie = eager.solve(f)
        ug, ig = graph.solve(f)
        ug2, ig2 = graph.solve(f)
        assert ie["iters"] == ig["iters"] == ig2["iters"]
        assert torch.equal(ue, ug) and torch.equal(ue, ug2)
