"""Domain extents (the axis-aligned geometry map): GPU path against the CPU oracle on
intervals, rectangles and boxes other than the unit ones.

Same bars as the other parity tests: operators and transfers 1e-13, V-cycle 1e-11,
E^-1 and T 1e-10, the solve at equal iteration count within 1e-10, the mixed FP32
V-cycle within 1e-6 of the FP64 oracle at tol 1e-10.
"""
import sys

import numpy as np
import pytest

from oracle import helmholtz as hz
from oracle import solver as osv

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def to_host(t):
    return t.cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rvec(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


CASES = {
    "1d_p3_L2.5": dict(dim=1, p=3, n_el=100, L=(2.5,), k=40.0, x0=(1.1,), opts=dict(defl_direct_max=40)),
    "2d_p3_rect": dict(dim=2, p=3, n_el=(48, 24), L=(2.0, 1.0), k=15.0, x0=(1.1, 0.4),
                       opts=dict(defl_direct_max=100, defl_kh_max=0)),
    "2d_p2_rect_randk": dict(dim=2, p=2, n_el=(40, 20), L=(1.0, 0.5), k=None, x0=(0.3, 0.2),
                             opts=dict(defl_mode=1)),
    "3d_p2_box": dict(dim=3, p=2, n_el=(16, 12, 20), L=(1.0, 0.75, 1.25), k=8.0, x0=(0.4, 0.3, 0.7),
                      opts=dict(defl_mode=1, mg_min_elems=3)),
}

_cache = {}


def k_field(c):
    if c["k"] is not None:
        return None
    rng = np.random.default_rng(8)
    return 20.0 + 10.0 * rng.random(tuple(np.atleast_1d(c["n_el"])[::-1]))


def build(name):
    if name in _cache:
        return _cache[name]
    from paper_2010_10232_amd import binding as B
    c = CASES[name]
    ke = k_field(c)
    k = c["k"] if c["k"] is not None else 1.0
    _say(f"[box {name}] oracle setup")
    op = hz.Problem(c["dim"], c["p"], c["n_el"], k, k_elem=ke, lengths=c["L"])
    osol = osv.Solver(op, osv.Options(**c["opts"]))
    _say(f"[box {name}] gpu assemble+setup")
    gp = B.Problem(c["dim"], c["p"], c["n_el"], k=k, k_elem=ke, lengths=c["L"])
    gs = B.Solver(gp, **c["opts"])
    _cache[name] = (c, op, osol, gp, gs)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_box_hierarchy_point_source_and_operators(name):
    c, op, osol, gp, gs = build(name)
    assert len(gs.levels) == len(osol.levels)
    assert gs.levels[0]["defl_direct_level"] == osol.Lz
    for g, o in zip(gs.levels, osol.levels):
        assert g["N"] == o.N
        assert abs(g["gersh"] - o.gersh) <= 1e-12 * o.gersh and abs(g["omega"] - o.omega) <= 1e-13
    _say(f"[box {name}] point source")
    f = to_host(gp.point_source(c["x0"]))
    ref = hz.point_source_rhs(op, c["x0"])
    assert np.max(np.abs(f - ref)) <= 1e-15
    assert np.array_equal(np.nonzero(f)[0], np.nonzero(ref)[0])
    for l, lv in enumerate(osol.levels):
        x = rvec(lv.N, 10 + l)
        xd = to_dev(x)
        _say(f"[box {name}] level {l} operators")
        for opname, r in (("A", lv.A @ x), ("MBETA", lv.Mb @ x), ("K", lv.K @ x), ("MK", lv.Mk @ x)):
            e = rel(to_host(gs.apply(opname, l, xd)), r)
            assert e <= 1e-13, (opname, l, e)
        if l + 1 < len(osol.levels):
            P = osol.levels[l + 1].P
            e = rel(to_host(gs.apply("RESTRICT", l, xd, out_level=l + 1)), P.T @ x)
            assert e <= 1e-13, e
            xc = rvec(P.shape[1], 20 + l)
            e = rel(to_host(gs.apply("PROLONG", l, to_dev(xc))), P @ xc)
            assert e <= 1e-13, e


@pytest.mark.parametrize("name", list(CASES))
def test_box_preconditioner_and_solve(name):
    c, op, osol, gp, gs = build(name)
    x = rvec(osol.levels[0].N, 3)
    _say(f"[box {name}] V-cycle, E^-1, T")
    e = rel(to_host(gs.apply("VCYCLE", 0, to_dev(x))), osol.vcycle(0, x))
    assert e <= 1e-11, e
    for l in range(1, osol.Lz + 1):
        xl = rvec(osol.levels[l].N, 30 + l)
        e = rel(to_host(gs.apply("EINV", l, to_dev(xl))), osol.coarse_solve(l, xl))
        assert e <= 1e-10, e
    e = rel(to_host(gs.apply("T", 0, to_dev(x))), osol.T(0, x))
    assert e <= 1e-10, e
    f = hz.point_source_rhs(op, c["x0"])
    _say(f"[box {name}] solves")
    u_ref, info_ref = osol.solve(f)
    u, info = gs.solve(to_dev(f))
    u = to_host(u)
    assert info["converged"] == 1 and info_ref.converged
    assert info["iters"] == info_ref.iters, (info["iters"], info_ref.iters)
    e = rel(u, u_ref)
    em = float(np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)))
    _say(f"[box {name}] iters {info['iters']} rel diff {e:.2e}, largest entry difference {em:.2e}")
    assert e <= 1e-10 and em <= 1e-10, (e, em)


def test_box_mixed_precision_within_1e6():
    from paper_2010_10232_amd import binding as B
    c = CASES["2d_p3_rect"]
    opts = dict(c["opts"], tol=1e-10)
    op = hz.Problem(2, c["p"], c["n_el"], c["k"], lengths=c["L"])
    u_ref, _ = osv.Solver(op, osv.Options(**opts)).solve(hz.point_source_rhs(op, c["x0"]))
    gp = B.Problem(2, c["p"], c["n_el"], k=c["k"], lengths=c["L"])
    u, info = B.Solver(gp, precision=1, **opts).solve(gp.point_source(c["x0"]))
    assert info["converged"] == 1
    assert rel(to_host(u), u_ref) <= 1e-6


def test_box_radiation_condition_on_a_longer_interval():
    """MP 1-A on (0, 2): u(0) = 1, u' - i k u = 0 at x = 2; the lifted right-hand side and
    the solve against the oracle, and the L2 error against e^{ikx} equal to the oracle's."""
    from paper_2010_10232_amd import binding as B
    p, n_el, k, L = 3, 120, 30.0, 2.0
    op = hz.Problem(1, p, n_el, k, sommerfeld=True, lengths=(L,))
    osol = osv.Solver(op, osv.Options(defl_direct_max=256, tol=1e-10))
    f_ref = hz.dirichlet_lift_rhs(op)
    gp = B.Problem(1, p, n_el, k=k, sommerfeld=True, lengths=(L,))
    f = gp.dirichlet_lift(1.0)
    assert np.max(np.abs(to_host(f) - f_ref)) <= 1e-13 * np.max(np.abs(f_ref))
    u_ref, info_ref = osol.solve(f_ref)
    u, info = B.Solver(gp, defl_direct_max=256, tol=1e-10).solve(f)
    u = to_host(u)
    assert info["converged"] == 1 and info["iters"] == info_ref.iters
    assert rel(u, u_ref) <= 1e-10
    exact = lambda x: np.exp(1j * k * x)
    e_gpu, e_ref = hz.l2_error_1d(op, u, exact), hz.l2_error_1d(op, u_ref, exact)
    assert abs(e_gpu - e_ref) <= 1e-6 * e_ref and e_ref < 1e-3
