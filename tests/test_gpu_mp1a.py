"""MP 1-A (section 2.1) on the GPU against the CPU oracle: 1D, u(0) = 1 and the
radiation condition u' - i k u = 0 at x = 1 (the boundary term -i k B joins A and
M_beta on every level; E is complex and inverted densely).  Right-hand side of
the boundary value, level operators, Jacobi, transfers (the last function
kept), V-cycle, E^-1, T and the solve are compared element by element, and the
GPU solution is measured against the exact solution e^{ikx}."""
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
    # the paper's Table 1 setting (k = 1), two-level deflation
    "k1_p2_16": dict(p=2, n_el=16, k=1.0, opts=dict(defl_mode=1)),
    # one level only: the coarsest dense solve is the whole V-cycle, no deflation
    "k1_p5_8": dict(p=5, n_el=8, k=1.0, opts=dict(defl_mode=1)),
    "k50_p2_80": dict(p=2, n_el=80, k=50.0, opts=dict()),
    # multilevel deflation: inner FGMRES on levels 1..3, direct (complex dense) at level 4
    "k100_p3_160_multi": dict(p=3, n_el=160, k=100.0, opts=dict(defl_direct_max=20, defl_kh_max=0)),
    "k200_p4_321": dict(p=4, n_el=321, k=200.0, opts=dict(defl_mode=1)),
    "k100_p1_160": dict(p=1, n_el=160, k=100.0, opts=dict(defl_direct_max=40, defl_kh_max=0)),
}

_cache = {}


def build(name):
    if name in _cache:
        return _cache[name]
    from paper_2010_10232_amd import binding as B
    c = CASES[name]
    _say(f"[mp1a {name}] oracle setup")
    op = hz.Problem(1, c["p"], c["n_el"], c["k"], sommerfeld=True)
    osol = osv.Solver(op, osv.Options(**c["opts"]))
    _say(f"[mp1a {name}] gpu setup")
    gp = B.Problem(1, c["p"], c["n_el"], k=c["k"], sommerfeld=True)
    gs = B.Solver(gp, **c["opts"])
    _cache[name] = (c, op, osol, gp, gs)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_mp1a_hierarchy_rhs_and_operators(name):
    c, op, osol, gp, gs = build(name)
    assert gp.N == osol.levels[0].N == c["n_el"] + c["p"] - 1
    assert len(gs.levels) == len(osol.levels)
    assert gs.levels[0]["defl_direct_level"] == osol.Lz
    _say(f"[mp1a {name}] right-hand side of u(0) = 1")
    f = to_host(gp.dirichlet_lift(1.0))
    ref = hz.dirichlet_lift_rhs(op, 1.0)
    assert np.max(np.abs(f - ref)) <= 1e-14 * np.max(np.abs(ref))
    assert np.array_equal(np.nonzero(f)[0], np.nonzero(ref)[0])
    for l, lv in enumerate(osol.levels):
        g = gs.levels[l]
        assert g["N"] == lv.N
        assert abs(g["gersh"] - lv.gersh) <= 1e-12 * lv.gersh and abs(g["omega"] - lv.omega) <= 1e-13
        x = rvec(lv.N, 10 + l)
        xd = to_dev(x)
        _say(f"[mp1a {name}] level {l} A / Mbeta / K / M_k / Jacobi")
        for opn, ref in (("A", lv.A @ x), ("MBETA", lv.Mb @ x), ("K", lv.K @ x), ("MK", lv.Mk @ x),
                         ("JACOBI0", lv.omega * x / lv.D)):
            e = rel(to_host(gs.apply(opn, l, xd)), ref)
            assert e <= 1e-13, (opn, e)
        if l + 1 < len(osol.levels):
            P = osol.levels[l + 1].P
            e = rel(to_host(gs.apply("RESTRICT", l, xd, out_level=l + 1)), P.T @ x)
            assert e <= 1e-13, e
            xc = rvec(P.shape[1], 20 + l)
            e = rel(to_host(gs.apply("PROLONG", l, to_dev(xc))), P @ xc)
            assert e <= 1e-13, e


@pytest.mark.parametrize("name", list(CASES))
def test_mp1a_preconditioner(name):
    c, op, osol, gp, gs = build(name)
    N0 = osol.levels[0].N
    x = rvec(N0, 3)
    _say(f"[mp1a {name}] V-cycle, E^-1, T")
    e = rel(to_host(gs.apply("VCYCLE", 0, to_dev(x))), osol.vcycle(0, x))
    assert e <= 1e-11, e
    for l in range(1, osol.Lz + 1):
        xl = rvec(osol.levels[l].N, 30 + l)
        e = rel(to_host(gs.apply("EINV", l, to_dev(xl))), osol.coarse_solve(l, xl))
        assert e <= 1e-10, e
    e = rel(to_host(gs.apply("T", 0, to_dev(x))), osol.T(0, x))
    assert e <= 1e-10, e


@pytest.mark.parametrize("name", list(CASES))
def test_mp1a_solve_matches_oracle_and_exact_solution(name):
    c, op, osol, gp, gs = build(name)
    f = hz.dirichlet_lift_rhs(op, 1.0)
    _say(f"[mp1a {name}] oracle solve")
    u_ref, info_ref = osol.solve(f)
    _say(f"[mp1a {name}] gpu solve")
    u, info = gs.solve(gp.dirichlet_lift(1.0))
    u = to_host(u)
    assert info["converged"] == 1 and info_ref.converged
    assert info["iters"] == info_ref.iters, (info["iters"], info_ref.iters)
    e = rel(u, u_ref)
    k = c["k"]
    err_gpu = hz.l2_error_1d(op, u, lambda x: np.exp(1j * k * x))
    err_ref = hz.l2_error_1d(op, u_ref, lambda x: np.exp(1j * k * x))
    _say(f"[mp1a {name}] iters {info['iters']} rel diff {e:.2e}; L2 error vs e^(ikx): gpu {err_gpu:.3e}, "
         f"oracle {err_ref:.3e}")
    assert e <= 1e-10, e
    # |err_gpu - err_ref| <= ||u_gpu - u_ref||_L2, a few times 1e-10 of the unit-size solution
    assert abs(err_gpu - err_ref) <= 1e-9


def test_mp1a_rejected_in_2d_and_with_variable_k():
    from paper_2010_10232_amd import binding as B
    with pytest.raises(Exception):
        B.Problem(2, 2, 16, k=5.0, sommerfeld=True)
    with pytest.raises(Exception):
        B.Problem(1, 2, 16, k_elem=np.full(16, 5.0), sommerfeld=True)
