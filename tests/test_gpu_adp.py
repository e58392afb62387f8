"""ADP deflation vectors (section 3: the adapted deflation preconditioner, with
and without the weight parameter) on the GPU against the CPU oracle.

Two-level deflation with Z the quadratic rational-Bezier interpolation: the
deflation restriction and prolongation, the Galerkin matrices E = Z^T A Z (and
its K and M_k parts) on the ADP level, E^-1 (fast diagonalisation for constant
k; dense or substructured for variable k), the preconditioner T and the full
solve, each compared element-wise with the oracle.  Bars as in the other parity
tests: single FP64 passes 1e-13, E^-1 and T 1e-10, the solve at equal iteration
count 1e-10.
"""
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


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def to_host(t):
    return t.cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_max(a, b):
    """Largest entry difference relative to the largest entry."""
    mb = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0))


def rvec(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


CASES = {
    # MP 1-B (1D, constant k): D C_MG and D_eps C_MG of the paper's tables
    "1d_p2_k50": dict(dim=1, p=2, n_el=80, k=50.0, x0=(0.5,), eps=0.0),
    "1d_p5_k100_eps": dict(dim=1, p=5, n_el=128, k=100.0, x0=(0.5,), eps=0.25),
    # 2D constant k: band half-widths q = (p + 4) / 2 = 2 (p = 1) and 4 (p = 4, odd counts)
    "2d_p1_k15": dict(dim=2, p=1, n_el=32, k=15.0, x0=(0.5, 0.5), eps=0.0),
    "2d_p4_odd_eps": dict(dim=2, p=4, n_el=37, k=20.0, x0=(0.3, 0.6), eps=0.3),
    # 200^2, p = 2: the finest operator on its strip kernel, 10,000 unknowns on the ADP level
    "2d_p2_k60_200": dict(dim=2, p=2, n_el=200, k=60.0, x0=(0.5, 0.5), eps=0.1),
    # MP 2-A at k = 100, p = 3, 160^2 elements (the paper's Table 5 mesh)
    "mp2a_k100_p3_160": dict(dim=2, p=3, n_el=160, k=100.0, x0=(0.5, 0.5), eps=0.0),
    # variable k: dense E^-1 (900 unknowns), substructured E^-1 (4,096 unknowns, q = 3
    # separator bands), 1D random k
    "2d_grf_p2_60": dict(dim=2, p=2, n_el=60, grf=20.0, x0=(0.5, 0.5), eps=0.0),
    "2d_wedge_p3_128": dict(dim=2, p=3, n_el=128, wedge=30.0, x0=(0.5, 0.95), eps=0.2),
    "1d_rand_p3_300": dict(dim=1, p=3, n_el=300, rand=40.0, x0=(0.37,), eps=0.0),
}


def k_field(c):
    n = c["n_el"]
    if "wedge" in c:
        return W.wedge_k(n, c["wedge"])
    if "grf" in c:
        return W.grf_k(n, kbar=c["grf"], seed=1)
    if "rand" in c:
        return c["rand"] * (1 + 0.4 * W.uniforms(7, n))
    return None


_cache = {}


def build(name):
    if name in _cache:
        return _cache[name]
    from paper_2010_10232_amd import binding as B
    c = CASES[name]
    ke = k_field(c)
    k = c.get("k", 1.0)
    opts = dict(defl_mode=1, defl_z=1, defl_eps=c["eps"])
    _say(f"[adp {name}] oracle setup")
    op = hz.Problem(c["dim"], c["p"], c["n_el"], k, k_elem=ke)
    osol = osv.Solver(op, osv.Options(**opts))
    _say(f"[adp {name}] gpu assemble+setup")
    gp = B.Problem(c["dim"], c["p"], c["n_el"], k=k, k_elem=ke)
    gs = B.Solver(gp, **opts)
    _cache[name] = (c, op, osol, gp, gs)
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
def test_adp_level_and_operators(name):
    c, op, osol, gp, gs = build(name)
    lz = gs.levels[0]["defl_direct_level"]
    assert lz == len(gs.levels) == len(osol.levels)
    info = gs.level_info(lz)
    Z = osol.Zadp
    nf = osol.levels[0].n
    assert (info["n"][0], info["n"][1]) == (nf[0] // 2, nf[1] // 2 if c["dim"] == 2 else 1)
    assert info["N"] == Z.shape[1]
    x = rvec(Z.shape[0], 5)
    xc = rvec(Z.shape[1], 6)
    _say(f"[adp {name}] Z^T / Z")
    e = rel_max(to_host(gs.apply("ZT", 0, to_dev(x), out_level=lz)), Z.T @ x)
    assert e <= 1e-14, e
    e = rel_max(to_host(gs.apply("Z", 0, to_dev(xc))), Z @ xc)
    assert e <= 1e-14, e
    A0 = osol.levels[0]
    _say(f"[adp {name}] E = Z^T A Z, Z^T K Z, Z^T M_k Z")
    xcd = to_dev(xc)
    e = rel(to_host(gs.apply("A", lz, xcd)), osol.Eadp @ xc)
    assert e <= 1e-13, e
    e = rel(to_host(gs.apply("K", lz, xcd)), Z.T @ (A0.K @ (Z @ xc)))
    assert e <= 1e-13, e
    e = rel(to_host(gs.apply("MK", lz, xcd)), Z.T @ (A0.Mk @ (Z @ xc)))
    assert e <= 1e-13, e
    _say(f"[adp {name}] E^-1")
    e = rel(to_host(gs.apply("EINV", lz, xcd)), osol.E_lu(xc))
    assert e <= 1e-10, e
    _say(f"[adp {name}] T level 0")
    e = rel(to_host(gs.apply("T", 0, to_dev(x))), osol.T(0, x))
    assert e <= 1e-10, e


def oracle_sensitivity(osol, f, u_ref, delta=1e-12):
    """How far the oracle's own converged iterate moves when its E^-1 is perturbed by a
    relative delta per entry (seeded): two exact factorisations of E in double (the
    oracle's LU, the library's fast diagonalisation or substructuring) differ by about
    1e-12.  With the ADP vectors the FGMRES iterate is far more sensitive to that than
    with the knot-insertion ones (MP 2-A, k = 100: 1e-8 against 1e-14), although the
    iteration counts and residuals agree: the bar of the solve comparison is derived
    from it."""
    lu = osol.E_lu
    rng = np.random.default_rng(12345)
    osol.E_lu = lambda c: lu(c) * (1.0 + delta * rng.standard_normal(c.shape))
    try:
        u1, _ = osol.solve(f)
    finally:
        osol.E_lu = lu
    return rel(u1, u_ref)


@pytest.mark.parametrize("name", list(CASES))
def test_adp_solve_matches_oracle(name):
    c, op, osol, gp, gs = build(name)
    f = hz.point_source_rhs(op, c["x0"])
    _say(f"[adp {name}] oracle solve")
    u_ref, info_ref = osol.solve(f)
    sens = oracle_sensitivity(osol, f, u_ref)
    bar = max(1e-10, 3.0 * sens)
    _say(f"[adp {name}] gpu solve")
    u, info = gs.solve(to_dev(f))
    u = to_host(u)
    assert info["converged"] == 1 and info_ref.converged
    assert info["iters"] == info_ref.iters, (info["iters"], info_ref.iters)
    e, em = rel(u, u_ref), rel_max(u, u_ref)
    _say(f"[adp {name}] iters {info['iters']} rel diff {e:.2e} (max entry {em:.2e}); "
         f"oracle sensitivity {sens:.2e}, bar {bar:.1e}")
    assert e <= bar and em <= bar, (e, em, bar)
    assert abs(info["relres_true"] - info_ref.relres_true) <= 1e-3 * info_ref.relres_true + 1e-15


def test_adp_mixed_precision_within_1e6():
    """FP32 V-cycle with the ADP deflation (FP64): within 1e-6 of the FP64 oracle at tol 1e-10."""
    from paper_2010_10232_amd import binding as B
    c, op, osol, gp, _ = build("2d_p4_odd_eps")
    opts = dict(defl_mode=1, defl_z=1, defl_eps=c["eps"], tol=1e-10)
    gs32 = B.Solver(gp, precision=1, **opts)
    o64 = osv.Solver(op, osv.Options(**opts))
    f = hz.point_source_rhs(op, c["x0"])
    u, info = gs32.solve(to_dev(f))
    u_ref, _ = o64.solve(f)
    assert info["converged"] == 1
    e = rel(to_host(u), u_ref)
    _say(f"[adp mixed] iters {info['iters']} rel err {e:.2e}")
    assert e <= 1e-6, e


def test_adp_rejected_with_multilevel_deflation():
    from paper_2010_10232_amd import binding as B
    gp = B.Problem(2, 2, 16, k=5.0)
    with pytest.raises(Exception):
        B.Solver(gp, defl_mode=2, defl_z=1)
