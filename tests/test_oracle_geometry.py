"""Pins of the oracle's domain extents (the axis-aligned geometry map F(xi) = (L_d xi_d)).

Each test checks the oracle against an independent fact: the change of variables
of the 1D integrals, brute-force quadrature on a rectangle, a manufactured
solution on a rectangle, the spline's value at a physical source point, and a
direct solve.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import bspline as bs
from oracle import helmholtz as hz
from oracle import solver as osv


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_1d_change_of_variables(p):
    """x = L xi: K_L = K_1 / L and M_L = L M_1 (derivatives scale by 1/L, dx by L)."""
    L = 2.5
    K1, M1 = hz.fine_operators(hz.Problem(1, p, 13, 1.0))
    KL, ML = hz.fine_operators(hz.Problem(1, p, 13, 1.0, lengths=(L,)))
    assert abs(KL - K1 / L).max() <= 1e-13 * abs(K1).max() / L
    assert abs(ML - L * M1).max() <= 1e-13 * L * abs(M1).max()


def test_rectangle_operators_equal_brute_force_quadrature():
    """K = int grad Phi . grad Phi and M = int Phi Phi on [0, 2] x [0, 0.5] by Gauss quadrature over
    the physical elements, the basis evaluated on breakpoints built here."""
    p, n_el, L = 2, (3, 4), (2.0, 0.5)
    k = 1.5
    K, Mk = hz.fine_operators(hz.Problem(2, p, n_el, k, lengths=L))
    bks = [np.linspace(0.0, L[d], n_el[d] + 1) for d in range(2)]
    m = [n + p for n in n_el]
    gx, gw = bs.gauss_legendre(p + 2)
    Kr = np.zeros((m[0] * m[1],) * 2)
    Mr = np.zeros_like(Kr)
    for e2 in range(n_el[1]):
        for e1 in range(n_el[0]):
            for qy, wy in zip(gx, gw):
                lo, hi = bks[1][e2], bks[1][e2 + 1]
                y = lo + (qy + 1) * 0.5 * (hi - lo)
                vy, dy = bs.basis_and_derivative_all(bks[1], p, y, elem=e2)
                jy = 0.5 * (hi - lo)
                for qx, wx in zip(gx, gw):
                    lo1, hi1 = bks[0][e1], bks[0][e1 + 1]
                    x = lo1 + (qx + 1) * 0.5 * (hi1 - lo1)
                    vx, dx = bs.basis_and_derivative_all(bks[0], p, x, elem=e1)
                    w = wx * wy * jy * 0.5 * (hi1 - lo1)
                    phi = np.outer(vy, vx).ravel()
                    gxv = np.outer(vy, dx).ravel()
                    gyv = np.outer(dy, vx).ravel()
                    Mr += w * np.outer(phi, phi)
                    Kr += w * (np.outer(gxv, gxv) + np.outer(gyv, gyv))
    idx = [i2 * m[0] + i1 for i2 in range(1, m[1] - 1) for i1 in range(1, m[0] - 1)]
    Kr, Mr = Kr[np.ix_(idx, idx)], Mr[np.ix_(idx, idx)]
    assert np.allclose(K.toarray(), Kr, rtol=1e-12, atol=1e-12 * np.abs(Kr).max())
    assert np.allclose(Mk.toarray(), k * k * Mr, rtol=1e-12, atol=1e-12 * k * k * np.abs(Mr).max())


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rectangle_manufactured_solution_rate(p):
    """u = sin(pi x / 2) sin(2 pi y / 0.5) on [0, 2] x [0, 0.5] (zero on the boundary), k = 2:
    the L2 error falls as h^(p+1)."""
    L, k = (2.0, 0.5), 2.0
    a = (np.pi / L[0], 2 * np.pi / L[1])
    lam = a[0] ** 2 + a[1] ** 2 - k * k
    nq = p + 4
    gx, gw = bs.gauss_legendre(nq)
    errs = []
    for n in (6, 12):
        prob = hz.Problem(2, p, (n, n), k, lengths=L)
        K, Mk = hz.fine_operators(prob)

        def tab(d):
            b = prob.breakpoints(d)
            pts, wts, B = [], [], []
            for e in range(n):
                lo, hi = b[e], b[e + 1]
                jac = 0.5 * (hi - lo)
                for xq, wq in zip(gx, gw):
                    x = lo + (xq + 1) * jac
                    pts.append(x)
                    wts.append(wq * jac)
                    B.append(bs.basis_all(b, p, x, elem=e))
            return np.array(pts), np.array(wts), np.array(B)

        (xs, wx, Bx), (ys, wy, By) = tab(0), tab(1)
        fx = (wx * np.sin(a[0] * xs)) @ Bx
        fy = (wy * np.sin(a[1] * ys)) @ By
        f = lam * np.kron(fy[1:-1], fx[1:-1])
        u = spla.spsolve((K - Mk).tocsc(), f)
        U = np.zeros((n + p, n + p))
        U[1:-1, 1:-1] = u.reshape(n + p - 2, n + p - 2)
        uh = By @ U @ Bx.T
        ex = np.sin(a[1] * ys)[:, None] * np.sin(a[0] * xs)[None, :]
        errs.append(np.sqrt(np.sum(wy[:, None] * wx[None, :] * (uh - ex) ** 2)))
    rate = np.log2(errs[0] / errs[1])
    assert rate > p + 1 - 0.4, (errs, rate)


def test_physical_source_point():
    """c . f = u_h(x0) at a physical point of [0, 2] x [0, 0.5]; spans from x0 / L."""
    p, n_el, L = 3, (10, 7), (2.0, 0.5)
    prob = hz.Problem(2, p, n_el, 4.0, lengths=L)
    x0 = (1.3, 0.2)
    assert hz.source_spans(prob, x0) == [int(np.floor(1.3 / 2.0 * 10)), int(np.floor(0.2 / 0.5 * 7))]
    f = hz.point_source_rhs(prob, x0).real
    n = [m + p - 2 for m in n_el]
    c = np.random.default_rng(3).standard_normal(n[0] * n[1])
    vx = bs.basis_all(np.linspace(0, 2.0, 11), p, 1.3)[1:-1]
    vy = bs.basis_all(np.linspace(0, 0.5, 8), p, 0.2)[1:-1]
    uh = vy @ c.reshape(n[1], n[0]) @ vx
    assert abs(c @ f - uh) <= 1e-12 * max(1.0, abs(uh))


def test_physical_source_point_3d():
    """c . f = u_h(x0) at a physical point of [0, 1] x [0, 0.6] x [0, 0.8]; spans from x0 / L."""
    p, n_el, L = 2, (6, 5, 7), (1.0, 0.6, 0.8)
    prob = hz.Problem(3, p, n_el, 4.0, lengths=L)
    x0 = (0.7, 0.2, 0.5)
    assert hz.source_spans(prob, x0) == [int(np.floor(x0[d] / L[d] * n_el[d])) for d in range(3)]
    f = hz.point_source_rhs(prob, x0).real
    n = [m + p - 2 for m in n_el]
    c = np.random.default_rng(4).standard_normal(n[0] * n[1] * n[2])
    v = [bs.basis_all(np.linspace(0, L[d], n_el[d] + 1), p, x0[d])[1:-1] for d in range(3)]
    uh = np.einsum("kji,k,j,i->", c.reshape(n[2], n[1], n[0]), v[2], v[1], v[0])
    assert abs(c @ f - uh) <= 1e-12 * max(1.0, abs(uh))
    assert np.count_nonzero(f) == (p + 1) ** 3


@pytest.mark.parametrize("dim,n_el,L", [(1, 60, (3.0,)), (2, (24, 12), (2.0, 1.0)), (3, (12, 8, 10), (1.0, 0.6, 0.8))])
def test_solver_on_a_box_matches_direct_solve(dim, n_el, L):
    prob = hz.Problem(dim, 2, n_el, 8.0, lengths=L)
    s = osv.Solver(prob, osv.Options(defl_mode=1, mg_min_elems=3, tol=1e-10))
    x0 = tuple(0.37 * v for v in L)
    f = hz.point_source_rhs(prob, x0)
    u, info = s.solve(f)
    assert info.converged
    ud = spla.spsolve(s.levels[0].A.tocsc().astype(complex), f)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) <= 1e-7
