"""Pins of the oracle's unit-cube (3D tensor-product) discretisation and solver.

Each test checks the oracle against an independent fact: brute-force
quadrature of the 3D Galerkin integrals, direct evaluation of the spline at the
source point, the convergence rate of a manufactured solution, nested-space
Galerkin identities and a direct solve.  Meshes are anisotropic so that a
swapped direction or Kronecker factor changes the result.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import bspline as bs
from oracle import helmholtz as hz
from oracle import solver as osv


def _full_3d_galerkin(n_el, p, lengths=(1.0, 1.0, 1.0)):
    """K and M of the full 3D tensor basis by Gauss quadrature over every element of the box
    [0, L1] x [0, L2] x [0, L3]: K = int grad Phi_I . grad Phi_J, M = int Phi_I Phi_J, with Phi_I
    at index (i3 * m2 + i2) * m1 + i1 (m_d = n_el_d + p functions per direction)."""
    bks = [np.linspace(0.0, L, n + 1) for n, L in zip(n_el, lengths)]
    m = [n + p for n in n_el]
    gx, gw = bs.gauss_legendre(p + 2)
    Ntot = m[0] * m[1] * m[2]
    K = np.zeros((Ntot, Ntot))
    M = np.zeros((Ntot, Ntot))
    # per direction: the points, weights, values and derivatives of all functions
    tabs = []
    for d in range(3):
        b = bks[d]
        rows = []
        for e in range(n_el[d]):
            lo, hi = b[e], b[e + 1]
            jac = 0.5 * (hi - lo)
            pts = []
            for xq, wq in zip(gx, gw):
                x = lo + (xq + 1) * jac
                v, dv = bs.basis_and_derivative_all(b, p, x, elem=e)
                pts.append((wq * jac, v, dv))
            rows.append(pts)
        tabs.append(rows)
    for e3 in range(n_el[2]):
        for e2 in range(n_el[1]):
            for e1 in range(n_el[0]):
                for wz, vz, dz in tabs[2][e3]:
                    for wy, vy, dy in tabs[1][e2]:
                        for wx, vx, dx in tabs[0][e1]:
                            w = wx * wy * wz
                            phi = np.einsum("k,j,i->kji", vz, vy, vx).ravel()
                            gxv = np.einsum("k,j,i->kji", vz, vy, dx).ravel()
                            gyv = np.einsum("k,j,i->kji", vz, dy, vx).ravel()
                            gzv = np.einsum("k,j,i->kji", dz, vy, vx).ravel()
                            M += w * np.outer(phi, phi)
                            K += w * (np.outer(gxv, gxv) + np.outer(gyv, gyv) + np.outer(gzv, gzv))
    idx = [(i3 * m[1] + i2) * m[0] + i1 for i3 in range(1, m[2] - 1) for i2 in range(1, m[1] - 1)
           for i1 in range(1, m[0] - 1)]
    return K[np.ix_(idx, idx)], M[np.ix_(idx, idx)]


@pytest.mark.parametrize("p,n_el", [(1, (3, 2, 4)), (2, (2, 3, 4)), (3, (3, 2, 2))])
def test_3d_operators_equal_brute_force_quadrature(p, n_el):
    k = 2.5
    K, Mk = hz.fine_operators(hz.Problem(3, p, n_el, k))
    Kr, Mr = _full_3d_galerkin(n_el, p)
    assert K.shape == Kr.shape
    assert np.allclose(K.toarray(), Kr, rtol=1e-12, atol=1e-12 * np.abs(Kr).max())
    assert np.allclose(Mk.toarray(), k * k * Mr, rtol=1e-12, atol=1e-12 * k * k * np.abs(Mr).max())


def test_3d_box_operators_equal_brute_force_quadrature():
    """On [0, 1.4] x [0, 0.6] x [0, 1.0] (three different lengths, meshes of different sizes):
    a length applied to the wrong direction changes K (M depends on the lengths' product only, and
    pins that)."""
    p, n_el, L, k = 2, (3, 2, 4), (1.4, 0.6, 1.0), 1.5
    K, Mk = hz.fine_operators(hz.Problem(3, p, n_el, k, lengths=L))
    Kr, Mr = _full_3d_galerkin(n_el, p, L)
    assert np.allclose(K.toarray(), Kr, rtol=1e-12, atol=1e-12 * np.abs(Kr).max())
    assert np.allclose(Mk.toarray(), k * k * Mr, rtol=1e-12, atol=1e-12 * k * k * np.abs(Mr).max())


@pytest.mark.parametrize("p", [2, 3])
def test_3d_point_source_is_the_spline_value_at_the_source(p):
    """c . f = u_h(x0) for any coefficients c: f_I = Phi_I(x0), evaluated here by
    contracting the coefficient array with each direction's basis values."""
    n_el = (5, 7, 6)
    x0 = (0.23, 0.61, 0.82)
    prob = hz.Problem(3, p, n_el, 4.0)
    f = hz.point_source_rhs(prob, x0)
    n = [m + p - 2 for m in n_el]
    rng = np.random.default_rng(5)
    c = rng.standard_normal(n[2] * n[1] * n[0])
    vals = [bs.basis_all(bs.uniform_breakpoints(m), p, x)[1:-1] for m, x in zip(n_el, x0)]
    U = c.reshape(n[2], n[1], n[0])
    uh = np.einsum("kji,k,j,i->", U, vals[2], vals[1], vals[0])
    assert abs(c @ f.real - uh) <= 1e-13 * max(1.0, abs(uh))
    assert abs(f.real.sum() - 1.0) < 1e-14     # interior source: partition of unity
    assert np.count_nonzero(f) == (p + 1) ** 3


@pytest.mark.parametrize("p", [1, 2, 3])
def test_3d_manufactured_solution_rate(p):
    """L2 error O(h^{p+1}) (section 4.1's rate, carried to the cube): u = sin(pi x) sin(2 pi y)
    sin(pi z), k = 2, Dirichlet on the whole boundary."""
    freqs = (1, 2, 1)
    errs = []
    for n_el in (4, 8):
        prob = hz.Problem(3, p, n_el, 2.0)
        K, Mk = hz.fine_operators(prob)
        f = hz.manufactured_rhs_3d(prob, freqs)
        u = spla.spsolve((K - Mk).tocsc(), f)
        errs.append(hz.l2_error_3d(prob, u, freqs))
    rate = np.log2(errs[0] / errs[1])
    assert rate > p + 1 - 0.4, (errs, rate)


@pytest.mark.parametrize("p", [2, 3])
def test_3d_galerkin_equals_rediscretisation(p):
    """Nested spaces: P^T K_f P and P^T M_f P on level 1 equal the operators assembled on
    the halved mesh (pins the order of the three prolongation factors)."""
    prob = hz.Problem(3, p, (8, 6, 10), 3.0)
    lev = osv.build_hierarchy(prob, osv.Options(mg_min_elems=3))
    assert [len(b) - 1 for b in lev[1].bks] == [4, 3, 5]
    Kc, Mc = hz.fine_operators(hz.Problem(3, p, (4, 3, 5), 3.0))
    assert abs(lev[1].K - Kc).max() <= 1e-11 * abs(Kc).max()
    assert abs(lev[1].Mk - Mc).max() <= 1e-13 * abs(Mc).max()
    assert lev[1].P.shape == (lev[0].N, lev[1].N)


@pytest.mark.parametrize("defl_mode", [0, 1, 2])
def test_3d_solver_matches_direct_solve(defl_mode):
    prob = hz.Problem(3, 2, (12, 10, 14), 8.0)
    extra = dict(defl_direct_max=64, defl_kh_max=0) if defl_mode == 2 else {}
    s = osv.Solver(prob, osv.Options(defl_mode=defl_mode, mg_min_elems=3, tol=1e-10, **extra))
    f = hz.point_source_rhs(prob, (0.4, 0.55, 0.3))
    u, info = s.solve(f)
    assert info.converged and info.relres_true <= 1e-10
    ud = spla.spsolve(s.levels[0].A.tocsc().astype(complex), f)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) <= 1e-7
    if defl_mode == 1:
        assert s.Lz == 1
    if defl_mode == 2:
        # multilevel: an inner FGMRES on level 1, the exact solve further down (the k h rule is
        # off, so that on this small mesh the deflation reaches past level 1)
        assert s.Lz >= 2 and s.levels[s.Lz].N <= 64 < s.levels[1].N


def test_3d_rejects_variable_k_and_other_preconditioners():
    with pytest.raises(ValueError):
        hz.Problem(3, 2, 4, 2.0, k_elem=np.ones((4, 4, 4)))
    prob = hz.Problem(3, 2, 4, 2.0)
    with pytest.raises(ValueError):
        osv.Solver(prob, osv.Options(precond=1))



@pytest.mark.parametrize("p,n_el,k", [(2, (20, 8, 10), 6.0), (3, 12, 6.0)])
def test_3d_finest_level_damping_keeps_the_vcycle_contracting(p, n_el, k):
    """On the cube D^-1 M_beta of the finest level reaches beyond 2/omega (omega = 0.8): with the
    coarse levels damped and the finest one not, the V-cycle iteration x <- x - V(M_beta x)
    grows; with omega_0 = min(omega, 2/g_0) on the finest level as well it contracts."""
    prob = hz.Problem(3, p, n_el, k)
    s = osv.Solver(prob, osv.Options(defl_mode=0, mg_min_elems=3))
    lv = s.levels[0]
    assert 2.0 / lv.gersh < 0.8 and lv.omega == 2.0 / lv.gersh
    rng = np.random.default_rng(2)
    x1 = rng.standard_normal(lv.N) + 0j
    growth = {}
    for om in (0.8, lv.omega):
        lv.omega = om
        x = x1.copy()
        for _ in range(15):
            x = x - s.vcycle(0, lv.Mb @ x)
        growth[om] = np.linalg.norm(x) / np.linalg.norm(x1)
    assert growth[0.8] > 1.0 and growth[lv.omega] < 0.5, growth



def test_3d_adp_vectors_are_the_tensor_product_and_deflate():
    """ADP on the cube: Z = Z_z (x) Z_y (x) Z_x with x fastest (each column the product of three
    1D columns), the deflation identities P_D A Z = 0, Q A Z = Z hold, and the ADP-deflated
    solve reaches the direct solution."""
    prob = hz.Problem(3, 3, (10, 8, 12), 6.0)
    n = [m + 1 for m in prob.n_el]
    Z = osv.adp_deflation(n, 3, 0.2).toarray()
    Zs = [osv.adp_deflation_1d(m, 0.2).toarray() for m in n]
    nc = [z.shape[1] for z in Zs]
    rng = np.random.default_rng(4)
    for _ in range(20):
        J = [int(rng.integers(0, c)) for c in nc]
        col = Z[:, (J[2] * nc[1] + J[1]) * nc[0] + J[0]].reshape(n[2], n[1], n[0])
        ref = np.einsum("k,j,i->kji", Zs[2][:, J[2]], Zs[1][:, J[1]], Zs[0][:, J[0]])
        assert np.array_equal(col, ref)
    s = osv.Solver(prob, osv.Options(defl_mode=1, defl_z=1, defl_eps=0.2, mg_min_elems=3, tol=1e-10))
    A = s.levels[0].A
    AZ = (A @ s.Zadp).toarray()
    E = s.Eadp.toarray()
    Q_AZ = s.Zadp @ np.linalg.solve(E, s.Zadp.T @ AZ)
    assert np.abs(Q_AZ - s.Zadp.toarray()).max() <= 1e-9
    PAZ = AZ - A @ Q_AZ
    assert np.abs(PAZ).max() <= 1e-9 * np.abs(AZ).max()
    f = hz.point_source_rhs(prob, (0.3, 0.65, 0.45))
    u, info = s.solve(f)
    assert info.converged and info.relres_true <= 1e-10
    ud = spla.spsolve(A.tocsc().astype(complex), f)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) <= 1e-7
