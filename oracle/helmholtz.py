"""Discrete Helmholtz operators of the CPU oracle (test infrastructure only).

Section 2.3 of the paper: Galerkin discretisation of -Lap u - k^2 u = f with
tensor-product B-splines on the unit interval / square and homogeneous
Dirichlet conditions (MP 1-B, MP 2-A, MP 2-B of section 2).  The system matrix
is A = K - M_k, with K the stiffness matrix and M_k the k^2-weighted mass
matrix.  The paper prints the variational form with the opposite sign of the
k^2 term; the model problems and the eigenvalues j^2 pi^2 - k^2 it gives for
MP 1-B (section 3) fix the sign used here.

MP 1-A (section 2.1, option sommerfeld=True, 1D, constant k): u(0) = u0 and the
radiation condition u' - i k u = 0 at x = 1.  The first basis function is
eliminated (its coefficient is u0, moved to the right-hand side), the last one
is kept, and the boundary term of the weak form adds -i k phi_i(1) phi_j(1):
A = K - k^2 M - i k B with B = e_n e_n^T (only the last function is nonzero at
x = 1).

A non-constant wave number is constant on each element of the finest mesh
(its value at the element centroid); M_k = sum_e k_e^2 (m_e^y (x) m_e^x).
Vectors are ordered with x fastest: index i2 * n1 + i1 over interior
control points.  All matrices are scipy.sparse in float64.

Domain extents (option lengths): the geometry map F of section 2.3 taken as the
axis-aligned scaling F(xi) = (L_1 xi_1, ..., L_d xi_d) of the parametric unit
square; the basis is built on the physical breakpoints L_d i / n_el, so K and
M carry the Jacobian (1D: K scales by 1/L, M by L), k is a physical wave
number and source points are physical.  Default: the unit interval / square / cube.

The unit cube (dim = 3, constant k, Dirichlet everywhere): the tensor-product
extension of section 2.3 to three directions, the setting where section 4.3
expects the cost advantage it measures in 2D to grow (section 3 names 2D and
3D as the sizes that rule out direct solvers); Phi = phi_i(x) phi_j(y) phi_l(z), so
K = Mz (x) My (x) Kx + Mz (x) Ky (x) Mx + Kz (x) My (x) Mx and
M = Mz (x) My (x) Mx, index (i3 * n2 + i2) * n1 + i1.
"""
import numpy as np
import scipy.sparse as sp

from . import bspline as bs


class Problem:
    """One Helmholtz problem: dimension, degree p, elements per side, wave number.

    k_elem (optional) holds k (not k^2) per finest element, x fastest, shape
    (n_el_y, n_el_x) in 2D or (n_el,) in 1D; otherwise the constant k is used.
    lengths (optional): the domain's extent per direction (default 1 each).
    """

    def __init__(self, dim, p, n_el, k, k_elem=None, sommerfeld=False, lengths=None):
        if dim not in (1, 2, 3):
            raise ValueError("dim must be 1, 2 or 3")
        if sommerfeld and (dim != 1 or k_elem is not None):
            raise ValueError("the radiation condition (MP 1-A) is built for 1D, constant k")
        if dim == 3 and k_elem is not None:
            raise ValueError("the unit cube is built for constant k")
        self.sommerfeld = bool(sommerfeld)
        self.dim = dim
        self.p = int(p)
        self.n_el = [int(n_el)] * dim if np.isscalar(n_el) else [int(v) for v in n_el]
        self.k = float(k)
        if k_elem is not None:
            k_elem = np.asarray(k_elem, dtype=np.float64)
            shape = tuple(self.n_el[::-1]) if dim == 2 else (self.n_el[0],)
            k_elem = k_elem.reshape(shape)
        self.k_elem = k_elem
        self.lengths = [1.0] * dim if lengths is None else [float(v) for v in lengths]
        if len(self.lengths) != dim or not all(np.isfinite(v) and v > 0 for v in self.lengths):
            raise ValueError("lengths: one positive extent per direction")

    def breakpoints(self, d):
        """Physical breakpoints of direction d: L_d i / n_el."""
        return self.lengths[d] * bs.uniform_breakpoints(self.n_el[d])

    def span(self, d, x):
        """Element of direction d holding the physical coordinate x (span rule on x / L_d)."""
        return bs.uniform_span(x / self.lengths[d], self.n_el[d])

    @property
    def k2_elem(self):
        """k^2 per finest element (array), or None for a constant wave number."""
        return None if self.k_elem is None else self.k_elem ** 2


def matrices_1d(b, p, keep_last=False):
    """Interior (Dirichlet-eliminated) 1D stiffness and mass as sparse matrices;
    keep_last: only the first function is eliminated (radiation condition at x = 1)."""
    K, M = bs.assemble_full(b, p)
    if keep_last:
        return sp.csr_matrix(K[1:, 1:]), sp.csr_matrix(M[1:, 1:])
    return sp.csr_matrix(bs.interior(K)), sp.csr_matrix(bs.interior(M))


def boundary_operator(prob):
    """B of the radiation condition (MP 1-A): 1 on the last unknown, else None."""
    if not prob.sommerfeld:
        return None
    n = prob.n_el[0] + prob.p - 1
    return sp.csr_matrix(([1.0], ([n - 1], [n - 1])), shape=(n, n))


def dirichlet_lift_rhs(prob, u0=1.0):
    """MP 1-A: f = -u0 (K - k^2 M)[:, 0] on the unknowns (the eliminated first function
    carries the boundary value u0; the equation itself has no source)."""
    b = prob.breakpoints(0)
    K, M = bs.assemble_full(b, prob.p)
    col = K[1:, 0] - prob.k ** 2 * M[1:, 0]
    return (-u0 * col).astype(np.complex128)


def l2_error_1d(prob, u, exact, u0=1.0, nq=None):
    """Continuous L2 norm of (u_h - exact) on [0, L], u_h = u0 phi_0 + sum_i u_i phi_i."""
    p = prob.p
    nq = nq or (p + 4)
    b = prob.breakpoints(0)
    U = np.zeros(prob.n_el[0] + p, dtype=np.complex128)
    U[0] = u0
    U[1:1 + len(u)] = u
    gx, gw = bs.gauss_legendre(nq)
    err2 = 0.0
    for e in range(prob.n_el[0]):
        lo, hi = b[e], b[e + 1]
        jac = 0.5 * (hi - lo)
        for x, w in zip(lo + (gx + 1) * jac, gw * jac):
            uh = bs.basis_all(b, p, x, elem=e) @ U
            err2 += w * abs(uh - exact(x)) ** 2
    return float(np.sqrt(err2))


def weighted_mass_1d(b, p, w_elem):
    """Interior 1D mass with element weights w_e (sum_e w_e m_e)."""
    _, M = bs.assemble_full(b, p, elem_weight=w_elem)
    return sp.csr_matrix(bs.interior(M))


def weighted_mass_2d(bx, by, p, w_elem):
    """Interior 2D mass sum_e w_e (m^y_{e2} (x) m^x_{e1}); w_elem shape (n_el_y, n_el_x).

    Each element adds its (p+1)^2 x (p+1)^2 local block at the global indices
    (e2 + a2 - 1, e1 + a1 - 1) of its local functions (a2, a1); functions 0 and
    n-1 of either direction are eliminated (Dirichlet).
    """
    _, Mex = bs.element_matrices(bx, p)
    _, Mey = bs.element_matrices(by, p)
    nelx, nely = len(bx) - 1, len(by) - 1
    n1, n2 = nelx + p - 2, nely + p - 2
    q = p + 1
    rows, cols, vals = [], [], []
    e1 = np.arange(nelx)
    for e2 in range(nely):
        for a2 in range(q):
            i2 = e2 + a2 - 1
            if i2 < 0 or i2 >= n2:
                continue
            for c2 in range(q):
                j2 = e2 + c2 - 1
                if j2 < 0 or j2 >= n2:
                    continue
                for a1 in range(q):
                    i1 = e1 + a1 - 1
                    for c1 in range(q):
                        j1 = e1 + c1 - 1
                        ok = (i1 >= 0) & (i1 < n1) & (j1 >= 0) & (j1 < n1)
                        v = w_elem[e2, ok] * Mey[e2, a2, c2] * Mex[ok, a1, c1]
                        rows.append(i2 * n1 + i1[ok])
                        cols.append(j2 * n1 + j1[ok])
                        vals.append(v)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n1 * n2, n1 * n2))


def fine_operators(prob):
    """Level-0 stiffness K and k^2-weighted mass M_k (sparse, interior)."""
    p = prob.p
    if prob.dim == 1:
        b = prob.breakpoints(0)
        K, M = matrices_1d(b, p, keep_last=prob.sommerfeld)
        if prob.k_elem is None:
            Mk = prob.k ** 2 * M
        else:
            Mk = weighted_mass_1d(b, p, prob.k2_elem)
        return K.tocsr(), Mk.tocsr()
    if prob.dim == 3:
        (Kx, Mx), (Ky, My), (Kz, Mz) = [matrices_1d(prob.breakpoints(d), p) for d in range(3)]
        K = sp.kron(Mz, sp.kron(My, Kx)) + sp.kron(Mz, sp.kron(Ky, Mx)) + sp.kron(Kz, sp.kron(My, Mx))
        Mk = prob.k ** 2 * sp.kron(Mz, sp.kron(My, Mx))
        return K.tocsr(), Mk.tocsr()
    bx = prob.breakpoints(0)
    by = prob.breakpoints(1)
    Kx, Mx = matrices_1d(bx, p)
    Ky, My = matrices_1d(by, p)
    K = sp.kron(My, Kx) + sp.kron(Ky, Mx)
    if prob.k_elem is None:
        Mk = prob.k ** 2 * sp.kron(My, Mx)
    else:
        Mk = weighted_mass_2d(bx, by, p, prob.k2_elem)
    return K.tocsr(), Mk.tocsr()


def point_source_rhs(prob, x0, amp=1.0):
    """f_i = amp * Phi_i(x0): the Galerkin load of a point source delta(x - x0).

    MP 1-B and MP 2-A/2-B (section 2) use a unit point source; tested against a
    basis function it gives the function's value at the source point.
    """
    p = prob.p
    if prob.dim == 1:
        b = prob.breakpoints(0)
        e = prob.span(0, x0[0])
        return amp * bs.basis_all(b, p, x0[0], elem=e)[1:-1].astype(np.complex128)
    if prob.dim == 3:
        f = [bs.basis_all(prob.breakpoints(d), p, x0[d], elem=prob.span(d, x0[d]))[1:-1] for d in range(3)]
        return amp * np.kron(f[2], np.kron(f[1], f[0])).astype(np.complex128)
    bx = prob.breakpoints(0)
    by = prob.breakpoints(1)
    ex = prob.span(0, x0[0])
    ey = prob.span(1, x0[1])
    fx = bs.basis_all(bx, p, x0[0], elem=ex)[1:-1]
    fy = bs.basis_all(by, p, x0[1], elem=ey)[1:-1]
    return amp * np.kron(fy, fx).astype(np.complex128)


def source_spans(prob, x0):
    """Element indices (per direction) that hold the source point (span rule)."""
    return [prob.span(d, x0[d]) for d in range(prob.dim)]


def manufactured_rhs_2d(prob, a, bfreq, nq=None):
    """Load vector of f = ((a^2 + b^2) pi^2 - k^2) sin(a pi x) sin(b pi y), constant k.

    Its exact solution is u = sin(a pi x) sin(b pi y) (homogeneous Dirichlet).
    Integrated element by element with nq-point Gauss-Legendre per direction.
    """
    p = prob.p
    nq = nq or (p + 4)
    bx = bs.uniform_breakpoints(prob.n_el[0])
    by = bs.uniform_breakpoints(prob.n_el[1])
    n1 = prob.n_el[0] + p - 2
    n2 = prob.n_el[1] + p - 2
    gx, gw = bs.gauss_legendre(nq)
    lam = (a * a + bfreq * bfreq) * np.pi ** 2 - prob.k ** 2
    # 1D load integrals of sin(a pi x) times each basis function factorise.
    def load_1d(b, freq, n_el):
        out = np.zeros(n_el + p)
        for e in range(n_el):
            lo, hi = b[e], b[e + 1]
            jac = 0.5 * (hi - lo)
            for xq, wq in zip(gx, gw):
                x = lo + (xq + 1) * jac
                v = bs.basis_all(b, p, x, elem=e)
                out += wq * jac * np.sin(freq * np.pi * x) * v
        return out[1:-1]
    fx = load_1d(bx, a, prob.n_el[0])
    fy = load_1d(by, bfreq, prob.n_el[1])
    assert len(fx) == n1 and len(fy) == n2
    return lam * np.kron(fy, fx)


def l2_error_2d(prob, u, exact, nq=None):
    """Continuous L2 norm of (u_h - exact) over the unit square by Gauss quadrature."""
    p = prob.p
    nq = nq or (p + 4)
    bx = bs.uniform_breakpoints(prob.n_el[0])
    by = bs.uniform_breakpoints(prob.n_el[1])
    n1 = prob.n_el[0] + p - 2
    U = np.zeros((prob.n_el[1] + p, prob.n_el[0] + p), dtype=u.dtype)
    U[1:-1, 1:-1] = u.reshape(prob.n_el[1] + p - 2, n1)
    gx, gw = bs.gauss_legendre(nq)
    err2 = 0.0
    # tabulate 1D basis values at the quadrature points of every element
    def tab(b, n_el):
        out = []
        for e in range(n_el):
            lo, hi = b[e], b[e + 1]
            jac = 0.5 * (hi - lo)
            xs = lo + (gx + 1) * jac
            out.append((xs, gw * jac, np.array([bs.basis_all(b, p, x, elem=e) for x in xs])))
        return out
    tx = tab(bx, prob.n_el[0])
    ty = tab(by, prob.n_el[1])
    for ys, wy, By in ty:
        for xs, wx, Bx in tx:
            uh = By @ U @ Bx.T                     # (nq_y, nq_x)
            ex = exact(xs[None, :], ys[:, None])
            err2 += np.sum(wy[:, None] * wx[None, :] * np.abs(uh - ex) ** 2)
    return np.sqrt(err2)


def sine_load_1d(b, p, freq, nq=None):
    """Interior load integrals of sin(freq pi x) against each basis function (Gauss-Legendre)."""
    nq = nq or (p + 4)
    n_el = len(b) - 1
    gx, gw = bs.gauss_legendre(nq)
    out = np.zeros(n_el + p)
    for e in range(n_el):
        lo, hi = b[e], b[e + 1]
        jac = 0.5 * (hi - lo)
        for xq, wq in zip(gx, gw):
            x = lo + (xq + 1) * jac
            out += wq * jac * np.sin(freq * np.pi * x) * bs.basis_all(b, p, x, elem=e)
    return out[1:-1]


def manufactured_rhs_3d(prob, freqs):
    """Load vector of f = ((a^2 + b^2 + c^2) pi^2 - k^2) sin(a pi x) sin(b pi y) sin(c pi z)
    (exact solution the product of the three sines, zero on the boundary of the cube)."""
    lam = sum(f * f for f in freqs) * np.pi ** 2 - prob.k ** 2
    loads = [sine_load_1d(bs.uniform_breakpoints(n), prob.p, f) for n, f in zip(prob.n_el, freqs)]
    return lam * np.kron(loads[2], np.kron(loads[1], loads[0]))


def l2_error_3d(prob, u, freqs, nq=None):
    """Continuous L2 norm of u_h minus the product of sines over the unit cube (tensor Gauss)."""
    p = prob.p
    nq = nq or (p + 4)
    gx, gw = bs.gauss_legendre(nq)
    n = [m + p - 2 for m in prob.n_el]
    U = np.zeros((n[2] + 2, n[1] + 2, n[0] + 2), dtype=np.complex128)
    U[1:-1, 1:-1, 1:-1] = np.asarray(u).reshape(n[2], n[1], n[0])
    tabs = []
    for d, m in enumerate(prob.n_el):
        b = bs.uniform_breakpoints(m)
        pts, wts, B = [], [], []
        for e in range(m):
            lo, hi = b[e], b[e + 1]
            jac = 0.5 * (hi - lo)
            for xq, wq in zip(gx, gw):
                x = lo + (xq + 1) * jac
                pts.append(x)
                wts.append(wq * jac)
                B.append(bs.basis_all(b, p, x, elem=e))
        tabs.append((np.array(pts), np.array(wts), np.array(B)))
    (xs, wx, Bx), (ys, wy, By), (zs, wz, Bz) = tabs
    uh = np.einsum("ci,bj,ak,ijk->abc", Bz, By, Bx, U)     # (z, y, x) at the quadrature points
    ex = (np.sin(freqs[2] * np.pi * zs)[:, None, None] * np.sin(freqs[1] * np.pi * ys)[None, :, None]
          * np.sin(freqs[0] * np.pi * xs)[None, None, :])
    w = wz[:, None, None] * wy[None, :, None] * wx[None, None, :]
    return float(np.sqrt(np.sum(w * np.abs(uh - ex) ** 2)))
