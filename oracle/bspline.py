"""Univariate B-spline machinery of the CPU oracle (test infrastructure only).

Follows the paper's section 2.3.1 ("B-spline basis functions"): open knot
vectors whose end knots are repeated p+1 times, the Cox-de Boor recursion
started from piecewise constants on half-open knot spans, and the Galerkin
stiffness / mass entries of section 2.3 (integrals of products of basis
derivatives and of basis functions).  Everything is plain float64 numpy.

Readings of silent points (recorded with the rest in the design notes):
  * span rule: a point x belongs to the non-empty span [xi_s, xi_{s+1}) with
    xi_s <= x < xi_{s+1}; the right end x == 1 belongs to the last non-empty
    span.  On a uniform level-0 mesh this is s = min(floor(x * n_el), n_el-1).
  * 0/0 := 0 inside the recursion (repeated knots).
  * element integrals use (p+1)-point Gauss-Legendre, which is exact for the
    degree-2p mass and degree-(2p-2) stiffness integrands.
  * coarse levels: keep every breakpoint with an even index plus the last one
    when the element count is odd (knot halving, nested spaces).
"""
import numpy as np


def uniform_breakpoints(n_el):
    """Breakpoints 0, 1/n_el, ..., 1 (breakpoint i is i / n_el in float64)."""
    return np.array([i / n_el for i in range(n_el + 1)], dtype=np.float64)


def halve_breakpoints(b):
    """Knot halving: keep even-indexed breakpoints, plus the last if the count is odd."""
    n_el = len(b) - 1
    keep = list(range(0, n_el + 1, 2))
    if keep[-1] != n_el:
        keep.append(n_el)
    return b[keep].copy()


def open_knot_vector(b, p):
    """Full knot vector: the end breakpoints repeated p+1 times (section 2.3.1)."""
    return np.concatenate([np.full(p, b[0]), b, np.full(p, b[-1])])


def n_basis(b, p):
    """Number of basis functions n = n_el + p."""
    return len(b) - 1 + p


def find_span(b, x):
    """Element (non-empty span) index of x, with x == b[-1] going to the last element."""
    n_el = len(b) - 1
    if x < b[0] or x > b[-1]:
        raise ValueError("point outside the parameter domain")
    # largest e with b[e] <= x, restricted to elements 0..n_el-1
    e = int(np.searchsorted(b, x, side="right")) - 1
    return min(max(e, 0), n_el - 1)


def uniform_span(x, n_el):
    """Span rule on a uniform mesh, evaluated in float64: min(floor(x*n_el), n_el-1)."""
    return min(int(np.floor(x * n_el)), n_el - 1)


def _ratio(num, den):
    return 0.0 if den == 0.0 else num / den


def basis_all(b, p, x, elem=None):
    """Values of all n_el+p degree-p basis functions at x (Cox-de Boor recursion).

    Degree 0: indicator of the span that holds x (the span rule above picks it);
    degree q: phi_{j,q} = (x - xi_j)/(xi_{j+q} - xi_j) phi_{j,q-1}
                         + (xi_{j+q+1} - x)/(xi_{j+q+1} - xi_{j+1}) phi_{j+1,q-1}.
    `elem` forces the span (used to evaluate at quadrature points of an element).
    """
    xi = open_knot_vector(b, p)
    if elem is None:
        elem = find_span(b, x)
    m = len(xi) - 1                       # number of degree-0 functions
    phi = np.zeros(m)
    phi[elem + p] = 1.0                   # span [xi_{e+p}, xi_{e+p+1}) is element e
    for q in range(1, p + 1):
        new = np.zeros(m - q)
        for j in range(m - q):
            new[j] = (_ratio(x - xi[j], xi[j + q] - xi[j]) * phi[j]
                      + _ratio(xi[j + q + 1] - x, xi[j + q + 1] - xi[j + 1]) * phi[j + 1])
        phi = new
    return phi


def basis_and_derivative_all(b, p, x, elem=None):
    """Values and first derivatives of all degree-p basis functions at x.

    Derivative of the recursion: phi'_{j,p} = p [phi_{j,p-1}/(xi_{j+p}-xi_j)
                                             - phi_{j+1,p-1}/(xi_{j+p+1}-xi_{j+1})].
    """
    xi = open_knot_vector(b, p)
    if elem is None:
        elem = find_span(b, x)
    val = basis_all(b, p, x, elem)
    if p == 0:
        return val, np.zeros_like(val)
    # degree p-1 functions on the same knot vector (indices 0..n+p-1 of that degree)
    m = len(xi) - 1
    phi = np.zeros(m)
    phi[elem + p] = 1.0
    for q in range(1, p):
        new = np.zeros(m - q)
        for j in range(m - q):
            new[j] = (_ratio(x - xi[j], xi[j + q] - xi[j]) * phi[j]
                      + _ratio(xi[j + q + 1] - x, xi[j + q + 1] - xi[j + 1]) * phi[j + 1])
        phi = new
    n = len(val)
    der = np.zeros(n)
    for j in range(n):
        der[j] = p * (_ratio(phi[j], xi[j + p] - xi[j])
                      - _ratio(phi[j + 1], xi[j + p + 1] - xi[j + 1]))
    return val, der


def gauss_legendre(npts):
    """Gauss-Legendre points and weights on [-1, 1] (numpy's routine)."""
    return np.polynomial.legendre.leggauss(npts)


def element_matrices(b, p):
    """Per-element local stiffness and mass blocks, (n_el, p+1, p+1) each.

    Local index a of element e is global basis function e+a; entries are the
    element integrals of phi'_i phi'_j and phi_i phi_j (section 2.3).
    """
    n_el = len(b) - 1
    gx, gw = gauss_legendre(p + 1)
    Ke = np.zeros((n_el, p + 1, p + 1))
    Me = np.zeros((n_el, p + 1, p + 1))
    for e in range(n_el):
        lo, hi = b[e], b[e + 1]
        jac = 0.5 * (hi - lo)
        for xq, wq in zip(gx, gw):
            x = lo + (xq + 1.0) * jac
            val, der = basis_and_derivative_all(b, p, x, elem=e)
            v = val[e:e + p + 1]
            d = der[e:e + p + 1]
            Ke[e] += wq * jac * np.outer(d, d)
            Me[e] += wq * jac * np.outer(v, v)
    return Ke, Me


def assemble_full(b, p, elem_weight=None):
    """Full (all n_el+p functions) stiffness K and mass M as dense arrays.

    `elem_weight` (length n_el) multiplies the element mass blocks, giving the
    element-weighted mass used for a piecewise-constant coefficient.
    """
    n_el = len(b) - 1
    n = n_el + p
    Ke, Me = element_matrices(b, p)
    K = np.zeros((n, n))
    M = np.zeros((n, n))
    for e in range(n_el):
        w = 1.0 if elem_weight is None else elem_weight[e]
        K[e:e + p + 1, e:e + p + 1] += Ke[e]
        M[e:e + p + 1, e:e + p + 1] += w * Me[e]
    return K, M


def interior(Afull):
    """Strong homogeneous Dirichlet elimination: drop the first and last basis function."""
    return Afull[1:-1, 1:-1]


def greville(b, p):
    """Greville abscissae (averages of p consecutive interior knots)."""
    xi = open_knot_vector(b, p)
    n = n_basis(b, p)
    if p == 0:
        return 0.5 * (xi[:-1] + xi[1:])
    return np.array([xi[j + 1:j + p + 1].mean() for j in range(n)])


def basis_matrix(b, p, pts):
    """Collocation matrix B[i, j] = phi_j(pts[i])."""
    return np.array([basis_all(b, p, x) for x in pts])


def knot_insertion_prolongation(b_fine, b_coarse, p):
    """Full prolongation P (n_f x n_c): phi^c_J = sum_i P[i, J] phi^f_i.

    The coarse space is nested in the fine one, so P is found exactly by
    collocation at the fine Greville points: B_f P = B_c.
    """
    g = greville(b_fine, p)
    Bf = basis_matrix(b_fine, p, g)
    Bc = basis_matrix(b_coarse, p, g)
    P = np.linalg.solve(Bf, Bc)
    P[np.abs(P) < 1e-14] = 0.0
    return P
