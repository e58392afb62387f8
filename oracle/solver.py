"""Deflated, multigrid-approximated CSLP preconditioner and FGMRES: CPU oracle.

Test infrastructure only.  Plain float64/complex128 numpy + scipy.sparse, each
step written as the paper states it (section 3) with the readings below.

  * CSLP (section 3, the shifted-Laplacian preconditioner): M_beta = K -
    (beta1 + i beta2) M_k, i.e. the shift multiplies the (k^2-weighted) mass
    matrix of the discretisation rather than the identity.
  * Its inverse is approximated by multigrid V-cycles with damped Jacobi
    smoothing (section 3; section 4.2 writes the two-grid form).  Coarse
    levels come from knot halving; the transfer is the exact knot-insertion
    prolongation P and restriction P^T; coarse operators are Galerkin
    P^T (.) P for K and M_k separately; the coarsest level is solved by dense LU.
    Option mg_coarse = 1 (the paper's "coarse-grid variant" of the CSLP read
    as a rediscretisation): the multigrid operators use M_k assembled on the
    coarse elements, with k^2 of a coarse element the mean of its children;
    the deflation matrices stay Galerkin.
  * Deflation (section 3, equation for P = I - AQ): Q = Z E^-1 Z^T with
    E = Z^T A Z and Z the same knot-insertion prolongation.  It is combined
    with the CSLP additively as a right preconditioner
        T(v) = Mtilde^-1 (v - A Q v) + Q v,
    which uses the same projection I - AQ and keeps the outer Krylov operator A
    itself.  Multilevel deflation solves E by a fixed number of inner FGMRES
    iterations preconditioned by the next level's T; the deepest deflation
    level is solved by dense LU.
  * Option defl_z = 1: the deflation vectors of the adapted deflation
    preconditioner (ADP, section 3): Z interpolates from the coarse unknowns
    by the quadratic rational Bezier curve (weights 1/2, 3/2, 1/2 at t = 1/2),
    optionally with the weight parameter eps on the coincident fine unknown;
    two-level only, E = Z^T A Z solved exactly.  See adp_deflation_1d.
  * Option precond = 1: the paper's comparison preconditioner C_ex (sections
    4.3 and 4.4): the CSLP with a small imaginary shift, M_ex = K - (1 + i
    beta2) M_k, inverted exactly (sparse LU), without multigrid or deflation;
    beta2 = 1/k in 1D and 1/(3k) in 2D unless given (cex_beta2).
  * Outer Krylov solver (sections 3 and 4.3): restarted flexible GMRES with
    modified Gram-Schmidt, complex Givens rotations, x0 = 0, stopping when the
    true relative residual ||f - A u|| / ||f|| is at most tol.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import bspline as bs
from .helmholtz import boundary_operator, fine_operators, weighted_mass_1d, weighted_mass_2d


class Options:
    """Solver parameters (defaults are the configuration the paper's method is run with)."""

    def __init__(self, beta=(1.0, 0.5), omega=0.8, nu_pre=1, nu_post=1, n_vcycles=1,
                 mg_min_elems=8, coarse_damping=1, defl_mode=2, defl_direct_max=16384,
                 defl_inner_its=(8, 4, 2, 1, 1, 1, 1, 1), restart=50, maxit=1000, tol=1e-7, mg_coarse=0,
                 defl_z=0, defl_eps=0.0, precond=0, cex_beta2=0.0, defl_kh_max=2.0):
        self.beta = complex(beta[0], beta[1])
        self.omega = float(omega)
        self.nu_pre = int(nu_pre)
        self.nu_post = int(nu_post)
        self.n_vcycles = int(n_vcycles)
        self.mg_min_elems = int(mg_min_elems)
        self.coarse_damping = int(coarse_damping)
        self.defl_mode = int(defl_mode)
        self.defl_direct_max = int(defl_direct_max)
        self.defl_inner_its = tuple(int(v) for v in defl_inner_its)
        self.restart = int(restart)
        self.maxit = int(maxit)
        self.tol = float(tol)
        self.mg_coarse = int(mg_coarse)
        self.defl_z = int(defl_z)
        self.defl_eps = float(defl_eps)
        self.precond = int(precond)
        self.cex_beta2 = float(cex_beta2)
        self.defl_kh_max = float(defl_kh_max)


class Level:
    pass


def build_hierarchy(prob, opts):
    """Levels 0..L: breakpoints per direction, Galerkin K_l, M_k,l, transfers P_l.

    Level l+1 is made from level l by knot halving in every direction; the
    coarsening stops once every direction has at most mg_min_elems elements.
    lev[l].P (l >= 1) maps level-l coefficients to level l-1 (interior rows and
    columns of the knot-insertion matrix; 2D: P_y (x) P_x; 3D: P_z (x) P_y (x) P_x).
    """
    p = prob.p
    bks = [prob.breakpoints(d) for d in range(prob.dim)]
    K, Mk = fine_operators(prob)
    levels = []
    lv = Level()
    lv.bks, lv.K, lv.Mk, lv.P = bks, K, Mk, None
    lv.B = boundary_operator(prob)
    levels.append(lv)
    while max(len(b) - 1 for b in levels[-1].bks) > opts.mg_min_elems:
        prev = levels[-1]
        cb = [bs.halve_breakpoints(b) for b in prev.bks]
        # interior rows and columns (radiation condition: the last function is kept)
        hi = None if prob.sommerfeld else -1
        Ps = [sp.csr_matrix(bs.knot_insertion_prolongation(fb, c, p)[1:hi, 1:hi])
              for fb, c in zip(prev.bks, cb)]
        P = Ps[0]
        for Pd in Ps[1:]:            # x fastest: P_z (x) P_y (x) P_x
            P = sp.kron(Pd, P)
        P = sp.csr_matrix(P)
        lv = Level()
        lv.bks = cb
        lv.P = P
        lv.K = (P.T @ prev.K @ P).tocsr()
        lv.Mk = (P.T @ prev.Mk @ P).tocsr()
        lv.B = None if prev.B is None else (P.T @ prev.B @ P).tocsr()
        levels.append(lv)
    k2 = prob.k2_elem
    for l, lv in enumerate(levels):
        lv.n = [len(b) - 1 + p - (1 if prob.sommerfeld else 2) for b in lv.bks]
        lv.N = int(np.prod(lv.n))
        # radiation condition: the unshifted boundary term -i k B in A and in M_beta
        rad = 0 if lv.B is None else -1j * prob.k * lv.B
        lv.A = (lv.K - lv.Mk + rad).tocsr()
        lv.Mk_mg = lv.Mk
        if opts.mg_coarse == 1 and k2 is not None and l > 0:
            k2 = coarse_mean(k2)
            lv.Mk_mg = rediscretised_mass(lv.bks, p, k2, prob.dim)
        lv.Mb = (lv.K - opts.beta * lv.Mk_mg + rad).tocsr()
        lv.D = lv.Mb.diagonal().copy()
        lv.gersh = gershgorin_bound(lv.Mb, lv.D)
        lv.omega = smoother_damping(l, lv.gersh, opts, prob.dim)
    # coarsest multigrid level: dense LU of M_beta
    levels[-1].Mb_lu = sla.lu_factor(levels[-1].Mb.toarray())
    return levels


def coarse_mean(k2):
    """k^2 of the next coarser level's elements: the mean over each one's children.

    Knot halving keeps the breakpoints of even index (and the last), so coarse
    element E covers fine elements 2E and 2E + 1 (only 2E at the end of an odd
    count).  k2: array [n_el_y][n_el_x] (1D: [n_el])."""
    k2 = np.atleast_2d(k2)
    ny, nx = k2.shape
    cy, cx = (ny + 1) // 2, (nx + 1) // 2
    out = np.zeros((cy, cx))
    for E2 in range(cy):
        for E1 in range(cx):
            out[E2, E1] = k2[2 * E2:2 * E2 + 2, 2 * E1:2 * E1 + 2].mean()
    return out


def rediscretised_mass(bks, p, k2, dim):
    """M_k assembled on the elements of breakpoints bks with weights k2 per element."""
    if dim == 1:
        return weighted_mass_1d(bks[0], p, np.ravel(k2))
    return weighted_mass_2d(bks[0], bks[1], p, k2)


def gershgorin_bound(Mb, D):
    """max_i sum_j |M_beta[i, j]| / |D_i|: a bound on the spectral radius of D^-1 M_beta."""
    rowsum = np.asarray(abs(Mb).sum(axis=1)).ravel()
    return float(np.max(rowsum / np.abs(D)))


def smoother_damping(l, gersh, opts, dim=2):
    """Jacobi damping at level l.

    The finest level uses omega as given.  On coarse levels the k^2-weighted
    B-spline mass dominates M_beta and D^-1 M_beta has eigenvalues beyond
    2/omega, so omega-Jacobi would amplify instead of smooth; with
    coarse_damping on, coarse levels use omega_l = min(omega, 2 / g_l), g_l the
    Gershgorin bound above (keeps |1 - omega_l lambda| bounded for every
    eigenvalue lambda of D^-1 M_beta in the disc the bound gives).  On the unit
    cube the three-fold tensor product of 1D masses already puts the finest
    level's D^-1 M_beta beyond 2/omega (the V-cycle then diverges for p >= 2 at
    k h below 1), so there the rule covers the finest level as well.
    """
    if (l == 0 and dim != 3) or opts.coarse_damping == 0:
        return opts.omega
    return min(opts.omega, 2.0 / gersh)


def deflation_levels(levels, opts, kmax=None):
    """Index L_z of the deflation level solved directly (0 when deflation is off).

    two-level: L_z = 1.  multilevel: the first level l >= 1 with at most
    defl_direct_max unknowns (never deeper than the coarsest multigrid level),
    and, with defl_kh_max > 0, not coarser than the last level l >= 1 whose
    largest k h_l (kmax the largest wave number, h_l the longest element of the
    level in either direction) is at most defl_kh_max: deflation levels too
    coarse to resolve the waves no longer hold A's near-null space.
    """
    L = len(levels) - 1
    if opts.defl_mode == 0 or L == 0:
        return 0
    if opts.defl_mode == 1:
        return 1
    lz = L
    for l in range(1, L + 1):
        if levels[l].N <= opts.defl_direct_max:
            lz = l
            break
    if opts.defl_kh_max > 0 and kmax is not None:
        lkh = 1
        for l in range(1, L + 1):
            h = max(float(np.max(np.diff(b))) for b in levels[l].bks)
            if kmax * h <= opts.defl_kh_max:
                lkh = l
        lz = min(lz, lkh)
    return lz


def adp_deflation_1d(nf, eps=0.0):
    """ADP deflation vectors along one direction (section 3), an nf x nc matrix.

    The paper's stencil is stated for 1-based unknowns: with nc = nf // 2 coarse
    unknowns, coarse unknown i sits at fine unknown 2i.  A fine unknown of even
    index j takes the quadratic rational Bezier curve through the coarse
    unknowns j/2 - 1, j/2, j/2 + 1 (Bernstein polynomials of degree 2, weights
    1/2, 3/2, 1/2, evaluated at t = 1/2), its centre weight lowered by eps / 8
    in the weighted variant; a fine unknown of odd index j is the mean of the
    coarse unknowns (j - 1)/2 and (j + 1)/2 (linear interpolation).  Coarse
    unknowns beyond either end are zero (homogeneous Dirichlet condition).
    """
    nc = nf // 2
    # the even-index weights from the curve itself
    t = 0.5
    w = np.array([0.5, 1.5, 0.5])
    b = np.array([(1 - t) ** 2, 2 * t * (1 - t), t ** 2])
    even = w * b / np.dot(w, b)
    even[1] -= eps / 8.0
    rows, cols, vals = [], [], []
    for j in range(1, nf + 1):
        if j % 2 == 0:
            taps = ((j // 2 - 1, even[0]), (j // 2, even[1]), (j // 2 + 1, even[2]))
        else:
            taps = (((j - 1) // 2, 0.5), ((j + 1) // 2, 0.5))
        for i, v in taps:
            if 1 <= i <= nc:
                rows.append(j - 1)
                cols.append(i - 1)
                vals.append(v)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def adp_deflation(prob_n, dim, eps=0.0):
    """ADP deflation matrix of the finest level: Z_x (1D), Z_y (x) Z_x (2D) or
    Z_z (x) Z_y (x) Z_x (3D), x fastest, prob_n the interior unknowns per direction."""
    Z = adp_deflation_1d(prob_n[0], eps)
    for d in range(1, dim):
        Z = sp.kron(adp_deflation_1d(prob_n[d], eps), Z)
    return sp.csr_matrix(Z)


# Deflation matrices up to this many unknowns are factored densely; larger ones
# (the 58k-unknown levels of the 480^2 and 960^2 workloads would need 27 GB
# dense) by a sparse LU.  Both are an exact factorisation of the same E, so E^-1 c
# agrees to rounding whichever is used.
DENSE_E_MAX = 4096


def exact_factor(E):
    """A function c -> E^-1 c for the real matrix E (complex c: real and imaginary
    parts solved separately, E being real): dense LU with partial pivoting for small E,
    SuperLU (scipy.sparse.linalg.splu) otherwise.  A complex E (radiation condition)
    is factored as it is."""
    if E.shape[0] <= DENSE_E_MAX:
        lu = sla.lu_factor(E.toarray())
        return lambda c: sla.lu_solve(lu, c)
    if np.iscomplexobj(E.data):
        lu = spla.splu(sp.csc_matrix(E))
        return lambda c: lu.solve(np.asarray(c, dtype=np.complex128))
    lu = spla.splu(sp.csc_matrix(E))
    return lambda c: lu.solve(np.ascontiguousarray(c.real)) + 1j * lu.solve(np.ascontiguousarray(c.imag))


class Solver:
    """The oracle's preconditioned solver for one problem.

    cnn_params (optional): learned finest-level smoother (see oracle.cnn); the
    finest-level Jacobi sweeps become x <- x + omega D^-1 r + ||r|| C(r/||r||, c).
    """

    def __init__(self, prob, opts=None, cnn_params=None):
        self.prob = prob
        self.opts = opts or Options()
        self.cnn_params = cnn_params
        self.levels = build_hierarchy(prob, self.opts)
        kmax = prob.k if prob.k_elem is None else float(np.max(prob.k_elem))
        self.Lz = deflation_levels(self.levels, self.opts, kmax)
        self.Zadp = None
        self.Mex_lu = None
        if prob.dim == 3 and (self.opts.precond != 0 or cnn_params is not None):
            raise ValueError("the unit cube is built with the multigrid CSLP (no C_ex, no learned smoother)")
        if self.opts.precond == 1:
            if prob.k_elem is not None:
                raise ValueError("C_ex is built for constant k only")
            b2 = self.opts.cex_beta2 or (1.0 / prob.k if prob.dim == 1 else 1.0 / (3.0 * prob.k))
            self.cex_beta2 = b2
            lv0 = self.levels[0]
            self.Mex = (lv0.K - (1.0 + 1j * b2) * lv0.Mk).tocsc()
            self.Mex_lu = spla.splu(self.Mex)
        if self.opts.defl_z == 1:
            if self.opts.defl_mode != 1:
                raise ValueError("ADP deflation vectors are two-level only (defl_mode = 1)")
            lv0 = self.levels[0]
            self.Zadp = adp_deflation(lv0.n, prob.dim, self.opts.defl_eps)
            self.Eadp = (self.Zadp.T @ lv0.A @ self.Zadp).tocsr()
            self.E_lu = exact_factor(self.Eadp)
        elif self.Lz > 0:
            self.E_lu = exact_factor(self.levels[self.Lz].A)

    # ---- multigrid on the CSLP --------------------------------------------
    def jacobi(self, l, b, x):
        """One damped Jacobi sweep x <- x + omega_l D^-1 (b - M_beta x) (learned on level 0)."""
        lv = self.levels[l]
        if l == 0 and self.cnn_params is not None:
            from . import cnn
            shape = (lv.n[1], lv.n[0]) if self.prob.dim == 2 else (1, lv.n[0])
            r = b - lv.Mb @ x
            return x + cnn.smoother_step(self.cnn_params, r, self.cnn_feature(), shape, lv.D, lv.omega)
        return x + lv.omega * (b - lv.Mb @ x) / lv.D

    def cnn_feature(self):
        """c = k^2 h^2 per finest-level unknown (element with the clamped index)."""
        from . import cnn
        lv = self.levels[0]
        p = self.prob
        if p.dim == 2:
            k2 = p.k2_elem if p.k_elem is not None else np.full((p.n_el[1], p.n_el[0]), p.k ** 2)
            return cnn.feature(k2, p.n_el[0], (lv.n[1], lv.n[0]), p.lengths[0])
        k2 = (p.k2_elem if p.k_elem is not None else np.full(p.n_el[0], p.k ** 2))[None, :]
        return cnn.feature(k2, p.n_el[0], (1, lv.n[0]), p.lengths[0])

    def vcycle_once(self, l, b):
        """One V(nu_pre, nu_post) cycle on M_beta,l from a zero initial guess."""
        lv = self.levels[l]
        if l == len(self.levels) - 1:
            return sla.lu_solve(lv.Mb_lu, b)
        x = np.zeros_like(b)
        for _ in range(self.opts.nu_pre):
            x = self.jacobi(l, b, x)
        r = b - lv.Mb @ x
        Pn = self.levels[l + 1].P
        x = x + Pn @ self.vcycle_once(l + 1, Pn.T @ r)
        for _ in range(self.opts.nu_post):
            x = self.jacobi(l, b, x)
        return x

    def vcycle(self, l, b):
        """n_vcycles V-cycles as the iteration x <- x + V(b - M_beta x), x0 = 0."""
        x = self.vcycle_once(l, b)
        for _ in range(self.opts.n_vcycles - 1):
            x = x + self.vcycle_once(l, b - self.levels[l].Mb @ x)
        return x

    # ---- deflation ---------------------------------------------------------
    def coarse_solve(self, l, c):
        """E^-1 c at deflation level l: dense LU at L_z, else inner FGMRES."""
        if l == self.Lz:
            return self.E_lu(c)
        m = self.opts.defl_inner_its[min(l - 1, len(self.opts.defl_inner_its) - 1)]
        x, _ = fgmres_fixed(lambda v: self.levels[l].A @ v, lambda v: self.T(l, v), c, m)
        return x

    def T(self, l, v):
        """Preconditioner at level l: Mtilde^-1 (v - A Q v) + Q v, Q = P E^-1 P^T."""
        if self.Mex_lu is not None:
            return self.Mex_lu.solve(np.asarray(v, dtype=np.complex128))
        if self.Zadp is not None:
            if l > 0:
                return self.vcycle(l, v)
            Z = self.Zadp
            q = Z @ self.E_lu(Z.T @ v)
            w = v - self.levels[0].A @ q
            return self.vcycle(0, w) + q
        if self.Lz == 0 or l >= self.Lz:
            return self.vcycle(l, v)
        Pn = self.levels[l + 1].P
        q = Pn @ self.coarse_solve(l + 1, Pn.T @ v)
        w = v - self.levels[l].A @ q
        return self.vcycle(l, w) + q

    def solve(self, f, u0=None, history=False):
        A0 = self.levels[0].A
        return fgmres(lambda v: A0 @ v, lambda v: self.T(0, v), f, self.opts.restart,
                      self.opts.tol, self.opts.maxit, u0=u0, history=history)


# ---- Krylov ----------------------------------------------------------------

def givens(a, b):
    """Complex rotation (c real, s complex) with [c s; -conj(s) c] (a, b) = (r, 0).

    b == 0: c = 1, s = 0.  a == 0: c = 0, s = conj(b)/|b|.  Otherwise
    t = sqrt(|a|^2 + |b|^2), c = |a|/t, s = (a/|a|) conj(b)/t.
    """
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    t = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    return abs(a) / t, (a / abs(a)) * np.conj(b) / t


def _arnoldi_cycle(Aop, Top, r0, m, stop_abs, record, trace=None):
    """One FGMRES cycle of at most m steps from residual r0; returns the update.

    Arnoldi with modified Gram-Schmidt (h_ij = v_i^H w), Givens QR of the
    Hessenberg matrix, upper-triangular solve, update sum_i z_i y_i.  The cycle
    stops early when |g_{j+1}| <= stop_abs or on breakdown (h_{j+1,j} == 0).
    trace (a dict, optional) receives the basis V, the preconditioned vectors Z
    and the Hessenberg matrix before rotation ("V", "Z", "H").
    """
    n = r0.shape[0]
    beta = np.linalg.norm(r0)
    if beta == 0.0:
        return np.zeros(n, dtype=np.complex128), 0, 0.0
    V = [r0 / beta]
    Z = []
    H = np.zeros((m + 1, m), dtype=np.complex128)
    cs = np.zeros(m)
    sn = np.zeros(m, dtype=np.complex128)
    g = np.zeros(m + 1, dtype=np.complex128)
    g[0] = beta
    j_done = 0
    for j in range(m):
        z = Top(V[j])
        Z.append(z)
        w = Aop(z)
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        hn = np.linalg.norm(w)
        H[j + 1, j] = hn
        if trace is not None:
            trace.setdefault("H", np.zeros((m + 1, m), dtype=np.complex128))[:j + 2, j] = H[:j + 2, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
        H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
        H[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        j_done = j + 1
        if record is not None:
            record.append(abs(g[j + 1]))
        if hn == 0.0 or abs(g[j + 1]) <= stop_abs:
            break
        V.append(w / hn)
    if trace is not None:
        trace["V"] = np.array(V + ([w / hn] if hn != 0.0 and len(V) == j_done else []))
        trace["Z"] = np.array(Z)
        trace["H"] = trace["H"][:j_done + 1, :j_done]
    y = np.zeros(j_done, dtype=np.complex128)
    for i in range(j_done - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:]) / H[i, i]
    dx = np.zeros(n, dtype=np.complex128)
    for i in range(j_done):
        dx = dx + Z[i] * y[i]
    return dx, j_done, abs(g[j_done])


def fgmres_fixed(Aop, Top, b, m, trace=None):
    """Exactly m FGMRES steps from x0 = 0 (fewer only on breakdown); no restart."""
    dx, its, _ = _arnoldi_cycle(Aop, Top, b.astype(np.complex128), m, -1.0, None, trace)
    return dx, its


class SolveInfo:
    def __init__(self):
        self.iters = 0
        self.restarts = 0
        self.relres_true = np.nan
        self.relres_est = np.nan
        self.converged = False
        self.history = []


def fgmres(Aop, Top, f, restart, tol, maxit, u0=None, history=False):
    """Restarted FGMRES(restart) on A u = f with right preconditioner T.

    Iterations count Arnoldi steps.  After each cycle the true residual
    f - A u is recomputed; the solve stops when ||f - A u|| <= tol ||f||, or
    after maxit steps (not converged).
    """
    f = np.asarray(f, dtype=np.complex128)
    info = SolveInfo()
    nf = np.linalg.norm(f)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.complex128)
    if nf == 0.0:
        info.relres_true = 0.0
        info.relres_est = 0.0
        info.converged = True
        return np.zeros_like(f), info
    r = f - Aop(u)
    rec = [] if history else None
    while True:
        if np.linalg.norm(r) <= tol * nf:
            info.converged = True
            break
        if info.iters >= maxit:
            break
        m = min(restart, maxit - info.iters)
        dx, its, gres = _arnoldi_cycle(Aop, Top, r, m, tol * nf, rec)
        u = u + dx
        info.iters += its
        info.relres_est = gres / nf
        r = f - Aop(u)
        if its == 0:
            break
        info.restarts += 1
    info.restarts = max(info.restarts - 1, 0)
    info.relres_true = np.linalg.norm(r) / nf
    info.converged = info.relres_true <= tol
    if history:
        info.history = rec
    return u, info
