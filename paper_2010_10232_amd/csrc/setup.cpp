// Host-side discretisation: knot vectors, B-spline values, Gauss-Legendre
// element matrices, knot-insertion transfers and Galerkin coarse stencils.
//
// Follows section 2.3 of the paper (open uniform knot vectors with the end
// knots repeated p+1 times, Cox-de Boor B-splines, Galerkin stiffness and mass
// entries) and section 3 (coarse spaces; the knot-insertion prolongation is the
// deflation matrix Z and the multigrid transfer).  Coarse levels halve the
// knot spans: they keep every second breakpoint plus the last one when the
// element count is odd, so the spaces are nested and only the last element of
// a level can be short.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "hh_internal.h"

namespace hh {

// Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on the
// three-term Legendre recurrence.
void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // final derivative at the converged node
        double p0 = 1.0, p1 = 0.0;
        for (int k = 1; k <= n; ++k) {
            double p2 = p1;
            p1 = p0;
            p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// The p+1 B-splines of degree p that are nonzero on knot span `span`
// (U[span] <= x < U[span+1]) and their first derivatives, by the triangular
// form of the Cox-de Boor recursion; N[r] belongs to global function span-p+r.
void basis_values(const std::vector<double>& U, int p, int span, double x, double* N, double* dN) {
    double ndu[7][7];
    double left[7], right[7];
    ndu[0][0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = x - U[span + 1 - j];
        right[j] = U[span + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            ndu[j][r] = right[r + 1] + left[j - r];
            double temp = ndu[r][j - 1] / ndu[j][r];
            ndu[r][j] = saved + right[r + 1] * temp;
            saved = left[j - r] * temp;
        }
        ndu[j][j] = saved;
    }
    for (int r = 0; r <= p; ++r) N[r] = ndu[r][p];
    if (!dN) return;
    if (p == 0) {
        dN[0] = 0.0;
        return;
    }
    // N'_{i,p} = p (N_{i,p-1} / (U_{i+p} - U_i) - N_{i+1,p-1} / (U_{i+p+1} - U_{i+1}))
    for (int r = 0; r <= p; ++r) {
        int i = span - p + r;
        double d = 0.0;
        if (r >= 1) d += ndu[r - 1][p - 1] / (U[i + p] - U[i]);
        if (r <= p - 1) d -= ndu[r][p - 1] / (U[i + p + 1] - U[i + 1]);
        dN[r] = p * d;
    }
}

static int level_elems(int nel_fine, int level) {
    int n = nel_fine;
    for (int l = 0; l < level; ++l) n = (n + 1) / 2;
    return n;
}

Axis make_trivial_axis() {
    Axis a;
    a.p = 0;
    a.nel = 1;
    a.n = 1;
    a.off = 0;
    a.nel_fine = 1;
    a.bk = {0.0, 1.0};
    a.U = a.bk;
    a.Kb = {0.0};
    a.Mb = {1.0};
    a.Me = {1.0};
    a.G = {1.0};
    a.pw = a.rw = 1;
    a.prow0 = {0};
    a.prow = {1.0};
    a.pcol0 = {0};
    a.pcol = {1.0};
    return a;
}

Axis make_axis(int p, int nel_fine, int level, bool keep_last, double len) {
    Axis a;
    a.p = p;
    a.level = level;
    a.nel_fine = nel_fine;
    a.nel = level_elems(nel_fine, level);
    a.n = a.nel + p - (keep_last ? 1 : 2);
    a.off = 1;
    // breakpoints: finest indices j * 2^level (j < nel) and the last one
    std::vector<int> idx;
    for (int j = 0; j < a.nel; ++j) idx.push_back(j << level);
    idx.push_back(nel_fine);
    for (int i : idx) a.bk.push_back(len * (i / (double)nel_fine));
    for (int i = 0; i < p; ++i) a.U.push_back(a.bk.front());
    for (double v : a.bk) a.U.push_back(v);
    for (int i = 0; i < p; ++i) a.U.push_back(a.bk.back());

    const int q = p + 1, bw = 2 * p + 1;
    double gx[8], gw[8], N[8], dN[8];
    gauss_legendre(q, gx, gw);
    // element matrices and the full banded K, M
    const int nfull = a.nel + p;
    std::vector<double> Kf((size_t)nfull * bw, 0.0), Mf((size_t)nfull * bw, 0.0);
    a.Me.assign((size_t)a.nel * q * q, 0.0);
    for (int e = 0; e < a.nel; ++e) {
        double lo = a.bk[e], hi = a.bk[e + 1], jac = 0.5 * (hi - lo);
        double ke[36] = {0}, me[36] = {0};
        for (int g = 0; g < q; ++g) {
            double x = lo + (gx[g] + 1.0) * jac;
            basis_values(a.U, p, e + p, x, N, dN);
            for (int i = 0; i < q; ++i)
                for (int j = 0; j < q; ++j) {
                    ke[i * q + j] += gw[g] * jac * dN[i] * dN[j];
                    me[i * q + j] += gw[g] * jac * N[i] * N[j];
                }
        }
        if (e == 0) {
            a.K0.assign(ke, ke + q);
            a.M0.assign(me, me + q);
        }
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) {
                Kf[(size_t)(e + i) * bw + (j - i + p)] += ke[i * q + j];
                Mf[(size_t)(e + i) * bw + (j - i + p)] += me[i * q + j];
                a.Me[(size_t)e * q * q + i * q + j] = me[i * q + j];
            }
    }
    // interior bands: drop the first and last function (homogeneous Dirichlet; with
    // keep_last only the first)
    a.Kb.assign((size_t)a.n * bw, 0.0);
    a.Mb.assign((size_t)a.n * bw, 0.0);
    for (int i = 0; i < a.n; ++i)
        for (int d = -p; d <= p; ++d) {
            int j = i + d;
            if (j < 0 || j >= a.n) continue;
            a.Kb[(size_t)i * bw + d + p] = Kf[(size_t)(i + 1) * bw + d + p];
            a.Mb[(size_t)i * bw + d + p] = Mf[(size_t)(i + 1) * bw + d + p];
        }
    // this level's basis on every finest element: blocks for the Galerkin
    // k^2-weighted mass (k^2 is constant on finest elements)
    a.G.assign((size_t)nel_fine * q * q, 0.0);
    for (int e = 0; e < nel_fine; ++e) {
        int E = e >> level;
        double lo = len * (e / (double)nel_fine), hi = len * ((e + 1) / (double)nel_fine), jac = 0.5 * (hi - lo);
        double* blk = &a.G[(size_t)e * q * q];
        for (int g = 0; g < q; ++g) {
            double x = lo + (gx[g] + 1.0) * jac;
            basis_values(a.U, p, E + p, x, N, nullptr);
            for (int i = 0; i < q; ++i)
                for (int j = 0; j < q; ++j) blk[i * q + j] += gw[g] * jac * N[i] * N[j];
        }
    }
    return a;
}

// A sparse row of the prolongation: coefficients of one fine-space B-spline
// coefficient in terms of the coarse coefficients (first column j0, values w).
struct PRow {
    int j0 = 0;
    std::vector<double> w;
};

static PRow row_combine(double a, const PRow& x, double b, const PRow& y) {
    PRow r;
    int lo = std::min(x.j0, y.j0);
    int hi = std::max(x.j0 + (int)x.w.size(), y.j0 + (int)y.w.size());
    r.j0 = lo;
    r.w.assign(hi - lo, 0.0);
    for (size_t t = 0; t < x.w.size(); ++t) r.w[x.j0 - lo + t] += a * x.w[t];
    for (size_t t = 0; t < y.w.size(); ++t) r.w[y.j0 - lo + t] += b * y.w[t];
    return r;
}

// Knot-insertion prolongation from `coarse` (level l+1) to `fine` (level l),
// restricted to interior functions, stored as row and column runs in `fine`.
// Boehm's algorithm: the knots of the fine vector missing from the coarse one
// are inserted one at a time; inserting t into span s (U_s <= t < U_{s+1})
// maps coefficients c to c'_i = c_i (i <= s-p), a_i c_i + (1 - a_i) c_{i-1}
// with a_i = (t - U_i)/(U_{i+p} - U_i) (s-p < i <= s), c_{i-1} (i > s).  Run on
// the identity it yields, row by row, the fine coefficients of every coarse
// B-spline (convex combinations only, so it is exact to rounding).
// Row and column tables of an interior transfer matrix P (nf x nc, entry
// Pint(i, J)) on the fine side's axis: per fine row a run of at most pw coarse
// entries, per coarse column a run of at most rw fine entries, each run
// shifted inward where it would pass the end.
template <class F>
static void transfer_tables(Axis& fine, int nf, int nc, int pw, int rw, F&& Pint) {
    fine.pw = std::min(pw, nc);
    fine.rw = std::min(rw, nf);
    fine.prow0.assign(nf, 0);
    fine.prow.assign((size_t)nf * fine.pw, 0.0);
    for (int i = 0; i < nf; ++i) {
        int first = -1, last = -1;
        for (int J = 0; J < nc; ++J)
            if (Pint(i, J) != 0.0) {
                if (first < 0) first = J;
                last = J;
            }
        if (first < 0) first = last = 0;
        HH_REQUIRE(last - first + 1 <= fine.pw, "transfer row wider than its table");
        int j0 = std::min(first, nc - fine.pw);
        fine.prow0[i] = j0;
        for (int t = 0; t < fine.pw; ++t) fine.prow[(size_t)i * fine.pw + t] = Pint(i, j0 + t);
    }
    fine.pcol0.assign(nc, 0);
    fine.pcol.assign((size_t)nc * fine.rw, 0.0);
    for (int J = 0; J < nc; ++J) {
        int first = -1, last = -1;
        for (int i = 0; i < nf; ++i)
            if (Pint(i, J) != 0.0) {
                if (first < 0) first = i;
                last = i;
            }
        if (first < 0) first = last = 0;
        HH_REQUIRE(last - first + 1 <= fine.rw, "transfer column wider than its table");
        int i0 = std::min(first, nf - fine.rw);
        fine.pcol0[J] = i0;
        for (int t = 0; t < fine.rw; ++t) fine.pcol[(size_t)J * fine.rw + t] = Pint(i0 + t, J);
    }
}

void make_transfer(Axis& fine, const Axis& coarse) {
    const int p = fine.p;
    std::vector<double> U = coarse.U;
    const int ncf = coarse.nel + p;
    std::vector<PRow> rows(ncf);
    for (int j = 0; j < ncf; ++j) {
        rows[j].j0 = j;
        rows[j].w = {1.0};
    }
    // knots to insert: fine breakpoints that are not coarse breakpoints
    std::vector<double> ins;
    {
        size_t c = 0;
        for (double b : fine.bk) {
            while (c < coarse.bk.size() && coarse.bk[c] < b) ++c;
            if (c < coarse.bk.size() && coarse.bk[c] == b) continue;
            ins.push_back(b);
        }
    }
    for (double t : ins) {
        int s = p;
        while (s + 1 < (int)U.size() && U[s + 1] <= t) ++s;
        const int n = (int)rows.size();
        std::vector<PRow> nr(n + 1);
        for (int i = 0; i <= n; ++i) {
            if (i <= s - p) {
                nr[i] = rows[i];
            } else if (i >= s + 1) {
                nr[i] = rows[i - 1];
            } else {
                const double a = (t - U[i]) / (U[i + p] - U[i]);
                nr[i] = row_combine(a, rows[i], 1.0 - a, rows[i - 1]);
            }
        }
        rows.swap(nr);
        U.insert(U.begin() + s + 1, t);
    }
    HH_REQUIRE((int)rows.size() == fine.nel + p, "knot insertion produced the wrong dimension");
    auto Pint = [&](int i, int J) -> double {  // interior entry (fine i, coarse J)
        const PRow& r = rows[i + 1];
        const int t = J + 1 - r.j0;
        if (t < 0 || t >= (int)r.w.size()) return 0.0;
        const double v = r.w[t];
        return std::fabs(v) < 1e-15 ? 0.0 : v;
    };
    // interior part (drop first/last function in both spaces)
    transfer_tables(fine, fine.n, coarse.n, p + 1, p + 2, Pint);
}

// Deflation vectors of the adapted deflation preconditioner (ADP, section 3)
// along one direction: nc = nf / 2 coarse unknowns, coarse c (0-based) at fine
// unknown 2c + 1.  That fine unknown takes the quadratic rational Bezier curve
// through coarse c - 1, c, c + 1 at t = 1/2 (Bernstein polynomials of degree
// 2 with weights 1/2, 3/2, 1/2: (1, 6, 1) / 8), its centre weight lowered by
// eps / 8 in the weighted form; fine unknown 2c is the mean of coarse c - 1
// and c.  Coarse unknowns past either end are zero (Dirichlet).
static double adp_entry(int nc, double eps, int i, int J) {
    if (J < 0 || J >= nc) return 0.0;
    if (i & 1) {
        const double b[3] = {0.25, 0.5, 0.25}, w[3] = {0.5, 1.5, 0.5};
        const double den = w[0] * b[0] + w[1] * b[1] + w[2] * b[2];
        const int d = J - (i - 1) / 2;
        if (d == 0) return w[1] * b[1] / den - eps / 8.0;
        if (d == -1) return w[0] * b[0] / den;
        if (d == 1) return w[2] * b[2] / den;
        return 0.0;
    }
    return (J == i / 2 - 1 || J == i / 2) ? 0.5 : 0.0;
}

void make_adp(const Axis& fine, double eps, Axis& zf, Axis& coarse) {
    const int nf = fine.n, nc = nf / 2, p = fine.p, bf = 2 * p + 1;
    HH_REQUIRE(nc >= 1, "too few unknowns for ADP deflation vectors");
    auto Z = [&](int i, int J) { return adp_entry(nc, eps, i, J); };
    transfer_tables(zf, nf, nc, 3, 5, Z);
    // coarse pseudo-axis: the Galerkin products Z^T K Z and Z^T M Z as bands
    // of half-width q (Z's columns span 5 fine unknowns, K and M 2p + 1)
    const int q = (p + 4) / 2, bq = 2 * q + 1;
    coarse = Axis{};
    coarse.p = q;
    coarse.n = nc;
    coarse.nel = std::max(1, fine.nel / 2);
    coarse.off = 0;
    coarse.nel_fine = fine.nel_fine;
    coarse.level = fine.level + 1;
    coarse.Kb.assign((size_t)nc * bq, 0.0);
    coarse.Mb.assign((size_t)nc * bq, 0.0);
    for (int a = 0; a < nc; ++a)
        for (int t = 0; t < zf.rw; ++t) {
            const int i = zf.pcol0[a] + t;
            const double za = Z(i, a);
            if (za == 0.0) continue;
            for (int d = -p; d <= p; ++d) {
                const int i2 = i + d;
                if (i2 < 0 || i2 >= nf) continue;
                const double kv = fine.Kb[(size_t)i * bf + d + p], mv = fine.Mb[(size_t)i * bf + d + p];
                for (int u = 0; u < zf.pw; ++u) {
                    const int b = zf.prow0[i2] + u;
                    const double zb = Z(i2, b);
                    if (zb == 0.0) continue;
                    HH_REQUIRE(std::abs(b - a) <= q, "ADP Galerkin band wider than expected");
                    coarse.Kb[(size_t)a * bq + b - a + q] += za * kv * zb;
                    coarse.Mb[(size_t)a * bq + b - a + q] += za * mv * zb;
                }
            }
        }
}

// Sc = Z^T S Z for the tensor-product deflation vectors Z = Z_y (x) Z_x, S a
// full stencil of the fine level (SoA [(2px+1)(2py+1)][N]) and Sc one of the
// coarse pseudo-axes (cx, cy), formed as Z^T (S Z) one fine row at a time.
void galerkin_stencil_z(const Axis& ax, const Axis& ay, const std::vector<double>& S, const Axis& zfx,
                        const Axis& zfy, const Axis& cxa, const Axis& cya, std::vector<double>& Sc) {
    const int n1 = ax.n, n2 = ay.n, px = ax.p, py = ay.p, bx = 2 * px + 1;
    const long long N = (long long)n1 * n2;
    const int m1 = cxa.n, m2 = cya.n, qx = cxa.p, qy = cya.p, cbx = 2 * qx + 1, cby = 2 * qy + 1;
    const long long Nc = (long long)m1 * m2;
    Sc.assign((size_t)cbx * cby * Nc, 0.0);
    // coarse columns touched from fine row j: those of Z's rows j - p .. j + p
    auto span = [](const Axis& zf, int n, int p, int j, int& lo, int& hi) {
        lo = zf.prow0[std::max(j - p, 0)];
        hi = zf.prow0[std::min(j + p, n - 1)] + zf.pw - 1;
    };
    std::vector<double> T;
    for (int j2 = 0; j2 < n2; ++j2) {
        int lo2, hi2;
        span(zfy, n2, py, j2, lo2, hi2);
        for (int j1 = 0; j1 < n1; ++j1) {
            int lo1, hi1;
            span(zfx, n1, px, j1, lo1, hi1);
            const int w1 = hi1 - lo1 + 1, w2 = hi2 - lo2 + 1;
            T.assign((size_t)w1 * w2, 0.0);
            const long long J = (long long)j2 * n1 + j1;
            // T[b] = sum over the stencil of fine row J of S[J, J'] Z[J', b]
            for (int d2 = -py; d2 <= py; ++d2) {
                const int k2 = j2 + d2;
                if (k2 < 0 || k2 >= n2) continue;
                for (int d1 = -px; d1 <= px; ++d1) {
                    const int k1 = j1 + d1;
                    if (k1 < 0 || k1 >= n1) continue;
                    const double sv = S[(size_t)((d2 + py) * bx + d1 + px) * N + J];
                    if (sv == 0.0) continue;
                    for (int u2 = 0; u2 < zfy.pw; ++u2) {
                        const double zy = zfy.prow[(size_t)k2 * zfy.pw + u2];
                        if (zy == 0.0) continue;
                        const int b2 = zfy.prow0[k2] + u2;
                        for (int u1 = 0; u1 < zfx.pw; ++u1) {
                            const double zx = zfx.prow[(size_t)k1 * zfx.pw + u1];
                            if (zx == 0.0) continue;
                            const int b1 = zfx.prow0[k1] + u1;
                            T[(size_t)(b2 - lo2) * w1 + (b1 - lo1)] += sv * zy * zx;
                        }
                    }
                }
            }
            // Sc[a, b] += Z[J, a] T[b] over the coarse a of Z's row J
            for (int u2 = 0; u2 < zfy.pw; ++u2) {
                const double zy = zfy.prow[(size_t)j2 * zfy.pw + u2];
                if (zy == 0.0) continue;
                const int a2 = zfy.prow0[j2] + u2;
                for (int u1 = 0; u1 < zfx.pw; ++u1) {
                    const double zx = zfx.prow[(size_t)j1 * zfx.pw + u1];
                    if (zx == 0.0) continue;
                    const int a1 = zfx.prow0[j1] + u1;
                    const long long A = (long long)a2 * m1 + a1;
                    for (int b2 = lo2; b2 <= hi2; ++b2)
                        for (int b1 = lo1; b1 <= hi1; ++b1) {
                            const double tv = T[(size_t)(b2 - lo2) * w1 + (b1 - lo1)];
                            if (tv == 0.0) continue;
                            const int e1 = b1 - a1, e2 = b2 - a2;
                            HH_REQUIRE(std::abs(e1) <= qx && std::abs(e2) <= qy, "ADP stencil wider than expected");
                            Sc[(size_t)((e2 + qy) * cbx + e1 + qx) * Nc + A] += zy * zx * tv;
                        }
                }
            }
        }
    }
}

// Galerkin k^2-weighted mass of the level of (ax, ay) as a full stencil.
// M_k = sum over finest elements e of k_e^2 (Gy_e2 (x) Gx_e1), where G are
// this level's basis mass blocks on finest elements; summed row by row of
// finest elements through the weighted 1D band B_e2 = sum_e1 k^2 Gx_e1.
void galerkin_mass_stencil(const Axis& ax, const Axis& ay, const std::vector<double>& k2,
                           std::vector<double>& S) {
    const int px = ax.p, py = ay.p, qx = px + 1, qy = py + 1;
    const int bx = 2 * px + 1, by = 2 * py + 1;
    const long long N = (long long)ax.n * ay.n;
    S.assign((size_t)bx * by * N, 0.0);
    std::vector<double> B((size_t)ax.n * bx);
    for (int e2 = 0; e2 < ay.nel_fine; ++e2) {
        std::fill(B.begin(), B.end(), 0.0);
        for (int e1 = 0; e1 < ax.nel_fine; ++e1) {
            const int E1 = e1 >> ax.level;
            const double w = k2[(size_t)e2 * ax.nel_fine + e1];
            const double* g = &ax.G[(size_t)e1 * qx * qx];
            for (int a1 = 0; a1 < qx; ++a1) {
                int I1 = E1 + a1 - ax.off;
                if (I1 < 0 || I1 >= ax.n) continue;
                for (int c1 = 0; c1 < qx; ++c1) {
                    int J1 = E1 + c1 - ax.off;
                    if (J1 < 0 || J1 >= ax.n) continue;
                    B[(size_t)I1 * bx + (c1 - a1 + px)] += w * g[a1 * qx + c1];
                }
            }
        }
        const int E2 = e2 >> ay.level;
        const double* gy = &ay.G[(size_t)e2 * qy * qy];
        for (int a2 = 0; a2 < qy; ++a2) {
            int I2 = E2 + a2 - ay.off;
            if (I2 < 0 || I2 >= ay.n) continue;
            for (int c2 = 0; c2 < qy; ++c2) {
                int J2 = E2 + c2 - ay.off;
                if (J2 < 0 || J2 >= ay.n) continue;
                const double gyv = gy[a2 * qy + c2];
                const int d2 = c2 - a2 + py;
                for (int I1 = 0; I1 < ax.n; ++I1)
                    for (int d1 = 0; d1 < bx; ++d1) {
                        double v = B[(size_t)I1 * bx + d1];
                        if (v != 0.0) S[(size_t)(d2 * bx + d1) * N + (long long)I2 * ax.n + I1] += gyv * v;
                    }
            }
        }
    }
}

// k^2 of every element of the next coarser level as the mean of its children:
// the one or two elements of this level inside it per direction (knot halving
// keeps the even breakpoints and the last one).  k2 [ny][nx] -> out [ncy][ncx].
void coarse_k2_mean(const std::vector<double>& k2, int nx, int ny, int ncx, int ncy, std::vector<double>& out) {
    out.assign((size_t)ncx * ncy, 0.0);
    for (int E2 = 0; E2 < ncy; ++E2)
        for (int E1 = 0; E1 < ncx; ++E1) {
            double s = 0.0;
            int c = 0;
            for (int c2 = 2 * E2; c2 < std::min(2 * E2 + 2, ny); ++c2)
                for (int c1 = 2 * E1; c1 < std::min(2 * E1 + 2, nx); ++c1) {
                    s += k2[(size_t)c2 * nx + c1];
                    ++c;
                }
            out[(size_t)E2 * ncx + E1] = s / c;
        }
}

// k^2-weighted mass of one level rediscretised on its own elements, weights
// k2l [nel_y][nel_x]: sum over elements E of k2l[E] (Me_y[E2] (x) Me_x[E1]), as a
// stencil in the layout of galerkin_mass_stencil.
void redisc_mass_stencil(const Axis& ax, const Axis& ay, const std::vector<double>& k2l, std::vector<double>& S) {
    const int px = ax.p, py = ay.p, qx = px + 1, qy = py + 1;
    const int bx = 2 * px + 1, by = 2 * py + 1;
    const long long N = (long long)ax.n * ay.n;
    S.assign((size_t)bx * by * N, 0.0);
    std::vector<double> B((size_t)ax.n * bx);
    for (int E2 = 0; E2 < ay.nel; ++E2) {
        std::fill(B.begin(), B.end(), 0.0);
        for (int E1 = 0; E1 < ax.nel; ++E1) {
            const double w = k2l[(size_t)E2 * ax.nel + E1];
            const double* m = &ax.Me[(size_t)E1 * qx * qx];
            for (int a1 = 0; a1 < qx; ++a1) {
                const int I1 = E1 + a1 - ax.off;
                if (I1 < 0 || I1 >= ax.n) continue;
                for (int c1 = 0; c1 < qx; ++c1) {
                    const int J1 = E1 + c1 - ax.off;
                    if (J1 < 0 || J1 >= ax.n) continue;
                    B[(size_t)I1 * bx + (c1 - a1 + px)] += w * m[a1 * qx + c1];
                }
            }
        }
        const double* my = &ay.Me[(size_t)E2 * qy * qy];
        for (int a2 = 0; a2 < qy; ++a2) {
            const int I2 = E2 + a2 - ay.off;
            if (I2 < 0 || I2 >= ay.n) continue;
            for (int c2 = 0; c2 < qy; ++c2) {
                const int J2 = E2 + c2 - ay.off;
                if (J2 < 0 || J2 >= ay.n) continue;
                const double g = my[a2 * qy + c2];
                const int d2 = c2 - a2 + py;
                for (int I1 = 0; I1 < ax.n; ++I1)
                    for (int d1 = 0; d1 < bx; ++d1) {
                        const double v = B[(size_t)I1 * bx + d1];
                        if (v != 0.0) S[(size_t)(d2 * bx + d1) * N + (long long)I2 * ax.n + I1] += g * v;
                    }
            }
        }
    }
}

// Generalised eigenpairs of one axis's symmetric-definite pencil (K, M):
// K V = M V diag(lam) with V^T M V = I.  M = L L^T (Cholesky), C = L^-1 K L^-T,
// C = Q diag(lam) Q^T by the cyclic Jacobi method (plane rotations that zero
// one off-diagonal pair each, row-by-row sweeps until the off-diagonal mass is
// negligible), V = L^-T Q.  V is row-major [i][a] (unknown i, mode a).
void axis_eigen(const Axis& a, std::vector<double>& V, std::vector<double>& lam) {
    const int n = a.n, p = a.p, bw = 2 * p + 1;
    std::vector<double> K((size_t)n * n, 0.0), L((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int d = -p; d <= p; ++d) {
            const int j = i + d;
            if (j < 0 || j >= n) continue;
            K[(size_t)i * n + j] = a.Kb[(size_t)i * bw + d + p];
            L[(size_t)i * n + j] = a.Mb[(size_t)i * bw + d + p];
        }
    // Cholesky in place (lower triangle of L)
    for (int j = 0; j < n; ++j) {
        double d = L[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0.0)) throw Err{HH_ENUMERIC, "mass matrix is not positive definite"};
        const double ljj = std::sqrt(d);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double v = L[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) v -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = v / ljj;
        }
        for (int i = 0; i < j; ++i) L[(size_t)i * n + j] = 0.0;
    }
    // X = L^-1 K (forward substitution per column), C = X L^-T = (L^-1 X^T)^T
    auto lower_solve_cols = [&](std::vector<double>& B) {
        for (int c = 0; c < n; ++c)
            for (int i = 0; i < n; ++i) {
                double v = B[(size_t)i * n + c];
                for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * B[(size_t)k * n + c];
                B[(size_t)i * n + c] = v / L[(size_t)i * n + i];
            }
    };
    std::vector<double> C = K;
    lower_solve_cols(C);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) std::swap(C[(size_t)i * n + j], C[(size_t)j * n + i]);
    lower_solve_cols(C);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double m = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
            C[(size_t)i * n + j] = C[(size_t)j * n + i] = m;
        }
    // QT = Q^T (row a holds eigenvector a) so that rotations touch contiguous rows;
    // C is kept symmetric: rows pp, q are updated and mirrored into the columns
    std::vector<double> QT((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) QT[(size_t)i * n + i] = 1.0;
    double total = 0.0;
    for (double v : C) total += v * v;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                if (i != j) off += C[(size_t)i * n + j] * C[(size_t)i * n + j];
        if (off <= 1e-32 * total) break;
        for (int pp = 0; pp < n - 1; ++pp)
            for (int q = pp + 1; q < n; ++q) {
                double* Cp = &C[(size_t)pp * n];
                double* Cq = &C[(size_t)q * n];
                const double apq = Cp[q];
                if (apq == 0.0) continue;
                const double app = Cp[pp], aqq = Cq[q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {
                    if (k == pp || k == q) continue;
                    const double g = Cp[k], h = Cq[k];
                    Cp[k] = c * g - sn * h;
                    Cq[k] = sn * g + c * h;
                    C[(size_t)k * n + pp] = Cp[k];
                    C[(size_t)k * n + q] = Cq[k];
                }
                Cp[pp] = app - t * apq;
                Cq[q] = aqq + t * apq;
                Cp[q] = Cq[pp] = 0.0;
                double* Qp = &QT[(size_t)pp * n];
                double* Qq = &QT[(size_t)q * n];
                for (int k = 0; k < n; ++k) {
                    const double g = Qp[k], h = Qq[k];
                    Qp[k] = c * g - sn * h;
                    Qq[k] = sn * g + c * h;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = C[(size_t)i * n + i];
    // V = L^-T Q (back substitution per column)
    V.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < n; ++a) V[(size_t)i * n + a] = QT[(size_t)a * n + i];
    for (int c = 0; c < n; ++c)
        for (int i = n - 1; i >= 0; --i) {
            double v = V[(size_t)i * n + c];
            for (int k = i + 1; k < n; ++k) v -= L[(size_t)k * n + i] * V[(size_t)k * n + c];
            V[(size_t)i * n + c] = v / L[(size_t)i * n + i];
        }
}

}  // namespace hh
