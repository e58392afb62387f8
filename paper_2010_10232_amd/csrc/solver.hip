// Solver driver: hierarchy setup, V-cycle, deflation recursion and FGMRES.
//
// Section 3 of the paper: the CSLP M_beta = K - (beta1 + i beta2) M_k is
// approximated by multigrid V-cycles with damped Jacobi smoothing; deflation
// uses Q = Z E^-1 Z^T with E = Z^T A Z and Z the knot-insertion prolongation.
// The two are combined as the right preconditioner
//     T_l(v) = Mtilde_l^-1 (v - A_l Q v) + Q v,    Q v = P_{l+1} E^-1 P_{l+1}^T v,
// inside restarted flexible GMRES on A itself (section 4.3: relative residual
// 1e-7).  E^-1 at the deepest deflation level L_z is an explicit dense inverse;
// between, E_l^-1 is a fixed number of inner FGMRES steps preconditioned by
// T_l (multilevel deflation).  Every step of a preconditioner application is a
// kernel on the caller's stream; the host only reads the convergence estimate
// of each outer Arnoldi step.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>

#include "solver.h"

namespace hh {

using zd = std::complex<double>;

// ---------------------------------------------------------------- problem --
ProblemImpl* build_problem(const hh_problem_desc* d) {
    HH_REQUIRE(d != nullptr, "null problem descriptor");
    HH_REQUIRE(d->dim >= 1 && d->dim <= 3, "dim must be 1, 2 or 3");
    HH_REQUIRE(d->p >= 1 && d->p <= 5, "p must be in 1..5");
    const int nx = d->n_el[0], ny = d->dim >= 2 ? d->n_el[1] : 1, nz = d->dim == 3 ? d->n_el_z : 1;
    HH_REQUIRE(nx >= 2 && (d->dim == 1 || ny >= 2) && (d->dim < 3 || nz >= 2), "at least 2 elements per direction");
    HH_REQUIRE(nx <= (1 << 20) && ny <= (1 << 20) && nz <= (1 << 20), "too many elements");
    HH_REQUIRE(d->dim < 3 || d->k_mode == 0, "3D problems are built for constant k");
    HH_REQUIRE(d->dim < 3 || (long long)(nx + d->p) * (ny + d->p) * (nz + d->p) < (1LL << 31),
               "3D problem too large (at most 2^31 unknowns)");
    HH_REQUIRE(d->k_mode == 0 || d->k_mode == 1, "k_mode must be 0 or 1");
    HH_REQUIRE(d->bc_right == 0 || d->bc_right == 1, "bc_right must be 0 (Dirichlet) or 1 (radiation condition)");
    HH_REQUIRE(d->bc_right == 0 || (d->dim == 1 && d->k_mode == 0),
               "the radiation condition (bc_right = 1) is built for 1D problems with constant k");
    auto* P = new ProblemImpl();
    P->somm = d->bc_right == 1;
    P->dim = d->dim;
    P->p = d->p;
    P->nel[0] = nx;
    P->nel[1] = ny;
    P->nel[2] = nz;
    for (int dd = 0; dd < 3; ++dd) {
        const double L = d->length[dd];
        if (!(std::isfinite(L) && L >= 0.0)) {
            delete P;
            throw Err{HH_EINVAL, "length must be finite and >= 0 (0: the unit extent)"};
        }
        P->len[dd] = (dd < d->dim && L > 0.0) ? L : 1.0;
    }
    P->k_mode = d->k_mode;
    P->k = d->k;
    if (d->k_mode == 0) {
        if (!(d->k > 0.0) || !std::isfinite(d->k)) {
            delete P;
            throw Err{HH_EINVAL, "k must be positive and finite"};
        }
    } else {
        if (!d->k_elem) {
            delete P;
            throw Err{HH_EINVAL, "k_elem is NULL with k_mode 1"};
        }
        P->k2.resize((size_t)nx * ny);
        for (size_t i = 0; i < P->k2.size(); ++i) {
            const double kv = d->k_elem[i];
            if (!(kv > 0.0) || !std::isfinite(kv)) {
                delete P;
                throw Err{HH_EINVAL, "k_elem values must be positive and finite"};
            }
            P->k2[i] = kv * kv;
        }
    }
    P->ax0 = make_axis(P->p, nx, 0, P->somm, P->len[0]);
    P->ay0 = d->dim >= 2 ? make_axis(P->p, ny, 0, false, P->len[1]) : make_trivial_axis();
    P->az0 = d->dim == 3 ? make_axis(P->p, nz, 0, false, P->len[2]) : make_trivial_axis();
    return P;
}

// ------------------------------------------------------------- host math --
// In-place inverse of a small dense complex matrix (Gauss-Jordan, partial pivoting).
static void invert_complex(int n, std::vector<zd>& A) {
    std::vector<int> piv(n);
    std::vector<zd> inv((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int pr = c;
        for (int r = c + 1; r < n; ++r)
            if (std::abs(A[(size_t)r * n + c]) > std::abs(A[(size_t)pr * n + c])) pr = r;
        if (std::abs(A[(size_t)pr * n + c]) == 0.0) throw Err{HH_ENUMERIC, "singular coarsest matrix"};
        if (pr != c)
            for (int j = 0; j < n; ++j) {
                std::swap(A[(size_t)c * n + j], A[(size_t)pr * n + j]);
                std::swap(inv[(size_t)c * n + j], inv[(size_t)pr * n + j]);
            }
        const zd d = 1.0 / A[(size_t)c * n + c];
        for (int j = 0; j < n; ++j) {
            A[(size_t)c * n + j] *= d;
            inv[(size_t)c * n + j] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const zd f = A[(size_t)r * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
                inv[(size_t)r * n + j] -= f * inv[(size_t)c * n + j];
            }
        }
    }
    A.swap(inv);
}

// --------------------------------------------------------------- helpers --
static void fill_krylov(KrylovDev& k, DevBuf& blob, int m) {
    const size_t nH = (size_t)(m + 1) * m, nb = 2048;
    const size_t nslots = 2 * 256 * 4;
    // one-reduction Arnoldi state: packed Gram rows and the vector-exchange words
    const int qcap = m <= kOneRedMaxM ? 2 * m - 1 : 0;
    const size_t ngram = qcap ? (size_t)m * (m - 1) / 2 + 1 : 0;
    const size_t nvslots = (size_t)kOneRedMaxBlocks * qcap * 4;
    size_t bytes = 16 * nH + 8 * m + 16 * m + 16 * (m + 1) + 16 * m + 8 * 8 + 16 * nb + 4 * 8 + 8 * nslots +
                   16 * ngram + 8 * nvslots;
    blob.alloc(bytes + 256);
    char* p = blob.as<char>();
    k.m = m;
    k.spin_limit = kSpinLimit;
    k.H = (cx<double>*)p;
    p += 16 * nH;
    k.sn = (cx<double>*)p;
    p += 16 * m;
    k.g = (cx<double>*)p;
    p += 16 * (m + 1);
    k.y = (cx<double>*)p;
    p += 16 * m;
    k.partials = (cx<double>*)p;
    p += 16 * nb;
    k.cs = (double*)p;
    p += 8 * m;
    k.scal = (double*)p;
    p += 8 * 8;
    k.ints = (int*)p;   // directly after scal: both reach the host in one transfer
    p += 4 * 8;
    k.slots = (unsigned long long*)p;   // zero words never carry a valid tag
    p += 8 * nslots;
    p = (char*)(((uintptr_t)p + 15) & ~(uintptr_t)15);
    k.gram = qcap ? (cx<double>*)p : nullptr;
    p += 16 * ngram;
    k.vslots = qcap ? (unsigned long long*)p : nullptr;
    k.qcap = qcap;
    k.hstep = nullptr;
    HH_HIP(hipMemset(blob.p, 0, blob.bytes));
}

template <class T>
static DevBuf& pick(DevBuf& a64, DevBuf& a32) {
    return sizeof(T) == 8 ? a64 : a32;
}

SolverImpl::~SolverImpl() {
    for (hipGraphExec_t g : gexec)
        if (g) (void)hipGraphExecDestroy(g);
    for (hipEvent_t e : {gfork, gjoin})
        if (e) (void)hipEventDestroy(e);
    if (gstream) (void)hipStreamDestroy(gstream);
    for (hipEvent_t e : evpool) (void)hipEventDestroy(e);
    if (pin_d) (void)hipHostFree(pin_d);
    if (pin_i) (void)hipHostFree(pin_i);
    if (pin_step) (void)hipHostFree(pin_step);
    for (hipEvent_t e : {ev_slot[0], ev_slot[1], ev_misc})
        if (e) (void)hipEventDestroy(e);
}

// Kernel-class timing: a pair of events around each launch of the selected
// class, recorded on the launch stream and read only once the solve has
// drained the stream, so the timed region is not serialised by the probes.
constexpr int kEvPairs = 4096;

void SolverImpl::tstart(int cls, hipStream_t s) {
    if (o.time_kernels != cls || ev_used >= kEvPairs) return;
    if (evpool.empty()) {
        evpool.resize(2 * kEvPairs);
        // timing-only events: no system-scope fence (cache write-back and
        // invalidation) around the timed kernels; read after the solve's sync
        for (auto& e : evpool) HH_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    HH_HIP(hipEventRecord(evpool[2 * ev_used], s));
    ev_pending = ev_used;
}

void SolverImpl::tstop(int cls, double bytes, hipStream_t s) {
    if (o.time_kernels != cls || ev_pending < 0) return;
    HH_HIP(hipEventRecord(evpool[2 * ev_pending + 1], s));
    ev_bytes += bytes;
    ev_used = ev_pending + 1;
    ev_pending = -1;
}

double SolverImpl::tcollect(int* count) {
    double ms = 0.0;
    for (int i = 0; i < ev_used; ++i) {
        float t = 0.f;
        HH_HIP(hipEventElapsedTime(&t, evpool[2 * i], evpool[2 * i + 1]));
        ms += t;
    }
    *count = ev_used;
    return ms;
}

// ----------------------------------------------------------------- setup --
void SolverImpl::setup(hipStream_t s) {
    const ProblemImpl& P = *prob;
    HH_REQUIRE(o.restart >= 1 && o.restart <= kMaxRestart, "restart must be in 1..200");
    HH_REQUIRE(o.maxit >= 1, "maxit must be >= 1");
    HH_REQUIRE(o.nu_pre >= 1 && o.nu_post >= 0 && o.n_vcycles >= 1, "bad smoothing counts");
    HH_REQUIRE(o.ortho == 0 || o.ortho == 1, "ortho is 0 or 1");
    HH_REQUIRE(o.defl_direct_solver >= 0 && o.defl_direct_solver <= 2, "defl_direct_solver is 0, 1 or 2");
    HH_REQUIRE(o.mg_coarse == 0 || o.mg_coarse == 1, "mg_coarse is 0 (Galerkin) or 1 (rediscretised, averaged k^2)");
    HH_REQUIRE(o.defl_z == 0 || o.defl_z == 1, "defl_z is 0 (knot insertion) or 1 (ADP)");
    HH_REQUIRE(o.defl_z == 0 || o.defl_mode == 1, "ADP deflation vectors (defl_z = 1) are two-level only (defl_mode = 1)");
    HH_REQUIRE(std::isfinite(o.defl_eps), "defl_eps must be finite");
    HH_REQUIRE(o.precond == 0 || o.precond == 1, "precond is 0 (deflated multigrid CSLP) or 1 (C_ex)");
    HH_REQUIRE(o.defl_refine >= -1 && o.defl_refine <= kSubMaxRefine, "defl_refine must be in -1..3");
    HH_REQUIRE(std::isfinite(o.defl_kh_max) && o.defl_kh_max >= 0.0, "defl_kh_max must be finite and >= 0");
    HH_REQUIRE(o.use_graph == 0 || o.use_graph == 1, "use_graph is 0 or 1");
    HH_REQUIRE(o.precond == 0 || P.k_mode == 0, "C_ex (precond = 1) is built for constant k only");
    HH_REQUIRE(std::isfinite(o.cex_beta2) && o.cex_beta2 >= 0.0, "cex_beta2 must be finite and >= 0");
    HH_REQUIRE(!P.somm || (o.precond == 0 && o.defl_z == 0),
               "the radiation condition is built with the knot-insertion deflation and the multigrid CSLP");
    HH_REQUIRE(o.mg_min_elems >= 2, "mg_min_elems must be >= 2");
    HH_REQUIRE(o.defl_mode >= 0 && o.defl_mode <= 2, "defl_mode must be 0, 1 or 2");
    HH_REQUIRE(o.precision == 0 || o.precision == 1, "precision must be 0 or 1");
    HH_REQUIRE(o.tol >= 0.0 && o.omega > 0.0, "bad tol or omega");
    HH_REQUIRE(o.defl_direct_max >= 1 && o.defl_direct_max <= 65536, "defl_direct_max must be in 1..65536");
    for (int i = 0; i < 8; ++i) HH_REQUIRE(o.defl_inner_its[i] >= 1 && o.defl_inner_its[i] <= 64, "defl_inner_its in 1..64");

    if (P.dim == 3) {
        setup_levels_3d(s);
        setup_finish(s);
        return;
    }
    const int p = P.p;
    const bool is2d = P.dim == 2;
    // multigrid levels by knot halving
    for (int l = 0;; ++l) {
        auto lv = std::make_unique<LevelDev>();
        lv->ax = l == 0 ? P.ax0 : make_axis(p, P.nel[0], l, P.somm, P.len[0]);
        lv->ay = is2d ? (l == 0 ? P.ay0 : make_axis(p, P.nel[1], l, false, P.len[1])) : make_trivial_axis();
        const int mx = std::max(lv->ax.nel, is2d ? lv->ay.nel : 0);
        HH_REQUIRE(lv->ax.n >= 1 && lv->ay.n >= 1, "level without interior unknowns");
        lev.push_back(std::move(lv));
        if (mx <= o.mg_min_elems) break;
    }
    L = (int)lev.size() - 1;
    for (int l = 0; l < L; ++l) {
        make_transfer(lev[l]->ax, lev[l + 1]->ax);
        if (is2d) make_transfer(lev[l]->ay, lev[l + 1]->ay);
    }
    const bool const_k = P.k_mode == 0;
    const double k2c = const_k ? P.k * P.k : 0.0;
    const zd beta(o.beta[0], o.beta[1]);
    // Sh: the mass stencil of each coarse level's multigrid operator; Shg: the
    // Galerkin one of its deflation operator A_l where they differ (mg_coarse =
    // REDISC_AVG rediscretises the multigrid operators with averaged k^2)
    std::vector<std::vector<double>> Sh(lev.size()), Shg(lev.size());
    const bool redisc = !const_k && o.mg_coarse == 1;
    std::vector<double> k2l = P.k2;
    int knx = P.nel[0], kny = P.dim == 2 ? P.nel[1] : 1;

    for (int l = 0; l <= L; ++l) {
        LevelDev& lv = *lev[l];
        lv.n1 = lv.ax.n;
        lv.n2 = lv.ay.n;
        lv.N = (long long)lv.n1 * lv.n2;
        lv.kind = const_k ? KIND_SEP : (l == 0 ? KIND_VARFINE : KIND_STENCIL);
        upload(lv.Kx, lv.ax.Kb);
        upload(lv.Mx, lv.ax.Mb);
        upload(lv.Ky, lv.ay.Kb);
        upload(lv.My, lv.ay.Mb);
        if (!const_k) galerkin_mass_stencil(lv.ax, lv.ay, P.k2, Sh[l]);
        if (redisc && l > 0) {
            std::vector<double> k2c;
            coarse_k2_mean(k2l, knx, kny, lv.ax.nel, lv.ay.nel, k2c);
            k2l.swap(k2c);
            knx = lv.ax.nel;
            kny = lv.ay.nel;
            Shg[l] = std::move(Sh[l]);
            redisc_mass_stencil(lv.ax, lv.ay, k2l, Sh[l]);
        }
        // radiation condition (MP 1-A): -i k on the last unknown of every level (the
        // Galerkin image of e_n e_n^T, the last function being interpolatory at x = 1)
        if (P.somm) {
            lv.bnd_I = lv.N - 1;
            lv.bnd_im = -P.k;
        }
        // Jacobi diagonal of M_beta and the Gershgorin bound of D^-1 M_beta
        std::vector<cx<double>> dinv((size_t)lv.N);
        std::vector<cx<float>> dinv32((size_t)lv.N);
        double g = 0.0;
        for (long long I = 0; I < lv.N; ++I) {
            zd diag = 0.0;
            double rowsum = 0.0;
            visit_row(lv.ax, lv.ay, const_k, k2c, Sh[l], I, [&](long long J, double kv, double mv) {
                zd e = kv - beta * mv;
                if (J == I && I == lv.bnd_I) e += zd(0.0, lv.bnd_im);
                rowsum += std::abs(e);
                if (J == I) diag = e;
            });
            HH_REQUIRE(std::abs(diag) > 0.0, "zero Jacobi diagonal");
            g = std::max(g, rowsum / std::abs(diag));
            const zd di = 1.0 / diag;
            dinv[I] = {di.real(), di.imag()};
            dinv32[I] = {(float)di.real(), (float)di.imag()};
        }
        lv.gersh = g;
        lv.omega = (l == 0 || o.coarse_damping == 0) ? o.omega : std::min(o.omega, 2.0 / g);
        upload(lv.Dinv64, dinv);
        upload(lv.Dinv32, dinv32);
        if (!const_k && l == 0) {
            if (!P.k2_dev.p) {
                P.k2_dev.alloc(P.k2.size() * sizeof(double));
                HH_HIP(hipMemcpyAsync(P.k2_dev.p, P.k2.data(), P.k2.size() * sizeof(double), hipMemcpyHostToDevice,
                                      s));
                HH_HIP(hipStreamSynchronize(s));
            }
            upload(lv.Mex, lv.ax.Me);
            upload(lv.Mey, lv.ay.Me);
        }
        if (!const_k && l > 0) {
            upload(lv.S64, Sh[l]);
            std::vector<float> s32(Sh[l].begin(), Sh[l].end());
            upload(lv.S32, s32);
            if (!Shg[l].empty()) upload(lv.S64a, Shg[l]);
        }
        const size_t v64 = (size_t)lv.N * 16, v32 = (size_t)lv.N * 8;
        lv.b64.alloc(v64);
        lv.x64.alloc(v64);
        lv.r64.alloc(v64);
        lv.t64.alloc(v64);
        lv.b32.alloc(v32);
        lv.x32.alloc(v32);
        lv.r32.alloc(v32);
        lv.t32.alloc(v32);
        if (o.n_vcycles > 1) {
            lv.vr64.alloc(v64);
            lv.vx64.alloc(v64);
            lv.vr32.alloc(v32);
            lv.vx32.alloc(v32);
        }
    }
    for (int l = 0; l < L; ++l) {
        LevelDev& lv = *lev[l];
        const LevelDev& lc = *lev[l + 1];
        upload(lv.prow0x, lv.ax.prow0);
        upload(lv.prowx, lv.ax.prow);
        upload(lv.pcol0x, lv.ax.pcol0);
        upload(lv.pcolx, lv.ax.pcol);
        upload(lv.prow0y, lv.ay.prow0);
        upload(lv.prowy, lv.ay.prow);
        upload(lv.pcol0y, lv.ay.pcol0);
        upload(lv.pcoly, lv.ay.pcol);
        Transfer& t = lv.tr;
        t.nf1 = lv.n1;
        t.nf2 = lv.n2;
        t.nc1 = lc.n1;
        t.nc2 = lc.n2;
        t.pw1 = lv.ax.pw;
        t.pw2 = lv.ay.pw;
        t.rw1 = lv.ax.rw;
        t.rw2 = lv.ay.rw;
        t.prow0x = lv.prow0x.as<int>();
        t.prowx = lv.prowx.as<double>();
        t.prow0y = lv.prow0y.as<int>();
        t.prowy = lv.prowy.as<double>();
        t.pcol0x = lv.pcol0x.as<int>();
        t.pcolx = lv.pcolx.as<double>();
        t.pcol0y = lv.pcol0y.as<int>();
        t.pcoly = lv.pcoly.as<double>();
    }
    // coarsest multigrid level: dense inverse of M_beta
    {
        LevelDev& lc = *lev[L];
        nL = (int)lc.N;
        HH_REQUIRE(nL <= 4096, "coarsest multigrid level too large");
        std::vector<zd> A((size_t)nL * nL, 0.0);
        for (long long I = 0; I < lc.N; ++I)
            visit_row(lc.ax, lc.ay, const_k, k2c, Sh[L], I,
                      [&](long long J, double kv, double mv) { A[(size_t)I * nL + J] += kv - beta * mv; });
        if (lc.bnd_I >= 0) A[(size_t)lc.bnd_I * nL + lc.bnd_I] += zd(0.0, lc.bnd_im);
        invert_complex(nL, A);
        std::vector<cx<double>> m64((size_t)nL * nL);
        std::vector<cx<float>> m32((size_t)nL * nL);
        for (size_t i = 0; i < A.size(); ++i) {
            m64[i] = {A[i].real(), A[i].imag()};
            m32[i] = {(float)A[i].real(), (float)A[i].imag()};
        }
        upload(Minv64, m64);
        upload(Minv32, m32);
    }
    // coarse tail: the levels from the first one with at most 1024 unknowns
    // whose right-hand sides, iterates, spare vectors (FP64) and coefficient
    // tables all fit in the LDS of one workgroup, down to the coarsest, run as
    // one single-workgroup V-cycle
    {
        int dev = 0, lds_max = 0;
        HH_HIP(hipGetDevice(&dev));
        HH_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const long long budget = std::min<long long>(lds_max, 160 * 1024) - 1024;
        tail_start = 1 << 30;
        tail_lds = 0;
        // LDS of one level in the tail: its three vectors and (above the coarsest
        // level) its bands and transfer tables, each region 16-byte aligned
        auto al16 = [](long long b) { return (b + 15) & ~15LL; };
        auto coef_bytes = [&](int m) -> long long {
            if (m >= L) return 0;
            const LevelDev& v = *lev[m];
            const int bx = 2 * p + 1, by = is2d ? 2 * p + 1 : 1;
            const Transfer& t = v.tr;
            return 2 * al16(8LL * v.n1 * bx) + 2 * al16(8LL * v.n2 * by) + al16(4LL * t.nf1) +
                   al16(8LL * t.nf1 * t.pw1) + al16(4LL * t.nf2) + al16(8LL * t.nf2 * t.pw2) + al16(4LL * t.nc1) +
                   al16(8LL * t.nc1 * t.rw1) + al16(4LL * t.nc2) + al16(8LL * t.nc2 * t.rw2);
        };
        // (the tail has no boundary term: problems with the radiation condition run
        // every level as separate kernels)
        for (int l = 1; l < L && L < kTailLevels && !P.somm; ++l) {
            long long bytes = 0;
            for (int m = l; m <= L; ++m) bytes += 3 * lev[m]->N * (long long)sizeof(cx<double>) + coef_bytes(m);
            // measured on MP 2-A: a level of 1681 unknowns runs faster as separate
            // kernels than inside the one-workgroup tail; from ~1000 down the tail wins
            if (bytes <= budget && lev[l]->N <= 1024) {
                tail_start = l;
                tail_lds = (int)bytes;
                break;
            }
        }
        if (tail_start < L) {
            auto fill = [&](auto& d, auto tag) {
                using T = decltype(tag);
                d.L = L;
                d.nL = nL;
                d.nu_pre = o.nu_pre;
                d.nu_post = o.nu_post;
                d.are = (T)o.beta[0];
                d.aim = (T)o.beta[1];
                d.k2c = k2c;
                d.Minv = pick<T>(Minv64, Minv32).template as<cx<T>>();
                d.lds_l0 = tail_start;
                // coefficient tables of all tail levels first (one contiguous
                // image, the same for both precisions), then the level vectors
                int off = 0;
                for (int l = tail_start; l <= L; ++l) {
                    auto& t = d.lv[l];
                    t.o_kx = t.o_mx = t.o_ky = t.o_my = -1;
                    t.o_prow0x = t.o_prowx = t.o_prow0y = t.o_prowy = -1;
                    t.o_pcol0x = t.o_pcolx = t.o_pcol0y = t.o_pcoly = -1;
                    if (l < L) {
                        const LevelDev& v = *lev[l];
                        const int bx = 2 * p + 1, by = is2d ? 2 * p + 1 : 1;
                        const Transfer& tr = v.tr;
                        auto take = [&](long long bytes) {
                            const int o = off;
                            off += (int)al16(bytes);
                            return o;
                        };
                        t.o_kx = take(8LL * v.n1 * bx);
                        t.o_mx = take(8LL * v.n1 * bx);
                        t.o_ky = take(8LL * v.n2 * by);
                        t.o_my = take(8LL * v.n2 * by);
                        t.o_prow0x = take(4LL * tr.nf1);
                        t.o_prowx = take(8LL * tr.nf1 * tr.pw1);
                        t.o_prow0y = take(4LL * tr.nf2);
                        t.o_prowy = take(8LL * tr.nf2 * tr.pw2);
                        t.o_pcol0x = take(4LL * tr.nc1);
                        t.o_pcolx = take(8LL * tr.nc1 * tr.rw1);
                        t.o_pcol0y = take(4LL * tr.nc2);
                        t.o_pcoly = take(8LL * tr.nc2 * tr.rw2);
                    }
                }
                d.img16 = off / 16;
                for (int l = tail_start; l <= L; ++l) {
                    const int vb = (int)al16(lev[l]->N * (long long)sizeof(cx<T>));
                    d.offb[l] = off;
                    d.offx[l] = off + vb;
                    d.offt[l] = off + 2 * vb;
                    off += 3 * vb;
                }
                // the coarsest inverse too, when small and within the budget
                const long long mb = (long long)nL * nL * (long long)sizeof(cx<T>);
                d.o_minv = -1;
                if (mb <= 32 * 1024 && off + al16(mb) <= budget) {
                    d.o_minv = off;
                    off += (int)al16(mb);
                }
                d.lds_bytes = off;
                for (int l = tail_start; l <= L; ++l) {
                    LevelDev& lv = *lev[l];
                    auto& t = d.lv[l];
                    t.n1 = lv.n1;
                    t.n2 = lv.n2;
                    t.px = p;
                    t.py = is2d ? p : 0;
                    t.kind = lv.kind;
                    t.omega = (T)lv.omega;
                    t.Kx = lv.Kx.as<double>();
                    t.Mx = lv.Mx.as<double>();
                    t.Ky = lv.Ky.as<double>();
                    t.My = lv.My.as<double>();
                    t.S = pick<T>(lv.S64, lv.S32).template as<T>();
                    t.dinv = pick<T>(lv.Dinv64, lv.Dinv32).template as<cx<T>>();
                    t.b = pick<T>(lv.b64, lv.b32).template as<cx<T>>();
                    t.x = pick<T>(lv.x64, lv.x32).template as<cx<T>>();
                    t.r = pick<T>(lv.r64, lv.r32).template as<cx<T>>();
                    t.t = pick<T>(lv.t64, lv.t32).template as<cx<T>>();
                    t.tr = lv.tr;
                }
            };
            std::vector<TailDesc<double>> d64(1);
            std::vector<TailDesc<float>> d32(1);
            std::memset((void*)d64.data(), 0, sizeof(TailDesc<double>));
            std::memset((void*)d32.data(), 0, sizeof(TailDesc<float>));
            fill(d64[0], double{});
            HH_REQUIRE(d64[0].img16 > 0, "tail coefficient image");
            tail_img.alloc((size_t)d64[0].img16 * 16);
            fill(d64[0], double{});
            fill(d32[0], float{});
            HH_REQUIRE(d32[0].img16 == d64[0].img16, "tail image layout");
            // the image: every table copied to its LDS offset (alignment gaps zero)
            HH_HIP(hipMemset(tail_img.p, 0, tail_img.bytes));
            {
                unsigned char* img = tail_img.as<unsigned char>();
                auto put = [&](int o, const void* src, long long bytes) {
                    if (o < 0 || bytes <= 0) return;
                    HH_REQUIRE(o + bytes <= (long long)tail_img.bytes, "tail image bounds");
                    HH_HIP(hipMemcpy(img + o, src, (size_t)bytes, hipMemcpyDeviceToDevice));
                };
                for (int l = tail_start; l < L; ++l) {
                    const LevelDev& v = *lev[l];
                    const auto& t = d64[0].lv[l];
                    const int bx = 2 * p + 1, by = is2d ? 2 * p + 1 : 1;
                    const Transfer& tr = v.tr;
                    put(t.o_kx, v.Kx.p, 8LL * v.n1 * bx);
                    put(t.o_mx, v.Mx.p, 8LL * v.n1 * bx);
                    put(t.o_ky, v.Ky.p, 8LL * v.n2 * by);
                    put(t.o_my, v.My.p, 8LL * v.n2 * by);
                    put(t.o_prow0x, tr.prow0x, 4LL * tr.nf1);
                    put(t.o_prowx, tr.prowx, 8LL * tr.nf1 * tr.pw1);
                    put(t.o_prow0y, tr.prow0y, 4LL * tr.nf2);
                    put(t.o_prowy, tr.prowy, 8LL * tr.nf2 * tr.pw2);
                    put(t.o_pcol0x, tr.pcol0x, 4LL * tr.nc1);
                    put(t.o_pcolx, tr.pcolx, 8LL * tr.nc1 * tr.rw1);
                    put(t.o_pcol0y, tr.pcol0y, 4LL * tr.nc2);
                    put(t.o_pcoly, tr.pcoly, 8LL * tr.nc2 * tr.rw2);
                }
            }
            for (int l = tail_start; l <= L; ++l)
                HH_REQUIRE(lev[l]->kind == KIND_SEP || lev[l]->kind == KIND_STENCIL, "tail level kind");
            upload(tail64, d64);
            upload(tail32, d32);
            tail_lds = d64[0].lds_bytes;
            tail_lds32 = d32[0].lds_bytes;
            tail_P = (is2d && p <= 5) ? p : 0;
            tail_prepare<double>(tail_lds);
            tail_prepare<float>(tail_lds32);
        }
    }
    // deflation levels
    Lz = 0;
    if (o.defl_mode == 1 && L >= 1) Lz = 1;
    if (o.defl_mode == 2 && L >= 1) {
        Lz = L;
        for (int l = 1; l <= L; ++l)
            if (lev[l]->N <= o.defl_direct_max) {
                Lz = l;
                break;
            }
        // not coarser than the last level that still resolves the waves:
        // k_max h_l <= defl_kh_max, h_l the level's longest element
        if (o.defl_kh_max > 0.0) {
            double kmax = P.k;
            if (!const_k) {
                kmax = 0.0;
                for (double v : P.k2) kmax = std::max(kmax, std::sqrt(v));
            }
            auto hmax = [](const Axis& a) {
                double h = 0.0;
                for (size_t i = 0; i + 1 < a.bk.size(); ++i) h = std::max(h, a.bk[i + 1] - a.bk[i]);
                return h;
            };
            int lkh = 1;
            for (int l = 1; l <= L; ++l) {
                const double h = is2d ? std::max(hmax(lev[l]->ax), hmax(lev[l]->ay)) : hmax(lev[l]->ax);
                if (kmax * h <= o.defl_kh_max) lkh = l;
            }
            Lz = std::min(Lz, lkh);
        }
    }
    // C_ex: M_ex = K - (1 + i beta2) k^2 M is separable like E, so its exact
    // inverse is a fast diagonalisation of the finest level with complex 1 / D
    cex = o.precond == 1;
    if (cex) {
        const LevelDev& l0 = *lev[0];
        cex_b2 = o.cex_beta2 > 0.0 ? o.cex_beta2 : (is2d ? 1.0 / (3.0 * P.k) : 1.0 / P.k);
        std::vector<double> Vx, Vy, lx, ly;
        axis_eigen(l0.ax, Vx, lx);
        axis_eigen(l0.ay, Vy, ly);
        const zd g(k2c, cex_b2 * k2c);
        std::vector<cx<double>> dinv((size_t)l0.N);
        for (int a = 0; a < l0.n2; ++a)
            for (int b = 0; b < l0.n1; ++b) {
                const zd d = 1.0 / (zd(ly[a] + lx[b]) - g);
                dinv[(size_t)a * l0.n1 + b] = {d.real(), d.imag()};
            }
        std::vector<double> VxT(Vx.size());
        for (int a = 0; a < l0.n1; ++a)
            for (int b = 0; b < l0.n1; ++b) VxT[(size_t)b * l0.n1 + a] = Vx[(size_t)a * l0.n1 + b];
        upload(cexVx, Vx);
        upload(cexVxT, VxT);
        upload(cexVy, Vy);
        upload(cexDinv, dinv);
        cexT1.alloc((size_t)l0.N * 16);
        cexT2.alloc((size_t)l0.N * 16);
    }
    // ADP deflation vectors: a deflation level of their own after the
    // multigrid levels, with E = Z^T A Z as Galerkin bands (constant k: separable)
    // or bands plus the coarse mass stencil Z^T M_k Z (variable k)
    std::vector<double> Sadp;
    zadp = o.defl_z == 1;
    if (zadp) {
        auto lz = std::make_unique<LevelDev>();
        const LevelDev& l0 = *lev[0];
        Axis zfx, zfy;
        make_adp(l0.ax, o.defl_eps, zfx, lz->ax);
        if (is2d) {
            make_adp(l0.ay, o.defl_eps, zfy, lz->ay);
        } else {
            zfy = make_trivial_axis();
            lz->ay = make_trivial_axis();
        }
        lz->n1 = lz->ax.n;
        lz->n2 = lz->ay.n;
        lz->N = (long long)lz->n1 * lz->n2;
        lz->kind = const_k ? KIND_SEP : KIND_STENCIL;
        upload(lz->Kx, lz->ax.Kb);
        upload(lz->Mx, lz->ax.Mb);
        upload(lz->Ky, lz->ay.Kb);
        upload(lz->My, lz->ay.Mb);
        if (!const_k) {
            galerkin_stencil_z(l0.ax, l0.ay, Sh[0], zfx, zfy, lz->ax, lz->ay, Sadp);
            upload(lz->S64, Sadp);
        }
        upload(zprow0x, zfx.prow0);
        upload(zprowx, zfx.prow);
        upload(zpcol0x, zfx.pcol0);
        upload(zpcolx, zfx.pcol);
        upload(zprow0y, zfy.prow0);
        upload(zprowy, zfy.prow);
        upload(zpcol0y, zfy.pcol0);
        upload(zpcoly, zfy.pcol);
        Transfer& t = ztr;
        t.nf1 = l0.n1;
        t.nf2 = l0.n2;
        t.nc1 = lz->n1;
        t.nc2 = lz->n2;
        t.pw1 = zfx.pw;
        t.pw2 = zfy.pw;
        t.rw1 = zfx.rw;
        t.rw2 = zfy.rw;
        t.prow0x = zprow0x.as<int>();
        t.prowx = zprowx.as<double>();
        t.prow0y = zprow0y.as<int>();
        t.prowy = zprowy.as<double>();
        t.pcol0x = zpcol0x.as<int>();
        t.pcolx = zpcolx.as<double>();
        t.pcol0y = zpcol0y.as<int>();
        t.pcoly = zpcoly.as<double>();
        lev.push_back(std::move(lz));
        Lz = L + 1;
    }
    // the direct deflation level's mass stencil (variable k)
    const std::vector<double>& Sz =
        zadp ? Sadp : (Lz > 0 && !Shg[Lz].empty() ? Shg[Lz] : Sh[std::min(Lz, L)]);
    if (Lz > 0 && P.somm) {
        // radiation condition: E = Z^T A Z is complex (boundary term on its last
        // unknown) and not separable; its dense inverse, formed on the host
        LevelDev& lz = *lev[Lz];
        nZ = (int)lz.N;
        HH_REQUIRE(nZ <= 4096, "direct deflation level too large for the radiation condition (at most 4096 unknowns)");
        std::vector<zd> Ez((size_t)nZ * nZ, 0.0);
        for (long long I = 0; I < lz.N; ++I)
            visit_row(lz.ax, lz.ay, const_k, k2c, Sz, I,
                      [&](long long J, double kv, double mv) { Ez[(size_t)I * nZ + J] += kv - mv; });
        Ez[(size_t)lz.bnd_I * nZ + lz.bnd_I] += zd(0.0, lz.bnd_im);
        invert_complex(nZ, Ez);
        std::vector<cx<double>> ez((size_t)nZ * nZ);
        for (size_t i = 0; i < Ez.size(); ++i) ez[i] = {Ez[i].real(), Ez[i].imag()};
        upload(EinvC, ez);
    } else if (Lz > 0 && const_k) {
        // separable E: exact inverse by fast diagonalisation, no dense matrix
        LevelDev& lz = *lev[Lz];
        nZ = (int)lz.N;
        std::vector<double> Vx, Vy, lx, ly;
        axis_eigen(lz.ax, Vx, lx);
        axis_eigen(lz.ay, Vy, ly);
        std::vector<double> dinv((size_t)nZ);
        double scale = k2c;
        for (double v : lx) scale = std::max(scale, std::fabs(v));
        for (double v : ly) scale = std::max(scale, std::fabs(v));
        for (int a = 0; a < lz.n2; ++a)
            for (int b = 0; b < lz.n1; ++b) {
                const double d = ly[a] + lx[b] - k2c;
                if (!(std::fabs(d) > 1e-14 * scale)) throw Err{HH_ENUMERIC, "deflation matrix E is singular"};
                dinv[(size_t)a * lz.n1 + b] = 1.0 / d;
            }
        upload(fdmVx, Vx);
        {
            std::vector<double> VxT(Vx.size());
            for (int a = 0; a < lz.n1; ++a)
                for (int b = 0; b < lz.n1; ++b) VxT[(size_t)b * lz.n1 + a] = Vx[(size_t)a * lz.n1 + b];
            upload(fdmVxT, VxT);
        }
        upload(fdmVy, Vy);
        upload(fdmDinv, dinv);
        fdmT1.alloc((size_t)nZ * 16);
        fdmT2.alloc((size_t)nZ * 16);
        fdm = true;
    } else if (Lz > 0) {
        LevelDev& lz = *lev[Lz];
        nZ = (int)lz.N;
        const bool want_sub = o.defl_direct_solver == 2 || (o.defl_direct_solver == 0 && nZ >= 2048);
        const auto cands = want_sub ? substruct_partitions(lz.n1, lz.n2, lz.ax.p, lz.ay.p, kSubCandidates)
                                    : std::vector<std::pair<int, int>>();
        if (o.defl_direct_solver == 2 && cands.empty())
            throw Err{HH_EINVAL, "no substructuring cut fits the direct deflation level"};
        // variable k, substructured: exact E^-1 from per-subdomain inverses and
        // the dense inverse of the separator Schur complement.  The block
        // elimination is exact but loses accuracy when a subdomain block is near
        // a Dirichlet resonance of the Helmholtz operator, so the cheapest cuts
        // are tried in turn until one passes the set-up check; the best one is
        // kept, with iterative refinement where it still falls short.
        std::unique_ptr<SubstructE> best;
        for (const auto& bxy : cands) {
            sub = std::make_unique<SubstructE>();
            substruct_build(
                *sub, lz.n1, lz.n2, lz.ax.p, lz.ay.p, bxy.first, bxy.second,
                [&](long long I, const std::function<void(long long, double)>& f) {
                    visit_row(lz.ax, lz.ay, const_k, k2c, Sz, I,
                              [&](long long J, double kv, double mv) { f(J, kv - mv); });
                },
                s);
            sub->check0 = substruct_check(s);
            if (!best || sub->check0 < best->check0) best = std::move(sub);
            if (best->check0 <= kSubCheckTol) break;
        }
        sub = std::move(best);
        if (sub) {
            const double c0 = sub->check0;
            if (!(c0 < 0.5))
                throw Err{HH_ENUMERIC, "substructured E^-1 check failed (relative residual " + std::to_string(c0) + ")"};
            // each refinement step multiplies the residual by about c0
            int m = 0;
            for (double r = c0; r > kSubCheckTol && m < kSubMaxRefine; r *= c0) ++m;
            if (o.defl_refine >= 0) m = o.defl_refine;
            sub->refine = m;
            sub->self_check = m ? substruct_check(s) : c0;
        }
    }
    if (Lz > 0 && !const_k && !sub && !P.somm) {
        // variable k: dense inverse of E, assembled on the device from its
        // nonzeros (E and its inverse are symmetric, so row- and column-major
        // storage coincide)
        LevelDev& lz = *lev[Lz];
        HH_REQUIRE(nZ <= 65536, "direct deflation level too large (at most 65536 unknowns)");
        ldZ = (nZ + 1) & ~1LL;   // even leading dimension: 16-byte aligned rows
        std::vector<long long> cidx;
        std::vector<double> cval;
        std::vector<std::pair<long long, double>> row;
        for (long long I = 0; I < lz.N; ++I) {
            row.clear();
            visit_row(lz.ax, lz.ay, const_k, k2c, Sz, I, [&](long long J, double kv, double mv) {
                for (auto& e : row)
                    if (e.first == J) {
                        e.second += kv - mv;
                        return;
                    }
                row.emplace_back(J, kv - mv);
            });
            for (const auto& e : row) {
                cidx.push_back(I * ldZ + e.first);
                cval.push_back(e.second);
            }
        }
        const size_t nn = (size_t)ldZ * nZ;
        Einv.alloc(nn * sizeof(double));
        {
            DevBuf di, dv;
            upload(di, cidx);
            upload(dv, cval);
            HH_HIP(hipMemsetAsync(Einv.p, 0, nn * sizeof(double), s));
            launch_scatter(cidx.size(), di.as<long long>(), dv.as<double>(), Einv.as<double>(), s);
            HH_HIP(hipStreamSynchronize(s));
        }
        rocblas_handle h;
        if (rocblas_create_handle(&h) != rocblas_status_success) throw Err{HH_EHIP, "rocblas_create_handle failed"};
        rocblas_set_stream(h, s);
        long long singular = 0;
        rocblas_status st;
        if (nZ <= 32768) {
            DevBuf ipiv, info;
            ipiv.alloc((size_t)nZ * sizeof(rocblas_int));
            info.alloc(sizeof(rocblas_int));
            st = rocsolver_dgetrf(h, nZ, nZ, Einv.as<double>(), (rocblas_int)ldZ, ipiv.as<rocblas_int>(),
                                  info.as<rocblas_int>());
            if (st == rocblas_status_success)
                st = rocsolver_dgetri(h, nZ, Einv.as<double>(), (rocblas_int)ldZ, ipiv.as<rocblas_int>(),
                                      info.as<rocblas_int>());
            HH_HIP(hipStreamSynchronize(s));
            rocblas_int hinfo = 0;
            HH_HIP(hipMemcpy(&hinfo, info.p, sizeof(hinfo), hipMemcpyDeviceToHost));
            singular = hinfo;
        } else {
            // more than 2^31 entries: 64-bit LU, then E^-1 = solve against the identity
            DevBuf ipiv, info, X;
            ipiv.alloc((size_t)nZ * sizeof(int64_t));
            info.alloc(sizeof(int64_t));
            X.alloc(nn * sizeof(double));
            HH_HIP(hipMemsetAsync(X.p, 0, nn * sizeof(double), s));
            launch_set_identity(nZ, ldZ, X.as<double>(), s);
            st = rocsolver_dgetrf_64(h, nZ, nZ, Einv.as<double>(), ldZ, ipiv.as<int64_t>(), info.as<int64_t>());
            HH_HIP(hipStreamSynchronize(s));
            int64_t hinfo = 0;
            HH_HIP(hipMemcpy(&hinfo, info.p, sizeof(hinfo), hipMemcpyDeviceToHost));
            singular = hinfo;
            if (st == rocblas_status_success && hinfo == 0)
                st = rocsolver_dgetrs_64(h, rocblas_operation_none, nZ, nZ, Einv.as<double>(), ldZ,
                                         ipiv.as<int64_t>(), X.as<double>(), ldZ);
            HH_HIP(hipStreamSynchronize(s));
            std::swap(Einv.p, X.p);
            std::swap(Einv.bytes, X.bytes);
        }
        rocblas_destroy_handle(h);
        if (st != rocblas_status_success) throw Err{HH_EHIP, "rocsolver LU inverse failed"};
        if (singular != 0) throw Err{HH_ENUMERIC, "deflation matrix E is singular"};
        // E^-1 is symmetric: keep only its upper triangle (half the bytes per product)
        if (nZ >= 2048) {
            EinvP.alloc((size_t)sym_packed_doubles(nZ) * sizeof(double));
            launch_sym_pack(nZ, ldZ, Einv.as<double>(), EinvP.as<double>(), s);
            symRow.alloc((size_t)sym_tiles(nZ) * 128 * sizeof(cx<double>));
            symCol.alloc((size_t)sym_tiles(nZ) * 128 * sizeof(cx<double>));
            HH_HIP(hipStreamSynchronize(s));
            Einv.release();
            sym = true;
        }
    }
    setup_finish(s);
}

// Unit cube (constant k, Dirichlet): the multigrid levels by knot halving in
// all three directions, their transfers P_z (x) P_y (x) P_x, Jacobi diagonals
// and damping, the dense inverse of the coarsest M_beta, and the deflation
// matrix E = A_Lz of the direct deflation level by fast diagonalisation (the
// three 1D pencils); the levels between 1 and Lz - 1 get inner FGMRES solves.
void SolverImpl::setup_levels_3d(hipStream_t s) {
    const ProblemImpl& P = *prob;
    HH_REQUIRE(P.k_mode == 0, "3D problems are built for constant k");
    HH_REQUIRE(o.precond == 0, "3D problems are built with the multigrid CSLP (no C_ex)");
    const int p = P.p;
    for (int l = 0;; ++l) {
        auto lv = std::make_unique<LevelDev>();
        lv->ax = l == 0 ? P.ax0 : make_axis(p, P.nel[0], l, false, P.len[0]);
        lv->ay = l == 0 ? P.ay0 : make_axis(p, P.nel[1], l, false, P.len[1]);
        lv->az = l == 0 ? P.az0 : make_axis(p, P.nel[2], l, false, P.len[2]);
        HH_REQUIRE(lv->ax.n >= 1 && lv->ay.n >= 1 && lv->az.n >= 1, "level without interior unknowns");
        const int mx = std::max({lv->ax.nel, lv->ay.nel, lv->az.nel});
        lev.push_back(std::move(lv));
        if (mx <= o.mg_min_elems) break;
    }
    L = (int)lev.size() - 1;
    for (int l = 0; l < L; ++l) {
        make_transfer(lev[l]->ax, lev[l + 1]->ax);
        make_transfer(lev[l]->ay, lev[l + 1]->ay);
        make_transfer(lev[l]->az, lev[l + 1]->az);
    }
    const double k2c = P.k * P.k;
    const zd beta(o.beta[0], o.beta[1]);
    for (int l = 0; l <= L; ++l) {
        LevelDev& lv = *lev[l];
        lv.n1 = lv.ax.n;
        lv.n2 = lv.ay.n;
        lv.n3 = lv.az.n;
        lv.N = (long long)lv.n1 * lv.n2 * lv.n3;
        lv.kind = KIND_SEP;
        upload(lv.Kx, lv.ax.Kb);
        upload(lv.Mx, lv.ax.Mb);
        upload(lv.Ky, lv.ay.Kb);
        upload(lv.My, lv.ay.Mb);
        upload(lv.Kz, lv.az.Kb);
        upload(lv.Mz, lv.az.Mb);
        std::vector<cx<double>> dinv((size_t)lv.N);
        std::vector<cx<float>> dinv32((size_t)lv.N);
        double g = 0.0;
        for (long long I = 0; I < lv.N; ++I) {
            zd diag = 0.0;
            double rowsum = 0.0;
            visit_row3(lv.ax, lv.ay, lv.az, k2c, I, [&](long long J, double kv, double mv) {
                const zd e = kv - beta * mv;
                rowsum += std::abs(e);
                if (J == I) diag = e;
            });
            HH_REQUIRE(std::abs(diag) > 0.0, "zero Jacobi diagonal");
            g = std::max(g, rowsum / std::abs(diag));
            const zd di = 1.0 / diag;
            dinv[I] = {di.real(), di.imag()};
            dinv32[I] = {(float)di.real(), (float)di.imag()};
        }
        lv.gersh = g;
        // the Gershgorin-bounded damping on every level, the finest included: the
        // three-fold product of 1D masses puts D^-1 M_beta of the finest level
        // beyond 2 / omega already
        lv.omega = o.coarse_damping == 0 ? o.omega : std::min(o.omega, 2.0 / g);
        upload(lv.Dinv64, dinv);
        upload(lv.Dinv32, dinv32);
        const size_t v64 = (size_t)lv.N * 16, v32 = (size_t)lv.N * 8;
        for (DevBuf* b : {&lv.b64, &lv.x64, &lv.r64, &lv.t64}) b->alloc(v64);
        for (DevBuf* b : {&lv.b32, &lv.x32, &lv.r32, &lv.t32}) b->alloc(v32);
        if (o.n_vcycles > 1) {
            lv.vr64.alloc(v64);
            lv.vx64.alloc(v64);
            lv.vr32.alloc(v32);
            lv.vx32.alloc(v32);
        }
    }
    for (int l = 0; l < L; ++l) {
        LevelDev& lv = *lev[l];
        const LevelDev& lc = *lev[l + 1];
        upload(lv.prow0x, lv.ax.prow0);
        upload(lv.prowx, lv.ax.prow);
        upload(lv.pcol0x, lv.ax.pcol0);
        upload(lv.pcolx, lv.ax.pcol);
        upload(lv.prow0y, lv.ay.prow0);
        upload(lv.prowy, lv.ay.prow);
        upload(lv.pcol0y, lv.ay.pcol0);
        upload(lv.pcoly, lv.ay.pcol);
        upload(lv.prow0z, lv.az.prow0);
        upload(lv.prowz, lv.az.prow);
        upload(lv.pcol0z, lv.az.pcol0);
        upload(lv.pcolz, lv.az.pcol);
        Transfer& t = lv.tr;
        t.nf1 = lv.n1;
        t.nf2 = lv.n2;
        t.nf3 = lv.n3;
        t.nc1 = lc.n1;
        t.nc2 = lc.n2;
        t.nc3 = lc.n3;
        t.pw1 = lv.ax.pw;
        t.pw2 = lv.ay.pw;
        t.pw3 = lv.az.pw;
        t.rw1 = lv.ax.rw;
        t.rw2 = lv.ay.rw;
        t.rw3 = lv.az.rw;
        t.prow0x = lv.prow0x.as<int>();
        t.prowx = lv.prowx.as<double>();
        t.prow0y = lv.prow0y.as<int>();
        t.prowy = lv.prowy.as<double>();
        t.prow0z = lv.prow0z.as<int>();
        t.prowz = lv.prowz.as<double>();
        t.pcol0x = lv.pcol0x.as<int>();
        t.pcolx = lv.pcolx.as<double>();
        t.pcol0y = lv.pcol0y.as<int>();
        t.pcoly = lv.pcoly.as<double>();
        t.pcol0z = lv.pcol0z.as<int>();
        t.pcolz = lv.pcolz.as<double>();
        const size_t na = (size_t)lv.n3 * lv.n2 * lc.n1, nb = (size_t)lv.n3 * lc.n2 * lc.n1;
        lv.tra64.alloc(na * sizeof(cx<double>));
        lv.trb64.alloc(nb * sizeof(cx<double>));
        lv.tra32.alloc(na * sizeof(cx<float>));
        lv.trb32.alloc(nb * sizeof(cx<float>));
        t.tmpa64 = lv.tra64.as<cx<double>>();
        t.tmpb64 = lv.trb64.as<cx<double>>();
        t.tmpa32 = lv.tra32.as<cx<float>>();
        t.tmpb32 = lv.trb32.as<cx<float>>();
    }
    {
        LevelDev& lc = *lev[L];
        nL = (int)lc.N;
        HH_REQUIRE(nL <= 4096, "coarsest multigrid level too large (raise the coarsening: mg_min_elems)");
        std::vector<zd> A((size_t)nL * nL, 0.0);
        for (long long I = 0; I < lc.N; ++I)
            visit_row3(lc.ax, lc.ay, lc.az, k2c, I,
                       [&](long long J, double kv, double mv) { A[(size_t)I * nL + J] += kv - beta * mv; });
        invert_complex(nL, A);
        std::vector<cx<double>> m64((size_t)nL * nL);
        std::vector<cx<float>> m32((size_t)nL * nL);
        for (size_t i = 0; i < A.size(); ++i) {
            m64[i] = {A[i].real(), A[i].imag()};
            m32[i] = {(float)A[i].real(), (float)A[i].imag()};
        }
        upload(Minv64, m64);
        upload(Minv32, m32);
    }
    // deflation levels as in 2D: two-level (level 1), or multilevel with the first level
    // of at most defl_direct_max unknowns solved directly, not coarser than the last
    // level that still resolves the waves (k h_l <= defl_kh_max)
    Lz = (o.defl_mode >= 1 && L >= 1) ? 1 : 0;
    if (o.defl_mode == 2 && L >= 1) {
        Lz = L;
        for (int l = 1; l <= L; ++l)
            if (lev[l]->N <= o.defl_direct_max) {
                Lz = l;
                break;
            }
        if (o.defl_kh_max > 0.0) {
            auto hmax = [](const Axis& a) {
                double h = 0.0;
                for (size_t i = 0; i + 1 < a.bk.size(); ++i) h = std::max(h, a.bk[i + 1] - a.bk[i]);
                return h;
            };
            int lkh = 1;
            for (int l = 1; l <= L; ++l) {
                const double h = std::max({hmax(lev[l]->ax), hmax(lev[l]->ay), hmax(lev[l]->az)});
                if (P.k * h <= o.defl_kh_max) lkh = l;
            }
            Lz = std::min(Lz, lkh);
        }
    }
    // ADP deflation vectors (two-level): Z = Z_z (x) Z_y (x) Z_x from level 0 to a
    // deflation level of its own, lev[L + 1]
    zadp = o.defl_z == 1;
    if (zadp) {
        auto lz = std::make_unique<LevelDev>();
        const LevelDev& l0 = *lev[0];
        Axis zf[3];
        make_adp(l0.ax, o.defl_eps, zf[0], lz->ax);
        make_adp(l0.ay, o.defl_eps, zf[1], lz->ay);
        make_adp(l0.az, o.defl_eps, zf[2], lz->az);
        lz->n1 = lz->ax.n;
        lz->n2 = lz->ay.n;
        lz->n3 = lz->az.n;
        lz->N = (long long)lz->n1 * lz->n2 * lz->n3;
        lz->kind = KIND_SEP;
        upload(lz->Kx, lz->ax.Kb);
        upload(lz->Mx, lz->ax.Mb);
        upload(lz->Ky, lz->ay.Kb);
        upload(lz->My, lz->ay.Mb);
        upload(lz->Kz, lz->az.Kb);
        upload(lz->Mz, lz->az.Mb);
        upload(zprow0x, zf[0].prow0);
        upload(zprowx, zf[0].prow);
        upload(zpcol0x, zf[0].pcol0);
        upload(zpcolx, zf[0].pcol);
        upload(zprow0y, zf[1].prow0);
        upload(zprowy, zf[1].prow);
        upload(zpcol0y, zf[1].pcol0);
        upload(zpcoly, zf[1].pcol);
        upload(zprow0z, zf[2].prow0);
        upload(zprowz, zf[2].prow);
        upload(zpcol0z, zf[2].pcol0);
        upload(zpcolz, zf[2].pcol);
        Transfer& t = ztr;
        t.nf1 = l0.n1;
        t.nf2 = l0.n2;
        t.nf3 = l0.n3;
        t.nc1 = lz->n1;
        t.nc2 = lz->n2;
        t.nc3 = lz->n3;
        t.pw1 = zf[0].pw;
        t.pw2 = zf[1].pw;
        t.pw3 = zf[2].pw;
        t.rw1 = zf[0].rw;
        t.rw2 = zf[1].rw;
        t.rw3 = zf[2].rw;
        t.prow0x = zprow0x.as<int>();
        t.prowx = zprowx.as<double>();
        t.prow0y = zprow0y.as<int>();
        t.prowy = zprowy.as<double>();
        t.prow0z = zprow0z.as<int>();
        t.prowz = zprowz.as<double>();
        t.pcol0x = zpcol0x.as<int>();
        t.pcolx = zpcolx.as<double>();
        t.pcol0y = zpcol0y.as<int>();
        t.pcoly = zpcoly.as<double>();
        t.pcol0z = zpcol0z.as<int>();
        t.pcolz = zpcolz.as<double>();
        // the deflation passes run in FP64 only (no FP32 intermediate grids)
        ztra64.alloc((size_t)l0.n3 * l0.n2 * lz->n1 * sizeof(cx<double>));
        ztrb64.alloc((size_t)l0.n3 * lz->n2 * lz->n1 * sizeof(cx<double>));
        t.tmpa64 = ztra64.as<cx<double>>();
        t.tmpb64 = ztrb64.as<cx<double>>();
        lev.push_back(std::move(lz));
        Lz = L + 1;
    }
    if (Lz > 0) {
        const LevelDev& lz = *lev[Lz];
        nZ = (int)lz.N;
        std::vector<double> V[3], lam[3];
        axis_eigen(lz.ax, V[0], lam[0]);
        axis_eigen(lz.ay, V[1], lam[1]);
        axis_eigen(lz.az, V[2], lam[2]);
        double scale = k2c;
        for (auto& l : lam)
            for (double v : l) scale = std::max(scale, std::fabs(v));
        std::vector<double> dinv((size_t)nZ);
        for (int c = 0; c < lz.n3; ++c)
            for (int a = 0; a < lz.n2; ++a)
                for (int b = 0; b < lz.n1; ++b) {
                    const double d = lam[2][c] + lam[1][a] + lam[0][b] - k2c;
                    if (!(std::fabs(d) > 1e-14 * scale)) throw Err{HH_ENUMERIC, "deflation matrix E is singular"};
                    dinv[((size_t)c * lz.n2 + a) * lz.n1 + b] = 1.0 / d;
                }
        auto transpose = [](const std::vector<double>& M, int n) {
            std::vector<double> T(M.size());
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) T[(size_t)b * n + a] = M[(size_t)a * n + b];
            return T;
        };
        upload(fdmVx, V[0]);
        upload(fdmVxT, transpose(V[0], lz.n1));
        upload(fdmVy, V[1]);
        upload(fdmVyT, transpose(V[1], lz.n2));
        upload(fdmVz, V[2]);
        upload(fdmVzT, transpose(V[2], lz.n3));
        upload(fdmDinv, dinv);
        fdmT1.alloc((size_t)nZ * 16);
        fdmT2.alloc((size_t)nZ * 16);
        fdm = true;
    }
}

void SolverImpl::setup_finish(hipStream_t s) {
    const ProblemImpl& P = *prob;
    const bool const_k = P.k_mode == 0;
    const double k2c = const_k ? P.k * P.k : 0.0;
    if (Lz > 0) {
        for (int l = 0; l < defl_end(); ++l) {
            LevelDev& lv = *lev[l];
            const size_t v64 = (size_t)lv.N * 16;
            lv.tq.alloc(v64);
            lv.tw.alloc(v64);
            lv.ts.alloc(v64);
        }
        for (int l = zadp ? Lz : 1; l <= Lz; ++l) {
            LevelDev& lv = *lev[l];
            const size_t v64 = (size_t)lv.N * 16;
            lv.tc.alloc(v64);
            lv.te.alloc(v64);
            if (l < Lz) {
                lv.m_inner = o.defl_inner_its[std::min(l - 1, 7)];
                lv.V.alloc(v64 * (lv.m_inner + 1));
                lv.Z.alloc(v64 * lv.m_inner);
                fill_krylov(lv.kd, lv.kstate, lv.m_inner);
            }
        }
    }
    // feature of the learned smoother: c = k^2 h^2 of the finest element with the
    // unknown's (clamped) index
    if (P.dim <= 2) {   // the learned smoother's feature (2D and 1D)
        const LevelDev& l0 = *lev[0];
        std::vector<float> c((size_t)l0.N);
        const double hx = P.len[0] / P.nel[0], h2 = hx * hx;   // the x extent of an element
        for (int i2 = 0; i2 < l0.n2; ++i2)
            for (int i1 = 0; i1 < l0.n1; ++i1) {
                const int e2 = std::min(i2, l0.ay.nel - 1), e1 = std::min(i1, l0.ax.nel - 1);
                const double k2 = const_k ? k2c : P.k2[(size_t)e2 * P.nel[0] + e1];
                c[(size_t)i2 * l0.n1 + i1] = (float)(k2 * h2);
            }
        upload(feat, c);
    }
    {
        const int nmax = std::max({lev[0]->n1, lev[0]->n2, lev[0]->n3});
        zero_bands.alloc((size_t)nmax * (2 * std::max(P.p, lev[Lz]->ax.p) + 1) * sizeof(double));
        HH_HIP(hipMemsetAsync(zero_bands.p, 0, zero_bands.bytes, s));
    }
    // outer FGMRES workspace
    m_outer = o.restart;
    const size_t v0 = (size_t)lev[0]->N * 16;
    V.alloc(v0 * (m_outer + 1));
    Z.alloc(v0 * m_outer);
    r.alloc(v0);
    fill_krylov(kd, kstate, m_outer);
    if (o.autotune) autotune_ops(s);
    HH_HIP(hipHostMalloc((void**)&pin_d, 16 * sizeof(double), hipHostMallocDefault));
    HH_HIP(hipHostMalloc((void**)&pin_i, 64 * sizeof(int), hipHostMallocDefault));
    std::memset(pin_d, 0, 16 * sizeof(double));
    std::memset(pin_i, 0, 64 * sizeof(int));
    HH_HIP(hipHostMalloc((void**)&pin_step, 256, hipHostMallocDefault));
    std::memset(pin_step, 0, 256);
    // the outer Arnoldi kernels store the host's step scalars in these slots
    // through their device address (without one, the driver copies them)
    void* dstep = nullptr;
    if (hipHostGetDevicePointer(&dstep, pin_step, 0) == hipSuccess && dstep)
        kd.hstep = (unsigned char*)dstep;
    else
        (void)hipGetLastError();
    for (hipEvent_t* e : {&ev_slot[0], &ev_slot[1], &ev_misc})
        HH_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
    if (o.use_graph) {
        // graphs are captured on a stream of the solver's own (the caller's may
        // be the legacy default stream, which cannot capture); default priority
        HH_HIP(hipStreamCreateWithFlags(&gstream, hipStreamNonBlocking));
        HH_HIP(hipEventCreateWithFlags(&gfork, hipEventDisableTiming));
        HH_HIP(hipEventCreateWithFlags(&gjoin, hipEventDisableTiming));
    }
    HH_HIP(hipStreamSynchronize(s));
}

// Strip-height autotuner of the level-operator kernel: on every level outside
// the single-workgroup tail (and of at least 4096 unknowns), time the residual
// kernel with 4, 8, ..., 64 rows per strip (one warm-up, then the best of three
// launches per candidate, HIP events on the setup stream) in FP64 and FP32 and
// keep the fastest.  Each output row sums its 2p+1 input rows in the same order
// whatever the strip height, so the choice changes speed only.
void SolverImpl::autotune_ops(hipStream_t s) {
    if (prob->dim == 1) return;
    // 2D: strip height of the row-marching kernel (64..4 rows); 3D: output slices
    // per workgroup of the slice-marching kernel (32..2); either gives the same bits
    const bool cube = prob->dim == 3;
    hipEvent_t e0, e1;
    HH_HIP(hipEventCreate(&e0));
    HH_HIP(hipEventCreate(&e1));
    auto tune = [&](int l, auto tag) {
        using T = decltype(tag);
        LevelDev& lv = *lev[l];
        int& slot = (sizeof(T) == 8) ? lv.ty64 : lv.ty32;
        cx<T>* x = pick<T>(lv.x64, lv.x32).template as<cx<T>>();
        cx<T>* b = pick<T>(lv.b64, lv.b32).template as<cx<T>>();
        cx<T>* y = pick<T>(lv.r64, lv.r32).template as<cx<T>>();
        HH_HIP(hipMemsetAsync(x, 0, (size_t)lv.N * sizeof(cx<T>), s));
        HH_HIP(hipMemsetAsync(b, 0, (size_t)lv.N * sizeof(cx<T>), s));
        float best = 1e30f;
        int best_ty = 0;
        for (int ty = cube ? 32 : 64; ty >= (cube ? 2 : 4); ty >>= 1) {
            slot = ty;
            op<T>(l, MODE_RESID, true, x, b, y, s);
            float t_min = 1e30f;
            for (int r = 0; r < 3; ++r) {
                HH_HIP(hipEventRecord(e0, s));
                op<T>(l, MODE_RESID, true, x, b, y, s);
                HH_HIP(hipEventRecord(e1, s));
                HH_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                HH_HIP(hipEventElapsedTime(&ms, e0, e1));
                t_min = std::min(t_min, ms);
            }
            if (t_min < best) {
                best = t_min;
                best_ty = ty;
            }
        }
        slot = best_ty;
    };
    const int last = std::min(L - 1, tail_start - 1);
    const bool timing = o.time_kernels;
    o.time_kernels = 0;
    for (int l = 0; l <= last; ++l) {
        // small constant-k levels use the direct kernel, stored stencils the
        // direct or the tiled kernel (no strips in either)
        if (!cube && lev[l]->N <= kOpDirectMax && lev[l]->kind != KIND_VARFINE) continue;
        if (lev[l]->kind == KIND_STENCIL) continue;
        tune(l, double{});
        tune(l, float{});
    }
    o.time_kernels = timing;
    HH_HIP(hipEventDestroy(e0));
    HH_HIP(hipEventDestroy(e1));
}

// ----------------------------------------------------------- hot path ----
template <class T>
void SolverImpl::op(int l, int mode, bool cslp, const cx<T>* x, const cx<T>* b, cx<T>* y, hipStream_t s, cx<T>* xo,
                    const cx<T>* yadd) {
    op_alpha<T>(l, mode, cslp ? o.beta[0] : 1.0, cslp ? o.beta[1] : 0.0, x, b, y, s, xo, yadd, cslp);
}

// y = K x - alpha M_k x at level l, with the residual / Jacobi epilogues (mode)
template <class T>
void SolverImpl::op_alpha(int l, int mode, double are, double aim, const cx<T>* x, const cx<T>* b, cx<T>* y,
                          hipStream_t s, cx<T>* xo, const cx<T>* yadd, bool mg, bool mass_only) {
    LevelDev& lv = *lev[l];
    OpArgs<T> a{};
    a.n1 = lv.n1;
    a.n2 = lv.n2;
    // mass_only: zero stiffness bands, so y = -alpha M_k x exactly
    a.Kx = mass_only ? zero_bands.as<double>() : lv.Kx.as<double>();
    a.Mx = lv.Mx.as<double>();
    a.Ky = mass_only ? zero_bands.as<double>() : lv.Ky.as<double>();
    a.My = lv.My.as<double>();
    a.k2c = prob->k_mode == 0 ? prob->k * prob->k : 0.0;
    a.k2 = prob->k2_dev.as<double>();
    a.nel1 = lv.ax.nel;
    a.nel2 = lv.ay.nel;
    a.off1 = lv.ax.off;
    a.off2 = lv.ay.off;
    a.Mex = lv.Mex.as<double>();
    a.Mey = lv.Mey.as<double>();
    // the deflation operator A_l of a rediscretised level keeps its Galerkin stencil
    a.S = (!mg && sizeof(T) == 8 && lv.S64a.p) ? lv.S64a.template as<T>() : pick<T>(lv.S64, lv.S32).template as<T>();
    a.are = (T)are;
    a.aim = (T)aim;
    a.x = x;
    a.b = b;
    a.y = y;
    a.dinv = pick<T>(lv.Dinv64, lv.Dinv32).template as<cx<T>>();
    a.omega = (T)lv.omega;
    a.xo = xo;
    a.yadd = mode == MODE_SMOOTH ? yadd : nullptr;
    a.ty = sizeof(T) == 8 ? lv.ty64 : lv.ty32;
    // the radiation condition's boundary term belongs to A and M_beta, not to K or M_k alone
    const bool with_bnd = !mass_only && (are != 0.0 || aim != 0.0);
    a.bnd_I = with_bnd ? lv.bnd_I : -1;
    a.bnd_im = (T)lv.bnd_im;
    if (prob->dim == 3) {
        a.n3 = lv.n3;
        a.Kz = mass_only ? zero_bands.as<double>() : lv.Kz.as<double>();
        a.Mz = lv.Mz.as<double>();
    }
    // band half-widths of the level (the degree p, or wider on the ADP level)
    const int px = lv.ax.p, py = prob->dim >= 2 ? lv.ay.p : 0;
    double st_bytes = 0.0;
    {
        // operands once: x, y, b (residual / sweep), D^-1 (sweep), the first-sweep
        // and added vectors, and the mass coefficients: the stored stencil or
        // k^2 per finest element
        const int p = px, bx = 2 * p + 1, by = py ? 2 * py + 1 : 1;
        const double v = (double)lv.N * sizeof(cx<T>);
        double bytes = 2 * v + (mode != MODE_APPLY ? v : 0.0) + (mode == MODE_SMOOTH || xo ? v : 0.0) +
                       (xo ? v : 0.0) + (a.yadd ? v : 0.0);
        double macs = 2.0 * bx * by + 2.0 * by;
        if (prob->dim == 3) macs = 7.0 * bx;   // sum factorised: x, y and z passes
        if (lv.kind == KIND_STENCIL) {
            bytes += (double)lv.N * bx * by * sizeof(T);
            macs += bx * by;
        } else if (lv.kind == KIND_VARFINE) {
            bytes += 8.0 * (double)lv.ax.nel * lv.ay.nel;
            macs += (py + 1) * (2.0 * (p + 1) * (p + 1) + (p + 1) * bx);
        }
        meter(bytes, 4.0 * macs * lv.N + (mode == MODE_SMOOTH ? 10.0 : 2.0) * lv.N);
        st_bytes = bytes;
    }
    // timing class 4: the tiled stored-stencil kernel (2D coarse variable-k levels
    // of at least kStencilTiledMin unknowns)
    const bool st_kernel = lv.kind == KIND_STENCIL && py > 0 && lv.N >= kStencilTiledMin;
    if (st_kernel) tstart(4, s);
    if (l == 0) tstart(1, s);
    launch_op<T>(lv.kind, mode, px, py, a, s);
    if (l == 0) tstop(1, st_bytes, s);
    if (st_kernel) tstop(4, st_bytes, s);
}

template <class T>
bool SolverImpl::vcycle_once(int l, const cx<T>* b, cx<T>* x, hipStream_t s, bool x_swept, cx<T>* zout,
                             const cx<T>* zadd) {
    LevelDev& lv = *lev[l];
    if (l == L) {
        launch_gemv<cx<T>, T>(nL, pick<T>(Minv64, Minv32).template as<cx<T>>(), b, x, s);
        return false;
    }
    if (l >= tail_start) {
        // the tail reads b and its coefficient tables once and writes x; its
        // levels live in LDS.  Flops: residual, two sweeps and transfers per level.
        {
            double fl = 0.0;
            const int p = prob->p, bx = 2 * p + 1, by = prob->dim == 2 ? bx : 1;
            for (int q = l; q <= L; ++q)
                fl += (q == L ? 8.0 * (double)nL * nL : 3.0 * 4.0 * (2.0 * bx * by + 2.0 * by) * lev[q]->N);
            meter(2.0 * sizeof(cx<T>) * lv.N + (double)tail_img.bytes + (double)nL * nL * sizeof(cx<T>), fl);
        }
        launch_vcycle_tail<T>(pick<T>(tail64, tail32).template as<TailDesc<T>>(), tail_img.p,
                              (int)(tail_img.bytes / 16), pick<T>(Minv64, Minv32).template as<cx<T>>(), tail_P, l,
                              sizeof(T) == 8 ? tail_lds : tail_lds32, b, x, s);
        return false;
    }
    cx<T>* t = pick<T>(lv.t64, lv.t32).template as<cx<T>>();
    cx<T>* r = pick<T>(lv.r64, lv.r32).template as<cx<T>>();
    const cx<T>* dinv = pick<T>(lv.Dinv64, lv.Dinv32).template as<cx<T>>();
    const bool learned = (cnn != nullptr && l == 0);
    if (learned) {
        // learned smoother from a zero guess: x = omega D^-1 b + rms(b) C(b/rms(b), c),
        // then further sweeps x += omega D^-1 r + rms(r) C(r/rms(r), c), r = b - M_beta x,
        // rms(r) = ||r|| / sqrt(N)
        cnn->step<T>(lv.n2, lv.n1, b, feat.as<float>(), dinv, (T)lv.omega, x, 0, s);
        for (int i = 1; i < o.nu_pre; ++i) {
            op<T>(l, MODE_RESID, true, x, b, r, s);
            cnn->step<T>(lv.n2, lv.n1, r, feat.as<float>(), dinv, (T)lv.omega, x, 1, s);
        }
    } else {
        // sweeps alternate between x and t; start where an even count of
        // further sweeps ends in x
        cx<T>* cur = ((o.nu_pre - 1) & 1) ? t : x;
        cx<T>* oth = ((o.nu_pre - 1) & 1) ? x : t;
        if (!x_swept) launch_jacobi0<T>(lv.N, dinv, (T)lv.omega, b, cur, s);
        for (int i = 1; i < o.nu_pre; ++i) {
            op<T>(l, MODE_SMOOTH, true, cur, b, oth, s);
            std::swap(cur, oth);
        }
    }
    op<T>(l, MODE_RESID, true, x, b, r, s);
    LevelDev& lc = *lev[l + 1];
    cx<T>* bc = pick<T>(lc.b64, lc.b32).template as<cx<T>>();
    cx<T>* xc = pick<T>(lc.x64, lc.x32).template as<cx<T>>();
    // with one pre-sweep on a coarser level that runs as separate kernels, the
    // restriction also forms that level's first sweep (x = omega D^-1 b)
    if (o.nu_pre == 1 && l + 1 < tail_start && l + 1 < L) {
        const cx<T>* dinvc = pick<T>(lc.Dinv64, lc.Dinv32).template as<cx<T>>();
        launch_restrict<T>(lv.tr, r, bc, s, dinvc, (T)lc.omega, xc);
        vcycle_once<T>(l + 1, bc, xc, s, true);
    } else {
        launch_restrict<T>(lv.tr, r, bc, s);
        vcycle_once<T>(l + 1, bc, xc, s);
    }
    if (learned) {
        launch_prolong<T>(lv.tr, xc, x, 1, s);
        for (int i = 0; i < o.nu_post; ++i) {
            op<T>(l, MODE_RESID, true, x, b, r, s);
            cnn->step<T>(lv.n2, lv.n1, r, feat.as<float>(), dinv, (T)lv.omega, x, 1, s);
        }
        return false;
    }
    // coarse-grid correction into t when an odd number of sweeps follows, so
    // that the last sweep writes x (or zout = x + zadd)
    cx<T>* cur = (o.nu_post & 1) ? t : x;
    cx<T>* oth = (o.nu_post & 1) ? x : t;
    launch_prolong_add<T>(lv.tr, xc, x, cur, s);
    const bool fold = zadd != nullptr && o.nu_post >= 1;
    for (int i = 0; i < o.nu_post; ++i) {
        if (fold && i + 1 == o.nu_post) {
            op<T>(l, MODE_SMOOTH, true, cur, b, zout, s, nullptr, zadd);
            break;
        }
        op<T>(l, MODE_SMOOTH, true, cur, b, oth, s);
        std::swap(cur, oth);
    }
    return fold;
}

template <class T>
bool SolverImpl::vcycle(int l, const cx<T>* b, cx<T>* x, hipStream_t s, bool x_swept, cx<T>* zout,
                        const cx<T>* zadd) {
    if (o.n_vcycles == 1) return vcycle_once<T>(l, b, x, s, x_swept, zout, zadd);
    vcycle_once<T>(l, b, x, s, x_swept);
    LevelDev& lv = *lev[l];
    for (int i = 1; i < o.n_vcycles; ++i) {
        cx<T>* vr = pick<T>(lv.vr64, lv.vr32).template as<cx<T>>();
        cx<T>* vx = pick<T>(lv.vx64, lv.vx32).template as<cx<T>>();
        op<T>(l, MODE_RESID, true, x, b, vr, s);
        vcycle_once<T>(l, vr, vx, s);
        launch_axpy<T>(lv.N, vx, x, s);
    }
    return false;
}

bool SolverImpl::precond_vcycle(int l, const cx<double>* b, cx<double>* x, hipStream_t s, bool x_swept,
                                cx<double>* zout, const cx<double>* zadd) {
    if (l == 0 && cap_buf && cap_n < cap_max) {
        const long long N = lev[0]->N;
        HH_HIP(hipMemcpyAsync(cap_buf + (size_t)cap_n * N, b, (size_t)N * sizeof(cx<double>), hipMemcpyDeviceToDevice,
                              s));
        ++cap_n;
    }
    if (o.precision == 0) return vcycle<double>(l, b, x, s, x_swept, zout, zadd);
    LevelDev& lv = *lev[l];
    // FP32 V-cycle: the entry level's own multigrid vectors carry the cast data
    launch_cast_d2f(lv.N, b, lv.b32.as<cx<float>>(), s);
    vcycle<float>(l, lv.b32.as<cx<float>>(), lv.x32.as<cx<float>>(), s);
    if (zadd) {
        launch_cast_f2d_add(lv.N, lv.x32.as<cx<float>>(), zadd, zout, s);
        return true;
    }
    launch_cast_f2d(lv.N, lv.x32.as<cx<float>>(), x, s);
    return false;
}

void SolverImpl::T_apply(int l, const cx<double>* v, cx<double>* z, hipStream_t s) {
    if (cex && l == 0) {
        const LevelDev& l0 = *lev[0];
        launch_fdm_solve(l0.n2, l0.n1, cexVx.as<double>(), cexVxT.as<double>(), cexVy.as<double>(), nullptr, v,
                         cexT1.as<cx<double>>(), cexT2.as<cx<double>>(), z, s, cexDinv.as<cx<double>>());
        return;
    }
    if (l >= defl_end()) {
        precond_vcycle(l, v, z, s);
        return;
    }
    LevelDev& lv = *lev[l];
    const int lnext = zadp ? Lz : l + 1;
    LevelDev& lc = *lev[lnext];
    const Transfer& tr = zadp ? ztr : lv.tr;
    launch_restrict<double>(tr, v, lc.tc.as<cx<double>>(), s);
    coarse_solve(lnext, lc.tc.as<cx<double>>(), lc.te.as<cx<double>>(), s);
    launch_prolong<double>(tr, lc.te.as<cx<double>>(), lv.tq.as<cx<double>>(), 0, s);
    // w = v - A q; with an FP64 V-cycle that starts with one Jacobi sweep on
    // separate kernels, the same kernel also forms that sweep (x = omega D^-1 w)
    const bool fuse = o.precision == 0 && o.nu_pre == 1 && !(cnn && l == 0) && l < tail_start && l < L;
    op<double>(l, MODE_RESID, false, lv.tq.as<cx<double>>(), v, lv.tw.as<cx<double>>(), s,
               fuse ? lv.ts.as<cx<double>>() : nullptr);
    // z = s + q, formed by the V-cycle's last step where it can (the last
    // smoothing sweep's epilogue, or the cast back from FP32)
    if (!precond_vcycle(l, lv.tw.as<cx<double>>(), lv.ts.as<cx<double>>(), s, fuse, z, lv.tq.as<cx<double>>()))
        launch_add(lv.N, lv.ts.as<cx<double>>(), lv.tq.as<cx<double>>(), z, s);
}

// One fused Arnoldi step on w = V[j+1]: a single workgroup for short vectors;
// otherwise a resident grid (or, for single solves, a cooperative one), or (in
// batched mode, when the grid is too large for up to 16 of them to be resident
// side by side) one kernel per Gram-Schmidt projection followed by the
// norm/Givens kernel and the scaling.
bool SolverImpl::arnoldi(long long N, int j, cx<double>* w, cx<double>* Vb, KrylovDev& k, hipStream_t s) {
    // MGS step j: v_0..v_j read once, w read and written once; j + 1 dots and
    // axpys, the norm and the scaling
    meter(16.0 * (j + 3) * N, 16.0 * (j + 1) * N + 6.0 * N);
    MeterScope quiet(nullptr);
    if (N <= kSmallArnoldi) {
        launch_arnoldi_small(N, j, w, Vb, N, k, s);
        return k.hstep != nullptr;
    }
    if (!grid_arnoldi_off && launch_arnoldi_grid(N, j, w, Vb, N, k, s, 4, allow_coop && !graphs_on(), o.ortho == 0))
        return k.hstep != nullptr;
    for (int i = 0; i <= j; ++i) launch_mgs(N, i, j, w, Vb, N, k, s);
    launch_norm_givens(N, j, w, Vb, N, k, s);
    launch_scale_by(N, w, w, &k.scal[1], s);
    return false;
}

// Substructured E^-1 (variable k): y_I = E_II^-1 c_I; x_S = S^-1 (c - E [y_I; 0])_S;
// x_I = E_II^-1 (c - E [0; x_S])_I.  xhat and xt are zero off the interior and
// separator entries (only those are ever written), so the level operator forms
// the off-diagonal products.
void SolverImpl::substruct_pass(const cx<double>* c, cx<double>* e, hipStream_t s) {
    SubstructE& E = *sub;
    const int* mp = E.map.as<int>();
    cx<double>* rp = E.rowpart.as<cx<double>>();
    cx<double>* cp = E.colpart.as<cx<double>>();
    cx<double>* xhat = E.xhat.as<cx<double>>();
    cx<double>* xt = E.xt.as<cx<double>>();
    cx<double>* rv = E.rvec.as<cx<double>>();
    // the tile launches are timing class 5 (the kernel that streams the stored factors)
    auto tiles = [&](const DevBuf& mats, int nmat, long long nt, int rows, const DevBuf& P, const cx<double>* x) {
        tstart(5, s);
        launch_symv_batch_tiles(mats.as<SymMat>(), nmat, nt, rows, P.as<double>(), mp, x, rp, cp, s);
        tstop(5, symv_batch_tile_bytes(nt), s);
    };
    tiles(E.subMats, E.nsub, E.sub_tiles, E.sub_rows, E.subP, c);
    launch_symv_batch_reduce(E.subMats.as<SymMat>(), E.nsub, E.sub_rows, mp, rp, cp, xhat, nullptr, s);
    op<double>(Lz, MODE_RESID, false, xhat, c, rv, s);
    tiles(E.SMats, 1, E.S_tiles, E.S_rows, E.SP, rv);
    launch_symv_batch_reduce(E.SMats.as<SymMat>(), 1, E.S_rows, mp, rp, cp, e, xt, s);
    op<double>(Lz, MODE_RESID, false, xt, c, rv, s);
    tiles(E.subMats, E.nsub, E.sub_tiles, E.sub_rows, E.subP, rv);
    launch_symv_batch_reduce(E.subMats.as<SymMat>(), E.nsub, E.sub_rows, mp, rp, cp, e, nullptr, s);
}

// One pass, then sub->refine steps of iterative refinement e += pass(c - E e).
void SolverImpl::substruct_apply(const cx<double>* c, cx<double>* e, hipStream_t s) {
    substruct_pass(c, e, s);
    SubstructE& E = *sub;
    const long long N = lev[Lz]->N;
    for (int i = 0; i < E.refine; ++i) {
        op<double>(Lz, MODE_RESID, false, e, c, E.rr.as<cx<double>>(), s);
        substruct_pass(E.rr.as<cx<double>>(), E.dd.as<cx<double>>(), s);
        launch_axpy<double>(N, E.dd.as<cx<double>>(), e, s);
    }
}

// Set-up check: ||c - E (E^-1 c)|| / ||c|| for a fixed pseudo-random c.
double SolverImpl::substruct_check(hipStream_t s) {
    const LevelDev& lz = *lev[Lz];
    std::vector<cx<double>> hc((size_t)lz.N), hr((size_t)lz.N);
    uint64_t st = 0x243F6A8885A308D3ull;
    auto uni = [&st]() {   // SplitMix64, top 53 bits, centred
        st += 0x9E3779B97F4A7C15ull;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * 0x1.0p-53 - 0.5;
    };
    for (auto& v : hc) v = {uni(), uni()};
    DevBuf dc, de, dr;
    upload(dc, hc);
    de.alloc((size_t)lz.N * 16);
    dr.alloc((size_t)lz.N * 16);
    substruct_apply(dc.as<cx<double>>(), de.as<cx<double>>(), s);
    op<double>(Lz, MODE_RESID, false, de.as<cx<double>>(), dc.as<cx<double>>(), dr.as<cx<double>>(), s);
    HH_HIP(hipMemcpyAsync(hr.data(), dr.p, hr.size() * 16, hipMemcpyDeviceToHost, s));
    HH_HIP(hipStreamSynchronize(s));
    double nc = 0.0, nr = 0.0;
    for (size_t i = 0; i < hc.size(); ++i) {
        nc += hc[i].re * hc[i].re + hc[i].im * hc[i].im;
        nr += hr[i].re * hr[i].re + hr[i].im * hr[i].im;
    }
    const double v = std::sqrt(nr / nc);
    return std::isfinite(v) ? v : 1e300;
}

void SolverImpl::coarse_solve(int l, const cx<double>* c, cx<double>* e, hipStream_t s) {
    if (l == Lz) {
        tstart(2, s);
        if (EinvC.p) {
            launch_gemv<cx<double>, double>(nZ, EinvC.as<cx<double>>(), c, e, s);
            tstop(2, 16.0 * nZ * (double)nZ + 32.0 * nZ, s);
        } else if (fdm && prob->dim == 3) {
            const LevelDev& lz = *lev[Lz];
            launch_fdm3_solve(lz.n3, lz.n2, lz.n1, fdmVx.as<double>(), fdmVxT.as<double>(), fdmVy.as<double>(),
                              fdmVyT.as<double>(), fdmVz.as<double>(), fdmVzT.as<double>(), fdmDinv.as<double>(), c,
                              fdmT1.as<cx<double>>(), fdmT2.as<cx<double>>(), e, s);
            // c, e, 1/D and the six eigenvector matrices once
            tstop(2, 40.0 * nZ + 16.0 * ((double)lz.n1 * lz.n1 + (double)lz.n2 * lz.n2 + (double)lz.n3 * lz.n3), s);
        } else if (fdm) {
            const LevelDev& lz = *lev[Lz];
            launch_fdm_solve(lz.n2, lz.n1, fdmVx.as<double>(), fdmVxT.as<double>(), fdmVy.as<double>(),
                             fdmDinv.as<double>(), c, fdmT1.as<cx<double>>(), fdmT2.as<cx<double>>(), e, s);
            // c, e, 1/D and both eigenvector matrices once
            tstop(2, 40.0 * nZ + 8.0 * ((double)lz.n1 * lz.n1 + (double)lz.n2 * lz.n2), s);
        } else if (sub) {
            substruct_apply(c, e, s);
            tstop(2, sub->bytes_per_apply(), s);
        } else {
            if (sym) {
                launch_symv(nZ, EinvP.as<double>(), c, symRow.as<cx<double>>(), symCol.as<cx<double>>(), e, s);
                // the stored triangle once, c and e
                tstop(2, 8.0 * 128.0 * 128.0 * (double)sym_tiles(nZ) + 32.0 * nZ, s);
            } else {
                launch_gemv_real(nZ, ldZ, Einv.as<double>(), c, e, s);
                tstop(2, 8.0 * nZ * (double)nZ + 32.0 * nZ, s);
            }
        }
        return;
    }
    LevelDev& lv = *lev[l];
    const long long N = lv.N;
    const int m = lv.m_inner;
    cx<double>* Vb = lv.V.as<cx<double>>();
    cx<double>* Zb = lv.Z.as<cx<double>>();
    KrylovDev& k = lv.kd;
    launch_norm_init(N, c, k, s);
    launch_scale_by(N, c, Vb, &k.scal[0], s);
    for (int j = 0; j < m; ++j) {
        cx<double>* vj = Vb + (size_t)j * N;
        cx<double>* zj = Zb + (size_t)j * N;
        cx<double>* w = Vb + (size_t)(j + 1) * N;
        T_apply(l, vj, zj, s);
        op<double>(l, MODE_APPLY, false, zj, nullptr, w, s);
        arnoldi(N, j, w, Vb, k, s);
    }
    launch_lsq(k, s);
    launch_update(N, Zb, N, k, e, 0, s);
}

// ------------------------------------------------------------- FGMRES ----
// Restarted FGMRES as a resumable state machine: every call of step() consumes
// the host copy of the scalars that earlier enqueued work produced (the norm of
// f, the cycle's starting residual, or one Arnoldi step's |g_{j+1}|), takes the
// decision the algorithm needs, and enqueues the next unit of work plus the
// device-to-host copy of its scalars.  Arnoldi steps run one ahead: step j + 1
// is enqueued before step j's scalars are read, so the device never waits for
// the host.  When step j ends the cycle, the step already enqueued after it
// only writes basis vector j + 2, Hessenberg column j + 1 and g[j + 1..j + 2],
// none of which the least-squares solve and update of the first j + 1 columns
// read (they take the column count from the host).  A batch of problems on
// several streams advances in lockstep, each waiting on its own event.
void SolveRun::mark(hipEvent_t e) {
    HH_HIP(hipEventRecord(e, s));
    waiting = e;
}

void SolveRun::start(SolverImpl* S_, const cx<double>* f_, cx<double>* u_, int use_u0_, hipStream_t s_) {
    S = S_;
    f = f_;
    u = u_;
    use_u0 = use_u0_;
    s = s_;
    t0 = std::chrono::steady_clock::now();
    S->ev_used = 0;
    S->ev_bytes = 0.0;
    S->ev_pending = -1;
    meter = Meter{};
    MeterScope ms(&meter);
    iters = cycles = j = m = 0;
    ahead = false;
    nf = stop = rn = gabs = 0.0;
    status = HH_OK;
    inf = hh_solve_info{};
    KrylovDev& kd = S->kd;
    const long long N = S->lev[0]->N;
    // a grid-exchange timeout of an earlier solve is reported there: this
    // solve starts with the flags of its Krylov states clear
    HH_HIP(hipMemsetAsync(&kd.ints[5], 0, sizeof(int), s));
    for (int l = 1; l < S->defl_end(); ++l)
        if (S->lev[l]->m_inner > 0) HH_HIP(hipMemsetAsync(&S->lev[l]->kd.ints[5], 0, sizeof(int), s));
    launch_dot_norm2(N, f, &kd.scal[3], &kd.ints[2], kd.partials, s);
    HH_HIP(hipMemcpyAsync(S->pin_d, kd.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    mark(S->ev_misc);
    phase = P_NF;
}

void SolveRun::enqueue_cycle_start() {
    KrylovDev& kd = S->kd;
    launch_norm_init(S->lev[0]->N, S->r.as<cx<double>>(), kd, s);
    HH_HIP(hipMemcpyAsync(S->pin_d, kd.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    mark(S->ev_misc);
    phase = P_RN;
}

void SolveRun::enqueue_step(int jj) {
    const Meter before = meter;
    KrylovDev& kd = S->kd;
    const long long N = S->lev[0]->N;
    cx<double>* Vb = S->V.as<cx<double>>();
    cx<double>* Zb = S->Z.as<cx<double>>();
    cx<double>* vj = Vb + (size_t)jj * N;
    cx<double>* zj = Zb + (size_t)jj * N;
    cx<double>* w = Vb + (size_t)(jj + 1) * N;
    const int slot = jj & 1;
    auto body = [&]() {
        S->T_apply(0, vj, zj, s);
        S->op<double>(0, MODE_APPLY, false, zj, nullptr, w, s);
        // MGS + norm + Givens + normalisation of w; algorithmic bytes: each basis
        // vector v_0..v_jj read once, w read once and written once
        S->tstart(3, s);
        const bool published = S->arnoldi(N, jj, w, Vb, kd, s);
        S->tstop(3, 16.0 * (jj + 3) * N, s);
        // the fused step kernels store |g_{j+1}| and the flags in the pinned slot
        // themselves; otherwise scal[0..7] and ints[0..5] (adjacent on the device)
        // are copied in one transfer
        if (!published)
            HH_HIP(hipMemcpyAsync(S->pin_step + 128 * slot, kd.scal, 8 * sizeof(double) + 6 * sizeof(int),
                                  hipMemcpyDeviceToHost, s));
    };
    if (S->graphs_on()) {
        // the step's launches depend on jj only (pointers into V and Z, the step
        // index); the Arnoldi kernels take their exchange tags from a device
        // counter, so a replayed graph is the same work as the launches
        if ((int)S->gexec.size() <= jj) {
            S->gexec.resize(jj + 1, nullptr);
            S->gbytes.resize(jj + 1, 0.0);
            S->gflops.resize(jj + 1, 0.0);
        }
        if (!S->gexec[jj]) {
            hipGraph_t g = nullptr;
            HH_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
            try {
                body();
            } catch (...) {
                (void)hipStreamEndCapture(s, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            HH_HIP(hipStreamEndCapture(s, &g));
            const hipError_t e = hipGraphInstantiate(&S->gexec[jj], g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HH_HIP(e);
            S->gbytes[jj] = meter.bytes - before.bytes;
            S->gflops[jj] = meter.flops - before.flops;
        } else {
            meter.bytes += S->gbytes[jj];
            meter.flops += S->gflops[jj];
        }
        HH_HIP(hipGraphLaunch(S->gexec[jj], s));
    } else {
        body();
    }
    HH_HIP(hipEventRecord(S->ev_slot[slot], s));
    step_bytes[slot] = meter.bytes - before.bytes;
    step_flops[slot] = meter.flops - before.flops;
}

void SolveRun::enqueue_final() {
    KrylovDev& kd = S->kd;
    for (int l = 1; l < S->defl_end() && l < 16; ++l)
        HH_HIP(hipMemcpyAsync(&S->pin_i[32 + l], &S->lev[l]->kd.ints[5], sizeof(int), hipMemcpyDeviceToHost, s));
    // the outer flag once more after the last step: a block that timed out in
    // the step's last exchange sets it after block 0 has published the step
    HH_HIP(hipMemcpyAsync(&S->pin_i[31], &kd.ints[5], sizeof(int), hipMemcpyDeviceToHost, s));
    launch_dot_norm2(S->lev[0]->N, S->r.as<cx<double>>(), &kd.scal[3], &kd.ints[2], kd.partials, s);
    HH_HIP(hipMemcpyAsync(S->pin_d, kd.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
    mark(S->ev_misc);
    phase = P_FINAL;
}

void SolveRun::step() {
    MeterScope ms(&meter);
    const long long N = S->lev[0]->N;
    const hh_solver_opts& o = S->o;
    cx<double>* rr = S->r.as<cx<double>>();
    KrylovDev& kd = S->kd;
    switch (phase) {
        case P_NF: {
            nf = std::sqrt(S->pin_d[3]);
            if (!std::isfinite(nf)) throw Err{HH_ENUMERIC, "right-hand side is not finite"};
            if (nf == 0.0) {
                launch_zero(N, u, s);
                inf.converged = 1;
                status = HH_OK;
                waiting = nullptr;
                phase = P_DONE;
                return;
            }
            stop = o.tol * nf;
            if (use_u0) {
                S->op<double>(0, MODE_RESID, false, u, f, rr, s);
            } else {
                launch_zero(N, u, s);
                launch_copy(N, f, rr, s);
            }
            enqueue_cycle_start();
            return;
        }
        case P_RN: {
            rn = S->pin_d[0];
            if (!std::isfinite(rn)) throw Err{HH_ENUMERIC, "residual is not finite"};
            if (rn <= stop || iters >= o.maxit) {
                enqueue_final();
                return;
            }
            m = std::min(S->m_outer, o.maxit - iters);
            launch_scale_by(N, rr, S->V.as<cx<double>>(), &kd.scal[0], s);
            j = 0;
            enqueue_step(0);
            ahead = (m > 1);
            if (ahead) enqueue_step(1);
            waiting = S->ev_slot[0];
            phase = P_STEP;
            return;
        }
        case P_STEP: {
            const int slot = j & 1;
            const double* pd = (const double*)(S->pin_step + 128 * slot);
            const int* pi = (const int*)(S->pin_step + 128 * slot + 8 * sizeof(double));
            gabs = pd[2];
            hist.push_back(gabs);
            ++iters;
            if (pi[5]) {
                exchange_timeout = true;
                throw Err{HH_EHIP, "grid barrier of the Arnoldi kernel timed out"};
            }
            if (!std::isfinite(gabs)) throw Err{HH_ENUMERIC, "Arnoldi recurrence produced NaN/Inf"};
            if (pi[1] || gabs <= stop || j + 1 >= m) {
                // end of the cycle: least squares, update, true residual on the
                // first j + 1 columns.  The step enqueued ahead (j + 1) is not
                // part of the method's work: its metered traffic is taken back.
                if (ahead) {
                    meter.bytes -= step_bytes[(j + 1) & 1];
                    meter.flops -= step_flops[(j + 1) & 1];
                }
                launch_lsq(kd, s, j + 1);
                launch_update(N, S->Z.as<cx<double>>(), N, kd, u, 1, s, j + 1);
                S->op<double>(0, MODE_RESID, false, u, f, rr, s);
                ++cycles;
                ahead = false;
                enqueue_cycle_start();
            } else {
                ++j;
                if (!ahead) enqueue_step(j);
                ahead = (j + 1 < m);
                if (ahead) enqueue_step(j + 1);
                waiting = S->ev_slot[j & 1];
            }
            return;
        }
        case P_FINAL: {
            exchange_timeout = S->pin_i[31] != 0;
            for (int l = 1; l < S->defl_end() && l < 16; ++l) exchange_timeout = exchange_timeout || S->pin_i[32 + l] != 0;
            if (exchange_timeout) throw Err{HH_EHIP, "grid barrier of an Arnoldi kernel timed out"};
            const double rtrue = std::sqrt(S->pin_d[3]);
            auto t1 = std::chrono::steady_clock::now();
            inf.iters = iters;
            inf.restarts = std::max(cycles - 1, 0);
            inf.relres_true = rtrue / nf;
            inf.relres_est = gabs / nf;
            inf.converged = (rtrue <= stop) ? 1 : 0;
            inf.t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
            int cnt = 0;
            inf.op_ms_total = S->tcollect(&cnt);
            inf.op_launches = cnt;
            inf.op_bytes_per_launch = cnt ? S->ev_bytes / cnt : 0.0;
            inf.model_bytes = meter.bytes;
            inf.model_flops = meter.flops;
            status = inf.converged ? HH_OK : HH_ENOCONV;
            waiting = nullptr;
            phase = P_DONE;
            return;
        }
        case P_DONE:
            return;
    }
}

// A grid-exchange timeout of the resident or cooperative Arnoldi kernels (the
// grid was not all resident, e.g. other streams held the CUs) ends the solve
// with HH_EHIP; from a zero initial guess the solve is then run once more with
// the per-projection kernels, which wait on no other workgroup.
int SolverImpl::solve(const cx<double>* f, cx<double>* u, int use_u0, hh_solve_info* info, hipStream_t s_caller) {
    // graphed solves run on the solver's own stream, after the caller's work
    hipStream_t s = s_caller;
    if (graphs_on()) {
        HH_HIP(hipEventRecord(gfork, s_caller));
        HH_HIP(hipStreamWaitEvent(gstream, gfork, 0));
        s = gstream;
    }
    for (int attempt = 0;; ++attempt) {
        SolveRun run;
        try {
            run.start(this, f, u, use_u0, s);
            while (run.phase != SolveRun::P_DONE) {
                HH_HIP(hipEventSynchronize(run.waiting));
                run.step();
            }
            HH_HIP(hipStreamSynchronize(s));
        } catch (const Err&) {
            if (!(run.exchange_timeout && attempt == 0 && !use_u0 && !grid_arnoldi_off)) throw;
            HH_HIP(hipStreamSynchronize(s));
            grid_arnoldi_off = true;
            drop_graphs();   // the steps now use the per-projection kernels
                    continue;
        }
        if (s != s_caller) {
            HH_HIP(hipEventRecord(gjoin, s));
            HH_HIP(hipStreamWaitEvent(s_caller, gjoin, 0));
        }
        run.inf.status = run.status;
        run.inf.arnoldi_fallback = attempt;
        last_hist.assign(run.hist.size(), 0.0);
        for (size_t i = 0; i < run.hist.size(); ++i) last_hist[i] = run.nf > 0.0 ? run.hist[i] / run.nf : 0.0;
        if (info) *info = run.inf;
        return run.status;
    }
}

void SolverImpl::set_spin_limit(int spins) {
    drop_graphs();   // the spin limit is a kernel argument
    kd.spin_limit = spins;
    for (auto& lv : lev) lv->kd.spin_limit = spins;
    grid_arnoldi_off = false;
}

template void SolverImpl::op<double>(int, int, bool, const cx<double>*, const cx<double>*, cx<double>*, hipStream_t,
                                     cx<double>*, const cx<double>*);
template void SolverImpl::op<float>(int, int, bool, const cx<float>*, const cx<float>*, cx<float>*, hipStream_t,
                                    cx<float>*, const cx<float>*);
template void SolverImpl::op_alpha<double>(int, int, double, double, const cx<double>*, const cx<double>*, cx<double>*,
                                           hipStream_t, cx<double>*, const cx<double>*, bool, bool);
template bool SolverImpl::vcycle<double>(int, const cx<double>*, cx<double>*, hipStream_t, bool, cx<double>*,
                                         const cx<double>*);
template bool SolverImpl::vcycle<float>(int, const cx<float>*, cx<float>*, hipStream_t, bool, cx<float>*,
                                        const cx<float>*);

}  // namespace hh
