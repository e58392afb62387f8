// Internal declarations of the isogeometric Helmholtz library (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hh.h"

namespace hh {

// ---------------------------------------------------------------- errors --
struct Err {
    int code;
    std::string msg;
};

void set_error(const std::string& msg);

#define HH_HIP(x)                                                                   \
    do {                                                                            \
        hipError_t e_ = (x);                                                        \
        if (e_ != hipSuccess)                                                       \
            throw ::hh::Err{HH_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define HH_REQUIRE(cond, msg)                                   \
    do {                                                        \
        if (!(cond)) throw ::hh::Err{HH_EINVAL, std::string(msg)}; \
    } while (0)

// --------------------------------------------------------------- complex --
template <class T>
struct cx {
    T re, im;
};

// Workgroups of a launch are dispatched to the eight XCDs (each with its own
// L2) in turn.  xcd_block maps workgroup b of nb to a logical block so that each
// XCD takes one contiguous range of logical blocks (a bijection of 0..nb-1): a
// stencil or transfer kernel then fetches each grid row and its halo into one
// L2 instead of several.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Algorithmic traffic and arithmetic of the work a solve enqueues: every
// launcher adds the bytes of its operands (each streamed once per kernel) and
// its flops (a complex x real multiply-add counts 4) to the meter installed on
// the calling thread, if any.  This is the model the whole-solve HBM fraction
// is measured against.
struct Meter {
    double bytes = 0.0, flops = 0.0;
};
extern thread_local Meter* g_meter;
inline void meter(double bytes, double flops) {
    if (g_meter) {
        g_meter->bytes += bytes;
        g_meter->flops += flops;
    }
}
struct MeterScope {
    Meter* prev;
    explicit MeterScope(Meter* m) : prev(g_meter) { g_meter = m; }
    ~MeterScope() { g_meter = prev; }
    MeterScope(const MeterScope&) = delete;
    MeterScope& operator=(const MeterScope&) = delete;
};

// Device buffer with owning semantics.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
        o.p = nullptr;
        o.bytes = 0;
    }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            bytes = o.bytes;
            o.p = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t n) {
        release();
        if (n == 0) return;
        if (hipMalloc(&p, n) != hipSuccess) {
            p = nullptr;
            throw Err{HH_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
        }
        bytes = n;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T* as() const { return static_cast<T*>(p); }
};

// Upload a host vector into a fresh device buffer (synchronous copy).
template <class T>
void upload(DevBuf& b, const std::vector<T>& h) {
    b.alloc(h.size() * sizeof(T));
    if (!h.empty()) HH_HIP(hipMemcpy(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

// ------------------------------------------------------------ host setup --
// One coordinate direction at one multigrid level.
struct Axis {
    int p = 0;          // degree (0 for the trivial second direction of 1D problems)
    int nel = 1;        // elements at this level
    int n = 1;          // interior unknowns
    int off = 0;        // Dirichlet shift: interior index = full index - off
    int nel_fine = 1;   // elements of the finest level (k^2 is piecewise on these)
    int level = 0;
    std::vector<double> bk;  // breakpoints
    std::vector<double> U;   // full open knot vector
    std::vector<double> Kb, Mb;  // interior bands [n][2p+1] (entry (i, i+d) at i*(2p+1)+d+p)
    std::vector<double> Me;      // element mass blocks [nel][(p+1)^2]
    std::vector<double> K0, M0;  // first element: function 0 against functions 0..p (Dirichlet lift)
    std::vector<double> G;       // mass blocks of this level's basis on every finest element
    // prolongation from the next-coarser level (this axis is the fine side):
    int pw = 1, rw = 1;          // row width (coarse entries per fine row), column width
    std::vector<int> prow0;      // per fine row: first coarse index
    std::vector<double> prow;    // per fine row: pw weights
    std::vector<int> pcol0;      // per coarse column: first fine index
    std::vector<double> pcol;    // per coarse column: rw weights
};

// ------------------------------------------------------------- host math --
// Visits the nonzero stencil entries of row I of level data (K entries from
// the bands; M_k entries from k^2 (constant) or the stored stencil S).
// Unit cube (constant k): the (2p+1)^3 entries of row I,
// K = Mz (x) My (x) Kx + Mz (x) Ky (x) Mx + Kz (x) My (x) Mx and M_k = k^2 Mz (x) My (x) Mx.
template <class F>
inline void visit_row3(const Axis& ax, const Axis& ay, const Axis& az, double k2c, long long I, F&& f) {
    const int px = ax.p, py = ay.p, pz = az.p, bx = 2 * px + 1, by = 2 * py + 1, bz = 2 * pz + 1;
    const int n1 = ax.n, n2 = ay.n, n3 = az.n;
    const int I1 = (int)(I % n1), I2 = (int)((I / n1) % n2), I3 = (int)(I / ((long long)n1 * n2));
    for (int d3 = -pz; d3 <= pz; ++d3) {
        const int J3 = I3 + d3;
        if (J3 < 0 || J3 >= n3) continue;
        const double mz = az.Mb[(size_t)I3 * bz + d3 + pz], kz = az.Kb[(size_t)I3 * bz + d3 + pz];
        for (int d2 = -py; d2 <= py; ++d2) {
            const int J2 = I2 + d2;
            if (J2 < 0 || J2 >= n2) continue;
            const double my = ay.Mb[(size_t)I2 * by + d2 + py], ky = ay.Kb[(size_t)I2 * by + d2 + py];
            for (int d1 = -px; d1 <= px; ++d1) {
                const int J1 = I1 + d1;
                if (J1 < 0 || J1 >= n1) continue;
                const double mx = ax.Mb[(size_t)I1 * bx + d1 + px], kx = ax.Kb[(size_t)I1 * bx + d1 + px];
                const double kv = mz * (my * kx + ky * mx) + kz * my * mx;
                f(((long long)J3 * n2 + J2) * n1 + J1, kv, k2c * mz * my * mx);
            }
        }
    }
}

template <class F>
inline void visit_row(const Axis& ax, const Axis& ay, bool const_k, double k2c, const std::vector<double>& S,
                      long long I, F&& f) {
    const int px = ax.p, py = ay.p, bx = 2 * px + 1, by = 2 * py + 1;
    const int n1 = ax.n, n2 = ay.n;
    const long long N = (long long)n1 * n2;
    const int I1 = (int)(I % n1), I2 = (int)(I / n1);
    for (int d2 = -py; d2 <= py; ++d2) {
        const int J2 = I2 + d2;
        if (J2 < 0 || J2 >= n2) continue;
        const double my = ay.Mb[(size_t)I2 * by + d2 + py], ky = ay.Kb[(size_t)I2 * by + d2 + py];
        for (int d1 = -px; d1 <= px; ++d1) {
            const int J1 = I1 + d1;
            if (J1 < 0 || J1 >= n1) continue;
            const double mxv = ax.Mb[(size_t)I1 * bx + d1 + px], kxv = ax.Kb[(size_t)I1 * bx + d1 + px];
            const double kv = my * kxv + ky * mxv;
            const double mv = const_k ? k2c * my * mxv : S[(size_t)((d2 + py) * bx + d1 + px) * N + I];
            f((long long)J2 * n1 + J1, kv, mv);
        }
    }
}

// Host-side builders (setup.cpp).
void gauss_legendre(int n, double* x, double* w);
// keep_last: only the first function is eliminated (radiation condition at the right end)
// len: the direction's extent (breakpoints len * i / nel_fine)
Axis make_axis(int p, int nel_fine, int level, bool keep_last = false, double len = 1.0);
Axis make_trivial_axis();
void make_transfer(Axis& fine, const Axis& coarse);
// ADP deflation vectors along one direction (zf: their tables on the fine
// side, coarse: the pseudo-axis of Z^T K Z and Z^T M Z), and the coarse stencil
// Z^T S Z of a full fine-level stencil S.
void make_adp(const Axis& fine, double eps, Axis& zf, Axis& coarse);
void galerkin_stencil_z(const Axis& ax, const Axis& ay, const std::vector<double>& S, const Axis& zfx,
                        const Axis& zfy, const Axis& cxa, const Axis& cya, std::vector<double>& Sc);
// Element-wise k^2-weighted Galerkin mass of `level` as a full stencil, SoA
// [(2px+1)(2py+1)][N] (k2: finest-element k^2, [nel_fine_y][nel_fine_x]).
// Coarse-level k^2 as the mean of the children, and the mass rediscretised
// with it (mg_coarse = REDISC_AVG).
void coarse_k2_mean(const std::vector<double>& k2, int nx, int ny, int ncx, int ncy, std::vector<double>& out);
void redisc_mass_stencil(const Axis& ax, const Axis& ay, const std::vector<double>& k2l, std::vector<double>& S);
void galerkin_mass_stencil(const Axis& ax, const Axis& ay, const std::vector<double>& k2,
                           std::vector<double>& S);
void basis_values(const std::vector<double>& U, int p, int span, double x, double* N, double* dN);
// K V = M V diag(lam), V^T M V = I for one axis (V row-major [unknown][mode]).
void axis_eigen(const Axis& a, std::vector<double>& V, std::vector<double>& lam);

// ------------------------------------------------------ device-side data --
enum OpKind { KIND_SEP = 0, KIND_VARFINE = 1, KIND_STENCIL = 2 };
// Levels up to this many unknowns (constant k or stored stencil, 2D) use the
// one-thread-per-unknown operator kernel instead of the strip kernel; measured
// on MP 2-A (levels of 25,921 / 6,561 / 1,681 unknowns): 5.78 ms per solve with
// this bound, 5.93 ms with 16384, 6.03 ms with the strip kernel only.
constexpr long long kOpDirectMax = 32768;
// 2D stored-stencil levels from this many unknowns use the tiled kernel (its
// coefficient loads are all in flight before use; the one-thread-per-unknown
// kernel leaves most of the device idle on such levels)
constexpr long long kStencilTiledMin = 2048;

enum OpMode { MODE_APPLY = 0, MODE_RESID = 1, MODE_SMOOTH = 2 };

// Arguments of the level-operator kernels: y = K x - alpha M_k x (+ epilogue).
template <class T>
struct OpArgs {
    int n1, n2;
    const double* Kx;
    const double* Mx;
    const double* Ky;
    const double* My;
    double k2c;            // KIND_SEP: constant k^2
    const double* k2;      // KIND_VARFINE: finest-element k^2 [nel2][nel1]
    int nel1, nel2, off1, off2;
    const double* Mex;     // KIND_VARFINE: element mass [nel1][(px+1)^2]
    const double* Mey;     // [nel2][(py+1)^2]
    const T* S;            // KIND_STENCIL: [(2px+1)(2py+1)][n1*n2]
    T are, aim;            // alpha
    int ty;                // strip height of the kernel (0: fixed rule)
    const cx<T>* x;
    const cx<T>* b;
    cx<T>* y;
    const cx<T>* dinv;
    T omega;
    cx<T>* xo;             // MODE_RESID: if set, also xo = omega D^-1 y (a first sweep on y)
    const cx<T>* yadd;     // MODE_SMOOTH: if set, y = the swept x + yadd
    // radiation condition: y[bnd_I] += i bnd_im x[bnd_I] (bnd_I < 0: none)
    long long bnd_I;
    T bnd_im;
    // unit cube (constant k): n3 >= 1 slices in z with bands Kz, Mz; 0 for 1D / 2D
    int n3;
    const double* Kz;
    const double* Mz;
};

struct Transfer {
    int nf1, nf2, nc1, nc2;
    int pw1, pw2, rw1, rw2;
    const int* prow0x;
    const double* prowx;
    const int* prow0y;
    const double* prowy;
    const int* pcol0x;
    const double* pcolx;
    const int* pcol0y;
    const double* pcoly;
    // unit cube: the z factor of P = P_z (x) P_y (x) P_x; nf3 = 0 for 1D / 2D
    int nf3, nc3, pw3, rw3;
    const int* prow0z;
    const double* prowz;
    const int* pcol0z;
    const double* pcolz;
    // unit cube: the two intermediate grids of the one-direction passes,
    // nf3 x nf2 x nc1 and nf3 x nc2 x nc1 entries, per precision
    cx<double>* tmpa64;
    cx<double>* tmpb64;
    cx<float>* tmpa32;
    cx<float>* tmpb32;
};

// State of one FGMRES instance (device memory), m = max Arnoldi steps.
struct KrylovDev {
    cx<double>* H;    // (m+1) x m, column j at H + j*(m+1)
    double* cs;       // m
    cx<double>* sn;   // m
    cx<double>* g;    // m+1
    cx<double>* y;    // m
    double* scal;     // [0] beta, [1] hn, [2] |g_{j+1}|, [3] norm accumulator
    int* ints;        // [0] jdone, [1] breakdown flag, [2] reduction counter,
                      // [5] grid-exchange timeout flag, [6] cooperative launch epoch,
                      // [7] epoch of the last full write of vslots
    cx<double>* partials;  // reduction partials (2 x 1024, double-buffered)
    unsigned long long* slots;  // grid-exchange words of the cooperative Arnoldi kernels (2 x 256 x 4)
    cx<double>* gram;           // one-reduction Arnoldi (m <= kOneRedMaxM only, else null): rows 1..m-1
                                // of the strictly lower part of V^H V, row i packed at i(i-1)/2
    unsigned long long* vslots; // its vector-exchange words: [block][qcap][4]
    int qcap;                   // 2m - 1 values per block (0 when not allocated)
    unsigned char* hstep;       // outer solve: device address of the pinned step slots (2 x 128 B), else null
    int m;
    int spin_limit;             // polls before a grid-exchange wait gives up and sets ints[5]
};

// Polls of a grid-exchange wait before it gives up (about a second of sleeps).
constexpr int kSpinLimit = 1 << 20;

// Longest outer restart (Krylov basis length) the solver accepts.
constexpr int kMaxRestart = 200;
// One-reduction Arnoldi: restart lengths and grid sizes it serves.
constexpr int kOneRedMaxM = 50;
constexpr int kOneRedMaxBlocks = 64;

// Coarse tail of the V-cycle run by one workgroup with its level vectors in
// LDS (all levels from some l0 to the coarsest are small): per-level data,
// filled once at setup and kept in device memory.
constexpr int kTailLevels = 16;
template <class T>
struct TailLevel {
    int n1, n2, px, py, kind;     // kind: KIND_SEP or KIND_STENCIL
    T omega;
    const double* Kx;
    const double* Mx;
    const double* Ky;
    const double* My;
    const T* S;                   // KIND_STENCIL: [(2px+1)(2py+1)][N]
    const cx<T>* dinv;
    cx<T>* b;                     // this level's right-hand side / iterate / residual / spare
    cx<T>* x;
    cx<T>* r;
    cx<T>* t;
    Transfer tr;                  // to the next-coarser level
    // LDS byte offsets of this level's coefficient tables (copied at kernel
    // start): bands Kx, Mx [n1][2px+1], Ky, My [n2][2py+1], and the transfer
    // tables to the next-coarser level (-1 at the coarsest level)
    int o_kx, o_mx, o_ky, o_my;
    int o_prow0x, o_prowx, o_prow0y, o_prowy, o_pcol0x, o_pcolx, o_pcol0y, o_pcoly;
};
template <class T>
struct TailDesc {
    int L, nL, nu_pre, nu_post;
    T are, aim;                   // M_beta = K - (are + i aim) M_k
    double k2c;                   // constant k^2 (KIND_SEP)
    const cx<T>* Minv;            // dense inverse of M_beta at level L
    int lds_bytes;                // LDS of the tail from level lds_l0 on
    int lds_l0;
    int img16;                    // coefficient image size in 16-byte units (LDS bytes [0, 16 img16))
    int o_minv;                   // LDS offset of the transposed coarsest inverse (-1: read from Minv)
    int offb[kTailLevels], offx[kTailLevels], offt[kTailLevels];  // byte offsets of b, x, t in LDS
    TailLevel<T> lv[kTailLevels];
};

// Kernel launchers (kernels.hip; op_p<degree>.hip for the level operator).
template <int P, class T>
void launch_op_deg(int kind, int mode, int py, const OpArgs<T>& a, hipStream_t s);
template <class T>
void launch_op(int kind, int mode, int px, int py, const OpArgs<T>& a, hipStream_t s);
template <class T>
void launch_restrict(const Transfer& t, const cx<T>* r, cx<T>* c, hipStream_t s, const cx<T>* dinv = nullptr,
                     T omega = T(0), cx<T>* xs = nullptr);   // dinv: also xs = omega D^-1 c
template <class T>
void launch_prolong(const Transfer& t, const cx<T>* e, cx<T>* x, int add, hipStream_t s);
template <class T>   // xout = xin + P e (xin may alias xout)
void launch_prolong_add(const Transfer& t, const cx<T>* e, const cx<T>* xin, cx<T>* xout, hipStream_t s);
template <class T>
void launch_jacobi0(long long N, const cx<T>* dinv, T omega, const cx<T>* b, cx<T>* x, hipStream_t s);
template <class T>
void launch_axpy(long long N, const cx<T>* x, cx<T>* y, hipStream_t s);           // y += x
void launch_add(long long N, const cx<double>* a, const cx<double>* b, cx<double>* y, hipStream_t s);
void launch_copy(long long N, const cx<double>* x, cx<double>* y, hipStream_t s);
void launch_zero(long long N, cx<double>* y, hipStream_t s);
void launch_cast_d2f(long long N, const cx<double>* x, cx<float>* y, hipStream_t s);
void launch_cast_f2d(long long N, const cx<float>* x, cx<double>* y, hipStream_t s);
void launch_cast_f2d_add(long long N, const cx<float>* x, const cx<double>* q, cx<double>* y,
                         hipStream_t s);   // y = x + q
template <class TM, class TV>
void launch_gemv(int n, const TM* A, const cx<TV>* x, cx<TV>* y, hipStream_t s);
// y = A x for a real n x n matrix with leading dimension ld (even ld: 16-byte rows)
void launch_gemv_real(int n, long long ld, const double* A, const cx<double>* x, cx<double>* y, hipStream_t s);
// symmetric dense matrix as packed upper-triangle 128 x 128 tiles
long long sym_tiles(int n);
long long sym_packed_doubles(int n);
void launch_sym_pack(int n, long long ld, const double* D, double* P, hipStream_t s);
// y = P x (P packed symmetric; rowpart, colpart: sym_tiles(n) * 128 complex scratch each)
void launch_symv(int n, const double* P, const cx<double>* x, cx<double>* rowpart, cx<double>* colpart,
                 cx<double>* y, hipStream_t s);
void launch_scatter(long long n, const long long* idx, const double* val, double* y, hipStream_t s);
void launch_set_identity(int n, long long ld, double* a, hipStream_t s);   // a: n x n zeros -> identity
// x = V-cycle(b) from level l0 through the coarsest level in one workgroup
// (lds_bytes: dynamic LDS of the level vectors; tail_prepare allows that size)
template <class T>
void tail_prepare(int lds_bytes);
template <class T>
void launch_vcycle_tail(const TailDesc<T>* desc, const void* img, int img16, const cx<T>* minv, int P, int l0,
                        int lds_bytes, const cx<T>* b, cx<T>* x,
                        hipStream_t s);   // P: degree of 2D levels (unrolled form), 0: any
// Unit cube (constant k): level operator, transfers and the fast-diagonalisation
// E^-1 (op3d.hip).  launch_op, launch_restrict and launch_prolong_add hand
// levels with a.n3 > 0 / t.nf3 > 0 to these.
template <class T>
void launch_op3d(int mode, int p, const OpArgs<T>& a, hipStream_t s);
template <class T>
void launch_restrict3(const Transfer& t, const cx<T>* r, cx<T>* c, hipStream_t s, const cx<T>* dinv, T omega,
                      cx<T>* xs);
template <class T>
void launch_prolong_add3(const Transfer& t, const cx<T>* e, const cx<T>* xin, cx<T>* xout, hipStream_t s);
// e = V diag(dinv) V^T c, V = Vz (x) Vy (x) Vx on an [n3][n2][n1] grid (VdT: V_d transposed,
// all row-major; t1, t2: N-vector scratch)
void launch_fdm3_solve(int n3, int n2, int n1, const double* Vx, const double* VxT, const double* Vy,
                       const double* VyT, const double* Vz, const double* VzT, const double* dinv,
                       const cx<double>* c, cx<double>* t1, cx<double>* t2, cx<double>* e, hipStream_t s);
// e = (Vy (x) Vx) diag(dinv) (Vy (x) Vx)^T c on an [n2][n1] grid (t1, t2: N-vector scratch);
// with cdinv the diagonal is complex (cdinv used, dinv ignored)
void launch_fdm_solve(int n2, int n1, const double* Vx, const double* VxT, const double* Vy, const double* dinv,
                      const cx<double>* c, cx<double>* t1, cx<double>* t2, cx<double>* e, hipStream_t s,
                      const cx<double>* cdinv = nullptr);
// Krylov kernels
int reduction_blocks(long long N);
void launch_norm_init(long long N, const cx<double>* r, KrylovDev& k, hipStream_t s);  // beta = ||r||, g = [beta,0..], state reset
void launch_scale_by(long long N, const cx<double>* x, cx<double>* y, const double* by, hipStream_t s);  // y = x / *by (0 -> 0)
void launch_mgs(long long N, int i, int j, cx<double>* w, const cx<double>* V, long long ldv,
                KrylovDev& k, hipStream_t s);
void launch_norm_givens(long long N, int j, cx<double>* w, const cx<double>* V, long long ldv,
                        KrylovDev& k, hipStream_t s);
void launch_lsq(KrylovDev& k, hipStream_t s, int ncols = -1);
// fused Arnoldi step (MGS + norm + Givens + normalise): one workgroup for short
// vectors, otherwise a grid of resident workgroups (launch_arnoldi_grid: false
// when neither a resident launch fits `concurrent` grids nor coop_ok allows a
// cooperative one; the caller then runs one kernel per projection).  With
// one_reduce, a grid the one-reduction kernel serves (k.qcap > 0, at most
// kOneRedMaxBlocks workgroups, resident) takes that form.
constexpr long long kSmallArnoldi = 4096;
bool launch_arnoldi_grid(long long N, int j, cx<double>* w, const cx<double>* V, long long ldv, KrylovDev& k,
                         hipStream_t s, int concurrent, bool coop_ok, bool one_reduce);
void launch_arnoldi_small(long long N, int j, cx<double>* w, const cx<double>* V, long long ldv,
                          KrylovDev& k, hipStream_t s);
void launch_update(long long N, const cx<double>* Z, long long ldz, KrylovDev& k, cx<double>* u,
                   int accumulate, hipStream_t s, int ncols = -1);
void launch_dot_norm2(long long N, const cx<double>* x, double* out, int* counter, cx<double>* partials,
                      hipStream_t s);

}  // namespace hh
