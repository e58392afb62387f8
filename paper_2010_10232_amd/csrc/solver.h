// Solver objects behind the C ABI.
#pragma once

#include <chrono>
#include <memory>

#include "cnn.h"
#include "hh_internal.h"
#include "substruct.h"

namespace hh {

struct ProblemImpl {
    int dim = 2, p = 3, nel[3] = {1, 1, 1};
    double len[3] = {1.0, 1.0, 1.0};   // domain extent per direction
    int k_mode = 0;
    double k = 0.0;
    bool somm = false;        // radiation condition at x = 1 (1D, constant k; MP 1-A)
    std::vector<double> k2;   // k^2 per finest element [nel_y][nel_x] (1D: [1][nel_x])
    mutable DevBuf k2_dev;    // the same on the device (uploaded by hh_assemble on its stream, else by hh_setup)
    Axis ax0, ay0, az0;       // finest-level axes (az0 trivial unless dim == 3)
    long long N() const { return (long long)ax0.n * ay0.n * az0.n; }
};

struct LevelDev {
    Axis ax, ay, az;          // az: trivial unless dim == 3
    int n1 = 1, n2 = 1, n3 = 1;
    long long N = 1;
    double omega = 0.8, gersh = 0.0;
    int kind = KIND_SEP;
    // radiation condition: the boundary term i bnd_im x on unknown bnd_I (-1: none)
    long long bnd_I = -1;
    double bnd_im = 0.0;
    int ty64 = 0, ty32 = 0;   // level-operator strip height (0: fixed rule), FP64 / FP32
    DevBuf Kx, Mx, Ky, My, Kz, Mz;
    DevBuf S64, S32;
    DevBuf S64a;              // Galerkin stencil of A_l when the multigrid one is rediscretised
    DevBuf k2, Mex, Mey;
    DevBuf Dinv64, Dinv32;
    // transfer to the next-coarser level (this level = fine side)
    DevBuf prow0x, prowx, pcol0x, pcolx, prow0y, prowy, pcol0y, pcoly;
    DevBuf prow0z, prowz, pcol0z, pcolz;
    DevBuf tra64, trb64, tra32, trb32;   // unit cube: intermediate grids of the transfer passes
    Transfer tr{};
    // multigrid work vectors
    DevBuf b64, x64, r64, t64, vr64, vx64;
    DevBuf b32, x32, r32, t32, vr32, vx32;
    // deflation work vectors (FP64)
    DevBuf tc, te, tq, tw, ts;
    // inner FGMRES (iterative deflation level)
    int m_inner = 0;
    DevBuf V, Z, kstate;
    KrylovDev kd{};
};

struct SolverImpl;

// One FGMRES solve as a resumable state machine (see solver.hip).
struct SolveRun {
    enum Phase { P_NF, P_RN, P_STEP, P_FINAL, P_DONE };
    SolverImpl* S = nullptr;
    const cx<double>* f = nullptr;
    cx<double>* u = nullptr;
    int use_u0 = 0;
    hipStream_t s = nullptr;
    Phase phase = P_DONE;
    double nf = 0, stop = 0, rn = 0, gabs = 0;
    int iters = 0, cycles = 0, j = 0, m = 0, status = 0;
    bool ahead = false;             // Arnoldi step j + 1 is already enqueued
    hipEvent_t waiting = nullptr;   // completes when the scalars step() reads are on the host
    bool exchange_timeout = false;  // the error thrown was a grid-exchange timeout
    Meter meter;                    // algorithmic bytes / flops of the work this solve used
    double step_bytes[2] = {0, 0}, step_flops[2] = {0, 0};   // per Arnoldi-step slot
    std::vector<double> hist;       // |g_{j+1}| of every Arnoldi step, in order
    hh_solve_info inf{};
    std::chrono::steady_clock::time_point t0;
    void start(SolverImpl* S, const cx<double>* f, cx<double>* u, int use_u0, hipStream_t s);
    void step();
    void enqueue_cycle_start();
    void enqueue_step(int jj);
    void enqueue_final();
    void mark(hipEvent_t e);
};

struct SolverImpl {
    const ProblemImpl* prob = nullptr;
    hh_solver_opts o{};
    int L = 0;      // coarsest multigrid level
    int Lz = 0;     // deflation level solved directly (0: none)
    // ADP deflation vectors (defl_z = 1): two-level, the deflation level is
    // lev[Lz], Lz = L + 1, outside the multigrid hierarchy; ztr maps level 0 to it
    bool zadp = false;
    Transfer ztr{};
    DevBuf zprow0x, zprowx, zpcol0x, zpcolx, zprow0y, zprowy, zpcol0y, zpcoly;
    DevBuf zprow0z, zprowz, zpcol0z, zpcolz, ztra64, ztrb64;   // unit cube
    // C_ex (precond = 1): exact inverse of K - (1 + i beta2) M_k on the finest
    // level by fast diagonalisation (eigenvectors of level 0, complex 1 / D)
    bool cex = false;
    double cex_b2 = 0.0;
    DevBuf cexVx, cexVxT, cexVy, cexDinv, cexT1, cexT2;
    // levels l < defl_end() are deflated (a deflation level lies below them);
    // 1 .. defl_end() - 1 are the inner FGMRES levels
    int defl_end() const { return zadp ? 1 : Lz; }
    std::vector<std::unique_ptr<LevelDev>> lev;
    DevBuf Minv64, Minv32;   // dense inverse of M_beta at level L (complex)
    DevBuf Einv;             // dense inverse of A at level Lz (real; variable k)
    DevBuf EinvC;            // dense inverse of the complex E (radiation condition), row-major
    // constant k: E^-1 at level Lz by fast diagonalisation (1D eigenvectors and 1 / D)
    bool fdm = false;
    DevBuf fdmVx, fdmVxT, fdmVy, fdmDinv, fdmT1, fdmT2;
    DevBuf fdmVyT, fdmVz, fdmVzT;   // unit cube: the y and z factors of the same form
    // levels >= tail_start (all small) run their V-cycle in one workgroup
    int tail_start = 1 << 30;
    int tail_lds = 0, tail_lds32 = 0;   // dynamic LDS bytes (FP64 / FP32 tail)
    DevBuf tail64, tail32;              // TailDesc<double>, TailDesc<float>
    DevBuf tail_img;                    // the tail's coefficient tables in their LDS layout
    int tail_P = 0;                     // degree of the tail's unrolled form (2D), 0: loop form
    int nL = 0, nZ = 0;
    long long ldZ = 0;       // leading dimension of Einv (even, >= nZ)
    // variable k, nZ >= 2048: E^-1 kept as its packed upper triangle (symmetric)
    bool sym = false;
    DevBuf EinvP, symRow, symCol;
    // variable k, substructured E^-1 (separator Schur complement)
    std::unique_ptr<SubstructE> sub;
    void substruct_pass(const cx<double>* c, cx<double>* e, hipStream_t s);
    void substruct_apply(const cx<double>* c, cx<double>* e, hipStream_t s);
    double substruct_check(hipStream_t s);
    // outer FGMRES
    int m_outer = 0;
    DevBuf V, Z, kstate, r, scratch;
    KrylovDev kd{};
    // pinned host copies of device scalars: two slots (Arnoldi steps alternate)
    // of 8 doubles / 16 ints; inner-level barrier flags at pin_i[32 + l]
    double* pin_d = nullptr;
    int* pin_i = nullptr;
    // per Arnoldi-step slot: the device scalars (8 doubles) and, right after
    // them in device memory, the counters (6 ints), copied in one transfer
    unsigned char* pin_step = nullptr;   // 2 slots x 128 bytes
    hipEvent_t ev_slot[2] = {nullptr, nullptr}, ev_misc = nullptr;
    // event timing of one kernel class (non-blocking: events are read after the solve)
    std::vector<hipEvent_t> evpool;
    int ev_used = 0;
    double ev_bytes = 0.0;
    int ev_pending = -1;
    void tstart(int cls, hipStream_t s);
    void tstop(int cls, double bytes, hipStream_t s);
    double tcollect(int* count);
    ~SolverImpl();

    void setup(hipStream_t s);
    void setup_levels_3d(hipStream_t s);   // unit cube: levels, transfers, coarsest inverse, E^-1
    void setup_finish(hipStream_t s);      // deflation, Krylov and host-side state (every dimension)
    void autotune_ops(hipStream_t s);
    // building blocks
    template <class T>
    void op(int l, int mode, bool cslp, const cx<T>* x, const cx<T>* b, cx<T>* y, hipStream_t s,
            cx<T>* xo = nullptr,            // xo: MODE_RESID also forms a first sweep on y
            const cx<T>* yadd = nullptr);   // yadd: MODE_SMOOTH writes the swept x + yadd
    // x_swept: x already holds the first sweep from zero.  zadd (with zout):
    // the last smoothing sweep writes zout = x + zadd instead of x, when the
    // cycle ends with such a sweep (the return value says whether it did).
    template <class T>
    bool vcycle_once(int l, const cx<T>* b, cx<T>* x, hipStream_t s, bool x_swept = false, cx<T>* zout = nullptr,
                     const cx<T>* zadd = nullptr);
    template <class T>
    bool vcycle(int l, const cx<T>* b, cx<T>* x, hipStream_t s, bool x_swept = false, cx<T>* zout = nullptr,
                const cx<T>* zadd = nullptr);
    bool precond_vcycle(int l, const cx<double>* b, cx<double>* x, hipStream_t s, bool x_swept = false,
                        cx<double>* zout = nullptr, const cx<double>* zadd = nullptr);
    void T_apply(int l, const cx<double>* v, cx<double>* z, hipStream_t s);
    void coarse_solve(int l, const cx<double>* c, cx<double>* e, hipStream_t s);
    // true when the step's kernel stored the host's scalars in the pinned slot itself
    bool arnoldi(long long N, int j, cx<double>* w, cx<double>* Vb, KrylovDev& k, hipStream_t s);
    bool allow_coop = true;
    bool in_batch = false;   // set by the batched solve: steps launched one by one
    // step graphs (use_graph): one executable graph per outer step index, its
    // metered work, and the stream the graphed solves run on
    hipStream_t gstream = nullptr;
    hipEvent_t gfork = nullptr, gjoin = nullptr;
    std::vector<hipGraphExec_t> gexec;
    std::vector<double> gbytes, gflops;
    bool graphs_on() const { return o.use_graph && !o.time_kernels && !cap_buf && !in_batch; }
    // forget the captured steps (the kernel sequence or its arguments changed)
    void drop_graphs() {
        for (hipGraphExec_t& g : gexec)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
    // set after a grid-exchange timeout: Arnoldi steps use the per-projection
    // kernels (no wait on other workgroups) from then on
    bool grid_arnoldi_off = false;
    void set_spin_limit(int spins);
    // learned fine-level smoother (null: damped Jacobi everywhere)
    CnnImpl* cnn = nullptr;
    DevBuf feat;                 // network feature c = k^2 h^2 per finest-level unknown (FP32)
    // capture of finest-level V-cycle inputs (training samples)
    cx<double>* cap_buf = nullptr;
    int cap_max = 0, cap_n = 0;
    // mg: the multigrid operator (rediscretised under mg_coarse = 1), else the
    // deflation operator A_l; mass_only: y = -alpha M_k x (zero stiffness bands)
    template <class T>
    void op_alpha(int l, int mode, double are, double aim, const cx<T>* x, const cx<T>* b, cx<T>* y, hipStream_t s,
                  cx<T>* xo = nullptr, const cx<T>* yadd = nullptr, bool mg = true, bool mass_only = false);
    DevBuf zero_bands;           // zero band table of the widest level (mass-only applies)
    int solve(const cx<double>* f, cx<double>* u, int use_u0, hh_solve_info* info, hipStream_t s);
    // the last completed solve's estimated relative residuals |g_{j+1}| / ||f||, one per step
    std::vector<double> last_hist;
};

ProblemImpl* build_problem(const hh_problem_desc* d);

// f = amp * Phi(x0) on the device (rhs.hip): staging allocated per call, or
// the fixed staging array (no allocation).
void rhs_point_source(const ProblemImpl& P, const double* x0, double amp, cx<double>* f, hipStream_t s);
void rhs_point_source_noalloc(const ProblemImpl& P, const double* x0, double amp, cx<double>* f, hipStream_t s);
// f = -u0 (K - k^2 M)_{:,0} (MP 1-A: the boundary value at x = 0 moved to the right-hand side)
void rhs_dirichlet_lift(const ProblemImpl& P, double u0, cx<double>* f, hipStream_t s);

}  // namespace hh

struct hh_problem {
    hh::ProblemImpl impl;
};
struct hh_solver {
    std::unique_ptr<hh::SolverImpl> impl;
};
struct hh_cnn {
    std::unique_ptr<hh::CnnImpl> impl;
};
