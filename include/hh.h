/*
 * hh.h - C ABI of the MI355X (gfx950) isogeometric Helmholtz solver.
 *
 * Solves A u = f for the B-spline Galerkin discretisation of
 *     -Lap u - k^2 u = f  on (0,1)^d, d = 1, 2 or 3 (or a box (0,L_1) x ... x (0,L_d)),
 *     u = 0 on the boundary
 * (the model problems MP 1-B, MP 2-A and MP 2-B, section 2 of Dwarka, Tielen,
 * Moeller and Vuik, "Towards accuracy and scalability: combining isogeometric
 * analysis with deflation ...").  A = K - M_k with K the stiffness matrix and
 * M_k the k^2-weighted mass matrix of section 2.3; A is real symmetric and
 * indefinite.  The solver is restarted flexible GMRES, right-preconditioned by
 * the deflated complex shifted Laplacian of section 3: multigrid V-cycles with
 * damped Jacobi smoothing on M_beta = K - (beta1 + i beta2) M_k, and the
 * deflation Q = Z E^-1 Z^T, E = Z^T A Z, with Z the knot-insertion prolongation.
 *
 * Conventions
 *  - Vectors are complex double (interleaved re, im; 16 bytes per entry) in
 *    DEVICE memory owned by the caller, indexed (i3 * n2 + i2) * n1 + i1 over
 *    interior control points (x fastest; 1D uses n2 = n3 = 1, 2D n3 = 1).
 *    n_d = n_el_d + p - 2 at the finest level; coarse levels are reported by
 *    hh_level_info.
 *  - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *    Calls enqueue on that stream; hh_solve, hh_setup and hh_assemble return
 *    after the stream has drained.
 *  - Every entry point returns an hh_status.  Errors are negative and leave
 *    the objects unchanged; hh_last_error() gives a thread-local message.
 *    No C++ exception crosses this interface.
 *  - Objects are not thread-safe; one object may be used by one thread at a
 *    time.  Calls on different solvers may run concurrently on different
 *    streams.
 */
#ifndef HH_H
#define HH_H

#ifdef __cplusplus
extern "C" {
#endif

typedef int hh_status;
#define HH_OK 0
#define HH_ENOCONV 1       /* warning: maxit reached; the best iterate is returned */
#define HH_EINVAL (-1)     /* invalid argument */
#define HH_ENOMEM (-2)     /* device or host allocation failed */
#define HH_EHIP (-3)       /* a HIP runtime call failed */
#define HH_ENUMERIC (-4)   /* NaN/Inf met in the Krylov recurrence */

typedef struct hh_problem hh_problem;
typedef struct hh_solver hh_solver;
typedef struct hh_cnn hh_cnn;

/* Problem statement (section 2): unit interval / square, uniform open knot
 * vectors of degree p (ends repeated p+1 times, section 2.3.1), homogeneous
 * Dirichlet conditions, constant or element-wise wave number; optionally (MP
 * 1-A, section 2.1) a radiation condition at the right end of a 1D problem.
 * dim = 3: the unit cube with the tensor-product basis phi_i(x) phi_j(y) phi_l(z)
 * (section 2.3 carried to three directions; section 4.3 expects the method's
 * advantage to grow there): constant k and Dirichlet conditions only,
 * K = Mz (x) My (x) Kx + Mz (x) Ky (x) Mx + Kz (x) My (x) Mx, M = Mz (x) My (x) Mx. */
typedef struct {
    int dim;               /* 1, 2 or 3 */
    int p;                 /* B-spline degree, 1..5 */
    int n_el[2];           /* elements in x and y (n_el[1] ignored when dim == 1); >= 2 */
    int k_mode;            /* 0: constant k; 1: one k per finest element */
    double k;              /* the constant wave number (k_mode 0), > 0 */
    const double* k_elem;  /* k_mode 1: HOST array of k (not k^2) per element,
                              x fastest, n_el[0] * n_el[1] values (n_el[0] in 1D);
                              copied, the caller may free it on return */
    int bc_right;          /* 0: Dirichlet at x = 1; 1: the radiation condition u' - i k u = 0 at
                              x = 1 (MP 1-A; dim 1 and constant k only, else HH_EINVAL): the last
                              basis function is kept (n_el + p - 1 unknowns) and the boundary
                              term -i k phi_i(1) phi_j(1) joins A and M_beta (unshifted) on every
                              level; the left end stays Dirichlet (its value enters through
                              hh_rhs_dirichlet_lift) */
    int n_el_z;            /* dim 3: elements in z (>= 2); ignored otherwise */
    double length[3];      /* extent of the domain per direction, (0, L_d): the geometry map
                              F(xi) = (L_1 xi_1, ...) of section 2.3 applied to the parametric
                              unit square (the basis lives on the physical breakpoints L_d i /
                              n_el, k is a physical wave number, source points are physical
                              coordinates in [0, L_d]); 0 means 1, negative or non-finite
                              values are HH_EINVAL */
} hh_problem_desc;

/* Preconditioner and Krylov parameters (hh_default_opts fills the defaults). */
typedef struct {
    double beta[2];          /* CSLP shift beta1 + i beta2 (section 3); default 1, 0.5 */
    double omega;            /* Jacobi damping on the finest level; default 0.8 */
    int nu_pre, nu_post;     /* smoothing sweeps; default 1, 1 */
    int n_vcycles;           /* V-cycles per preconditioner application; default 1 */
    int mg_min_elems;        /* coarsen while some direction has more elements; default 8 */
    int coarse_damping;      /* 1: coarse levels use min(omega, 2/g_l), g_l the Gershgorin
                                bound of D^-1 M_beta,l (3D: the finest level too); 0: omega
                                everywhere; default 1 */
    int defl_mode;           /* 0 none, 1 two-level, 2 multilevel; default 2 */
    int defl_direct_max;     /* multilevel: first level with at most this many unknowns is
                                solved directly; 1..65536, default 16384 (variable k: a
                                dense FP64 inverse of N_z^2 entries, 34 GB at 65536) */
    int defl_inner_its[8];   /* fixed inner FGMRES steps at deflation levels 1..8;
                                default 8, 4, 2, 1, 1, 1, 1, 1 */
    int restart;             /* outer FGMRES restart length, 1..200; default 50 */
    int maxit;               /* outer Arnoldi steps cap; default 1000 */
    double tol;              /* stop at ||f - A u|| <= tol ||f||; default 1e-7 */
    int precision;           /* 0: all FP64; 1: V-cycle in FP32, rest FP64; default 0 */
    int time_kernels;        /* kernel class timed with HIP events during hh_solve (results
                                in hh_solve_info): 0 none (default), 1 finest-level operator
                                (stencil) kernels, 2 exact E^-1 solve of the direct
                                deflation level (all its kernels), 3 outer Arnoldi MGS
                                kernels, 4 the tiled stored-stencil operator of coarse
                                variable-k levels, 5 the packed symmetric tile products of
                                the substructured E^-1 */
    int autotune;            /* 1 (default): at setup, time the strip level-operator kernel
                                of every level that uses it (FP64 and FP32; levels of at
                                most 32768 unknowns with constant k use a one-thread-per-
                                unknown kernel instead, 2D stored-stencil levels a tiled
                                kernel from 2048 unknowns on, below it the one-thread-per-
                                unknown kernel) with strip heights
                                4..64 rows and keep the fastest; 0: a fixed rule (the
                                tallest strip that still gives 2048 waves).  3D: the output
                                slices per workgroup of the slice-marching operator (2..32;
                                fixed rule: the longest of 16..2 that gives 1024
                                workgroups) on every level above the coarsest.  Results do
                                not depend on it. */
    int ortho;               /* Arnoldi orthogonalisation, modified Gram-Schmidt in both forms:
                                0 (default): where the restart length is at most 50 and
                                the vectors at most 65536 entries, the one-reduction form
                                (the triangular system (I + L) h = V^H w, L the strictly
                                lower part of V^H V: equal to the projection-by-projection
                                coefficients in exact arithmetic, one grid-wide sum per
                                step instead of j + 1); 1: always one grid-wide sum per
                                projection.  Results agree to rounding. */
    int defl_direct_solver;  /* exact E^-1 at the direct deflation level when k varies
                                (constant k always uses the fast diagonalisation):
                                0 (default): substructured from 2048 unknowns on, else a
                                dense inverse; 1: dense inverse (LU, N_z^2 entries);
                                2: substructured - bands of p grid lines cut the level into
                                subdomains whose interiors are eliminated exactly (dense
                                inverse per subdomain) and the separator Schur complement
                                is inverted densely; HH_EINVAL if no such cut exists.  All
                                three are exact factorisations of E (section 3). */
    int mg_coarse;           /* coarse multigrid operators when k varies: 0 (default) Galerkin
                                P^T M_beta P; 1 rediscretised on the coarse elements with k^2 of
                                a coarse element the mean over its children (the one or two
                                elements per direction of the next finer level), a cheaper
                                coarse-grid variant of the CSLP (section 3).  Only the V-cycle
                                changes: the deflation matrices stay Galerkin.  Constant k:
                                both are the same operator. */
    int defl_z;              /* deflation vectors: 0 (default) the knot-insertion prolongation
                                of the multigrid hierarchy (Z = P, any defl_mode); 1 the
                                adapted deflation preconditioner's (ADP, section 3): along
                                each direction nc = nf / 2 coarse unknowns, coarse c (0-based)
                                at fine 2c + 1 with weights (1, 6 - defl_eps, 1) / 8 there
                                (quadratic rational Bezier curve) and (1, 1) / 2 on the fine
                                unknowns between; 2D: Z_y (x) Z_x, 3D: Z_z (x) Z_y (x) Z_x.
                                E = Z^T A Z (a band of half-width (p + 4) / 2 per direction)
                                is solved exactly.
                                Two-level only: defl_mode must be 1 (HH_EINVAL otherwise). */
    double defl_eps;         /* the ADP weight parameter epsilon (section 3); default 0.  The
                                paper takes its value from an earlier work without printing it. */
    int precond;             /* 0 (default): the deflated, multigrid-approximated CSLP above;
                                1: the paper's comparison preconditioner C_ex (sections 4.3,
                                4.4): M_ex = K - (1 + i cex_beta2) M_k inverted exactly by
                                fast diagonalisation of the finest level (constant k only:
                                HH_EINVAL otherwise); multigrid and deflation options are not
                                used by the solve */
    double cex_beta2;        /* C_ex shift; 0 (default): the paper's, 1/k in 1D, 1/(3k) in 2D */
    int defl_refine;         /* iterative refinement steps of the substructured E^-1: -1 (default)
                                as many as bring the set-up check below 1e-12 (at most 3);
                                0..3: that many */
    double defl_kh_max;      /* multilevel deflation: the direct level is also never coarser than
                                the last level l >= 1 with k_max h_l <= defl_kh_max (k_max the
                                largest wave number, h_l the level's longest element); coarser
                                deflation levels no longer hold A's near-null space and the inner
                                solves stall.  Default 2.0; 0 turns the rule off */
    int use_graph;           /* 1: every outer Arnoldi step (the preconditioner T with its inner
                                solves, A z and the MGS/Givens step) is captured once per step
                                index into a HIP graph on a stream of the solver's own and
                                replayed by later steps and solves (same kernels, same results);
                                not while a kernel class is timed or samples are captured, and
                                without cooperative launches.  0 (default): launched one by one */
} hh_solver_opts;

typedef struct {
    int iters;               /* outer Arnoldi steps */
    int restarts;            /* completed restarts */
    int converged;           /* 1 if ||f - A u|| <= tol ||f|| */
    double relres_true;      /* ||f - A u|| / ||f||, recomputed in FP64 */
    double relres_est;       /* |g_{j+1}| / ||f|| of the last Arnoldi step */
    double t_solve_ms;       /* wall time of hh_solve (host clock, stream drained) */
    double op_ms_total;      /* time_kernels: summed device time of the timed kernel class */
    int op_launches;         /* time_kernels: number of such launches */
    double op_bytes_per_launch; /* algorithmic HBM bytes per launch of that class (mean) */
    int status;              /* the hh_status of this solve (per problem in hh_solve_batched) */
    double model_bytes;      /* algorithmic HBM bytes of the work the solve used: every kernel's
                                operands counted once per launch (vectors, stencil or k^2
                                coefficients, stored factors of E^-1, Krylov basis); the
                                whole-solve HBM fraction is model_bytes / t_solve / peak */
    double model_flops;      /* floating-point operations of the same work (a complex x real
                                multiply-add counts 4, complex x complex 8) */
    int arnoldi_fallback;    /* hh_solve: 1 if a grid-wide Arnoldi kernel gave up waiting for
                                other workgroups (bounded wait) and the solve, started from
                                zero, was run again with the per-projection kernels (which
                                the solver keeps using); 0 otherwise */
} hh_solve_info;

typedef struct {
    int n[2];                /* interior unknowns per direction at this level */
    int n_el[2];             /* elements per direction */
    long long N;             /* n[0] * n[1] * n_z */
    double omega;            /* Jacobi damping used at this level */
    double gersh;            /* Gershgorin bound g_l of D^-1 M_beta,l */
    int n_levels;            /* multigrid levels (finest = 0) */
    int defl_direct_level;   /* L_z: deflation level solved directly (0: no deflation).  With
                                the ADP vectors (defl_z = 1) it is n_levels: a level of its
                                own, outside the multigrid hierarchy, that hh_level_info and
                                hh_apply (HH_OP_A, HH_OP_K, HH_OP_MK, HH_OP_EINV) accept */
    int op_rows[2];          /* strip height (rows) of the level-operator kernel, FP64 / FP32
                                (3D: output slices per workgroup); 0: the fixed rule */
    int defl_sub[2];         /* substructured E^-1 (defl_direct_solver): subdomains per
                                direction at the direct deflation level, else 0 */
    long long defl_sep;      /* separator unknowns of that cut (0 if not substructured) */
    double defl_check;       /* ||c - E E^-1 c|| / ||c|| for a fixed pseudo-random c, taken
                                at setup (substructured E^-1 only; -1 otherwise) */
    int defl_refine;         /* iterative refinement steps per substructured E^-1 (set-up
                                chooses 0..3 from the residual of one pass; each step costs
                                one more pass) */
    int n_z;                 /* interior unknowns in z at this level (1 unless dim == 3);
                                N = n[0] * n[1] * n_z */
    int n_el_z;              /* elements in z (1 unless dim == 3) */
} hh_level_stats;

/* Debug / parity operators of hh_apply. */
#define HH_OP_A        0   /* y = A_l x */
#define HH_OP_MBETA    1   /* y = M_beta,l x */
#define HH_OP_JACOBI0  2   /* y = omega_l D_l^-1 x (first sweep from a zero guess) */
#define HH_OP_RESTRICT 3   /* y (level l+1) = P_{l+1}^T x (level l) */
#define HH_OP_PROLONG  4   /* y (level l) = P_{l+1} x (level l+1) */
#define HH_OP_VCYCLE   5   /* y = V-cycle(s) from level l applied to x */
#define HH_OP_T        6   /* y = T_l x: deflated CSLP preconditioner at level l */
#define HH_OP_EINV     7   /* y = E^-1 x at deflation level l >= 1 (direct or inner FGMRES) */
#define HH_OP_K        8   /* y = K_l x (stiffness, section 2.3; Galerkin = rediscretised) */
#define HH_OP_MK       9   /* y = M_k,l x (k^2-weighted mass of A_l = K_l - M_k,l; Galerkin) */
#define HH_OP_ZT      10   /* y = Z^T x: deflation restriction from level l to the next
                              deflation level (defl_z = 0: P^T, as HH_OP_RESTRICT; defl_z = 1:
                              the ADP vectors, level 0 only) */
#define HH_OP_Z       11   /* y = Z x: the matching deflation prolongation */

/* Fills *o with the defaults listed above. */
void hh_default_opts(hh_solver_opts* o);

/* Thread-local message of the last error ("" if none). */
const char* hh_last_error(void);

/* Builds the problem: knot vectors, element matrices (Gauss-Legendre,
 * p+1 points), k^2 per element (section 2.3).  Host work, plus the upload of
 * the k^2 field (k_mode 1) to the current device, ordered on `stream`; returns
 * after the stream has drained. */
hh_status hh_assemble(const hh_problem_desc* d, void* stream, hh_problem** out);

/* Idempotent on NULL. */
hh_status hh_problem_destroy(hh_problem* pr);

/* Interior unknowns per direction at the finest level (n[1] = 1 in 1D).
 * HH_EINVAL for a 3D problem (use hh_problem_size3). */
hh_status hh_problem_size(const hh_problem* pr, int n[2]);

/* The same for every dimension: n[0..2], with 1 for the directions a 1D or 2D
 * problem does not have. */
hh_status hh_problem_size3(const hh_problem* pr, int n[3]);

/* Element (knot-span) index holding x0 per direction: floor(x0 / L * n_el), with
 * x0 == L mapped to the last element (the half-open span rule of section
 * 2.3.1).  x0 outside [0,L] -> HH_EINVAL.  x0 and spans hold dim entries. */
hh_status hh_point_spans(const hh_problem* pr, const double* x0, int* spans);

/* Point source load f_i = amp * Phi_i(x0) (the Galerkin load of amp * delta(x - x0),
 * MP 1-B / MP 2-A / MP 2-B; x0 holds dim coordinates).  f_dev: device, N complex
 * doubles, overwritten. */
hh_status hh_rhs_point_source(const hh_problem* pr, const double* x0, double amp,
                              void* f_dev, void* stream);

/* MP 1-A (section 2.1): the right-hand side of the boundary value u(0) = u0 with no
 * source, f_i = -u0 (K - k^2 M)_{i,0}: the eliminated first basis function's
 * column moved to the right-hand side.  Problems with bc_right = 1 only
 * (HH_EINVAL otherwise).  f_dev: device, N complex doubles, overwritten. */
hh_status hh_rhs_dirichlet_lift(const hh_problem* pr, double u0, void* f_dev, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same load as
 * hh_rhs_point_source, bit-identical, with no device or heap allocation.  The
 * 1D basis factors are staged in a fixed device array of 65536 doubles
 * (512 KB) that each device keeps for the life of the process; HH_EINVAL if
 * n[0] + n[1] (+ n[2] in 3D) of the finest level exceeds 65536.  The current device must be
 * the one that holds f_dev and stream.  Every call on a device shares that
 * array (the last call's contents stay in it): calls that overlap on one
 * device race; within one process they are serialised by a lock, from several
 * processes they must not overlap.  Returns after the stream has drained. */
hh_status hh_rhs_point_source_noalloc(const hh_problem* pr, const double* x0, double amp,
                                      void* f_dev, void* stream);

/* Finest-level operators of an assembled problem in CSR form (section 2.3:
 * stiffness, k^2-weighted mass and A = K - M_k after Dirichlet elimination),
 * for exact comparisons of sparsity and values on small meshes; host only.
 * which: 0 K, 1 M_k, 2 A.  Rows and columns are interior indices (x fastest);
 * every entry of the tensor-product band (|i1 - j1| <= p and |i2 - j2| <= p,
 * and |i3 - j3| <= p in 3D, in range) is stored, columns ascending within a row.  Call with row_ptr NULL to
 * get *nnz only; otherwise row_ptr (N + 1), col_idx and val (capacity entries
 * each, host) are filled and HH_EINVAL is returned if capacity < nnz.  Under the
 * radiation condition (bc_right = 1) A is complex: which = 2 gives HH_EINVAL. */
hh_status hh_export_csr(const hh_problem* pr, int which, long long* nnz, long long* row_ptr, int* col_idx,
                        double* val, long long capacity);

/* Builds the multigrid / deflation hierarchy and allocates all device workspace
 * (section 3): coarse knot vectors by knot halving, knot-insertion transfers,
 * Galerkin coarse operators, Jacobi diagonals, the dense inverse of the coarsest
 * M_beta, and the exact solver of the deflation matrix E at L_z: for constant k,
 * E = My (x) Kx + Ky (x) Mx - k^2 My (x) Mx is diagonalised by the generalised
 * eigenvectors of the two 1D pencils (K, M) (fast diagonalisation: four small
 * dense passes per solve, no N_z x N_z matrix); for variable k, a dense inverse
 * (LU).  HH_ENUMERIC if E is singular.  3D problems: multigrid with two-level,
 * multilevel or no deflation, E diagonalised by the three 1D pencils (six dense
 * passes; with the ADP vectors the pencils of their Galerkin bands), no coarse
 * one-workgroup tail, and neither C_ex nor a learned smoother.  The solver keeps a reference to
 * the problem, which must outlive it. */
hh_status hh_setup(const hh_problem* pr, const hh_solver_opts* o, void* stream,
                   hh_solver** out);

/* Idempotent on NULL. */
hh_status hh_solver_destroy(hh_solver* s);

/* Solves A u = f.  f_dev, u_dev: device, N complex doubles.  use_u0 = 1 starts
 * from the contents of u_dev, else from zero.  Returns HH_ENOCONV (with the last
 * iterate in u_dev) when maxit is reached.  info may be NULL. */
hh_status hh_solve(hh_solver* s, const void* f_dev, void* u_dev, int use_u0,
                   hh_solve_info* info, void* stream);

/* Batched solve: n independent problems, each with its own solver (problems
 * may differ in size, degree and wave number), solved concurrently by up to
 * four host workers, each on its own HIP stream of a pool (default priority):
 * a worker takes the largest problem not yet started, runs its solve as
 * hh_solve does, then the next.  The small, latency-bound solves of a batch
 * thus overlap on the GPU.  s, f, u, infos:
 * arrays of n entries; f[i], u[i] device vectors of problem i (as in hh_solve,
 * zero initial guess).  The pool streams wait for the work already on `stream`,
 * and `stream` waits for them before the call returns.  Per-problem results and
 * status are in infos[i] (use_graph is not applied inside a batch: the steps
 * are launched one by one); the return value is the first negative status (its
 * message names the problem), HH_ENOCONV if some problem did not converge, else
 * HH_OK.  The solvers must not be used elsewhere during the call. */
hh_status hh_solve_batched(hh_solver* const* s, int n, const void* const* f, void* const* u,
                           hh_solve_info* infos, void* stream);

/* Residual history of the last completed hh_solve (or batched solve) on this solver:
 * the estimated relative residual |g_{j+1}| / ||f|| of every Arnoldi step in order,
 * across restarts (section 4.3 stops on it within a cycle; the true residual is
 * recomputed at every cycle's end).  *n receives the count; with out non-NULL,
 * min(capacity, count) values are copied to the HOST array out. */
hh_status hh_solve_history(const hh_solver* s, double* out, int capacity, int* n);

/* Level sizes and parameters; level in [0, n_levels), or defl_direct_level. */
hh_status hh_level_info(const hh_solver* s, int level, hh_level_stats* out);

/* Selects the kernel class timed during later hh_solve calls (values as for
 * hh_solver_opts.time_kernels); 0 turns timing off. */
hh_status hh_set_kernel_timing(hh_solver* s, int cls);

/* Debug / tests only: polls a grid-exchange wait of the Arnoldi kernels makes
 * before it gives up and flags a timeout (spins >= 1; 0 restores the default,
 * about a second).  A tiny value forces the timeout path while every kernel
 * still exits normally.  Also re-enables the grid-wide Arnoldi kernels after a
 * fallback. */
hh_status hh_debug_set_spin_limit(hh_solver* s, int spins);

/* Applies one building block of the preconditioner (HH_OP_*) at `level` to a
 * device vector: for checking against a reference implementation.  x_dev and
 * y_dev must not overlap. */
hh_status hh_apply(hh_solver* s, int op, int level, const void* x_dev, void* y_dev,
                   void* stream);

/* ---- learned fine-level smoother (not in the paper) ----
 * A complex 3x3 CNN C (complex channels 2 -> 16 -> 16 -> 16 -> 1, CReLU after
 * the first three layers, zero padding) on the finest interior control-point
 * grid.  Inputs: r/||r|| and c = k^2 h^2 (k of the finest element with the
 * unknown's clamped index).  As the finest-level smoother it adds a learned
 * correction to the damped Jacobi step: x += omega D^-1 r + rms C(r/rms, c),
 * r = b - M_beta x, rms = ||r|| / sqrt(N) (inputs of order one on any grid),
 * so zero weights give damped Jacobi exactly.  Weights and
 * activations are BF16 with FP32 accumulation (MFMA).  Parameters are float
 * (re, im) pairs, per layer W[co][ci][dy][dx] then b[co]. */

/* Creates a network with seeded random parameters. */
hh_status hh_cnn_create(unsigned long long seed, hh_cnn** out);
/* Idempotent on NULL. */
hh_status hh_cnn_destroy(hh_cnn* c);
/* Number of floats of the parameter vector (twice the complex parameters). */
hh_status hh_cnn_num_params(const hh_cnn* c, int* n_floats);
/* Host copies of the FP32 master parameters (n_floats must match). */
hh_status hh_cnn_get_params(const hh_cnn* c, float* host, int n_floats);
/* Replaces the parameters (HH_ENUMERIC if any is not finite; then nothing
 * changes) and resets the optimiser state. */
hh_status hh_cnn_set_params(hh_cnn* c, const float* host, int n_floats);
/* Training loss L = ||r - M_beta s||^2 / ||r||^2 with s the smoother step above for
 * one finest-level residual r_dev (device, N complex doubles) of solver s, and
 * (if grad_host != NULL) the gradient dL/dRe + i dL/dIm of every parameter. */
hh_status hh_cnn_loss_grad(hh_cnn* c, hh_solver* s, const void* r_dev, double* loss, float* grad_host,
                           int n_floats, void* stream);
/* Debug / parity (tests only): fused = 1 (default) evaluates the network of
 * the smoother step in one kernel per step (all four layers on LDS-resident
 * tiles); 0 uses one kernel per layer, as training does.  Both give
 * bit-identical results. */
hh_status hh_cnn_set_fused(hh_cnn* c, int fused);
/* One Adam step (beta 0.9 / 0.999) with learning rate lr on the loss above. */
hh_status hh_cnn_train_step(hh_cnn* c, hh_solver* s, const void* r_dev, double lr, double* loss, void* stream);
/* Training on captured V-cycle inputs (hh_solver_capture): Adam steps over the
 * (problem, sample) pairs of n problems in an order drawn from `seed`
 * (Fisher-Yates with SplitMix64), each step the loss and gradient above plus
 * one Adam update.  samples[i]: device, counts[i] finest-level vectors of
 * solvers[i] back to back.  loss_before / loss_after (may be NULL): the mean
 * loss over all pairs before and after.  out_weights (may be NULL): the
 * trained parameters are also written to that file (hh_cnn_save format).
 * HH_ENUMERIC if a loss is not finite (the parameters then hold the last
 * finite step). */
typedef struct {
    int steps;                /* Adam steps; <= 0: 800 */
    double lr;                /* learning rate; <= 0: 3e-4 */
    unsigned long long seed;  /* order of the pairs */
} hh_cnn_train_opts;
hh_status hh_cnn_train(hh_cnn* c, const hh_cnn_train_opts* o, hh_solver* const* solvers,
                       const void* const* samples, const int* counts, int n, double* loss_before,
                       double* loss_after, const char* out_weights, void* stream);
/* Weight files: 8 bytes "HHCNNv1\0", int32 n (floats), n float32 parameters
 * (as hh_cnn_get_params), uint64 FNV-1a hash of those n * 4 bytes; little
 * endian.  hh_cnn_load creates a network from such a file (HH_EINVAL for a
 * file of another format, size or hash). */
hh_status hh_cnn_save(const hh_cnn* c, const char* path);
hh_status hh_cnn_load(const char* path, hh_cnn** out);
/* Uses the network as the finest-level smoother of s (NULL: damped Jacobi).
 * The network must outlive its use by s. */
hh_status hh_solver_set_smoother(hh_solver* s, hh_cnn* c);
/* Training-sample capture: during later solves, every finest-level V-cycle
 * input vector is copied into buf_dev (device, max_samples x N complex
 * doubles) until it is full.  buf_dev NULL stops the capture and keeps the
 * count; hh_solver_captured reports how many vectors the last capture wrote.
 * The copies are stream-ordered: read buf_dev after the solve's stream. */
hh_status hh_solver_capture(hh_solver* s, void* buf_dev, int max_samples);
hh_status hh_solver_captured(const hh_solver* s, int* n);

#ifdef __cplusplus
}
#endif

#endif /* HH_H */
