// C ABI entry points (include/hh.h): argument checks, error capture, dispatch.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <cstring>
#include <atomic>
#include <mutex>
#include <thread>
#include <algorithm>
#include <set>

#include "solver.h"

namespace hh {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace hh

using namespace hh;

#define HH_TRY try {
#define HH_CATCH                                          \
    }                                                     \
    catch (const Err& e) {                                \
        set_error(e.msg);                                 \
        return e.code;                                    \
    }                                                     \
    catch (const std::bad_alloc&) {                       \
        set_error("host allocation failed");              \
        return HH_ENOMEM;                                 \
    }                                                     \
    catch (const std::exception& e) {                     \
        set_error(e.what());                              \
        return HH_EINVAL;                                 \
    }

extern "C" {

void hh_default_opts(hh_solver_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->beta[0] = 1.0;
    o->beta[1] = 0.5;
    o->omega = 0.8;
    o->nu_pre = 1;
    o->nu_post = 1;
    o->n_vcycles = 1;
    o->mg_min_elems = 8;
    o->coarse_damping = 1;
    o->defl_mode = 2;
    o->defl_direct_max = 16384;
    const int its[8] = {8, 4, 2, 1, 1, 1, 1, 1};
    for (int i = 0; i < 8; ++i) o->defl_inner_its[i] = its[i];
    o->restart = 50;
    o->maxit = 1000;
    o->tol = 1e-7;
    o->precision = 0;
    o->time_kernels = 0;
    o->autotune = 1;
    o->ortho = 0;
    o->defl_direct_solver = 0;
    o->mg_coarse = 0;
    o->defl_z = 0;
    o->defl_eps = 0.0;
    o->precond = 0;
    o->cex_beta2 = 0.0;
    o->defl_refine = -1;
    o->defl_kh_max = 2.0;
    o->use_graph = 0;
}

const char* hh_last_error(void) { return g_err.c_str(); }

hh_status hh_assemble(const hh_problem_desc* d, void* stream, hh_problem** out) {
    HH_TRY
    if (!out) throw Err{HH_EINVAL, "out is NULL"};
    *out = nullptr;
    std::unique_ptr<ProblemImpl> P(build_problem(d));
    int ndev = 0;
    if (!P->k2.empty() && hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
        // the finest-level k^2 field, read by the operator kernels of level 0
        // (host-only uses - spans, CSR export - need no device; hh_setup
        // uploads it if it is not there yet)
        hipStream_t s = (hipStream_t)stream;
        P->k2_dev.alloc(P->k2.size() * sizeof(double));
        HH_HIP(hipMemcpyAsync(P->k2_dev.p, P->k2.data(), P->k2.size() * sizeof(double), hipMemcpyHostToDevice, s));
        HH_HIP(hipStreamSynchronize(s));
    }
    auto* h = new hh_problem();
    h->impl = std::move(*P);
    *out = h;
    set_error("");
    return HH_OK;
    HH_CATCH
}

hh_status hh_problem_destroy(hh_problem* pr) {
    delete pr;
    return HH_OK;
}

hh_status hh_problem_size(const hh_problem* pr, int n[2]) {
    HH_TRY
    if (!pr || !n) throw Err{HH_EINVAL, "NULL argument"};
    if (pr->impl.dim == 3) throw Err{HH_EINVAL, "a 3D problem has three sizes (hh_problem_size3)"};
    n[0] = pr->impl.ax0.n;
    n[1] = pr->impl.ay0.n;
    return HH_OK;
    HH_CATCH
}

hh_status hh_problem_size3(const hh_problem* pr, int n[3]) {
    HH_TRY
    if (!pr || !n) throw Err{HH_EINVAL, "NULL argument"};
    n[0] = pr->impl.ax0.n;
    n[1] = pr->impl.ay0.n;
    n[2] = pr->impl.az0.n;
    return HH_OK;
    HH_CATCH
}

static int span_of(double x, int nel) {
    int e = (int)std::floor(x * nel);
    return e < nel - 1 ? e : nel - 1;
}

hh_status hh_point_spans(const hh_problem* pr, const double* x0, int* spans) {
    HH_TRY
    if (!pr || !x0 || !spans) throw Err{HH_EINVAL, "NULL argument"};
    const ProblemImpl& P = pr->impl;
    for (int d = 0; d < P.dim; ++d) {
        if (!(x0[d] >= 0.0 && x0[d] <= P.len[d])) throw Err{HH_EINVAL, "source point outside the domain"};
        spans[d] = span_of(x0[d] / P.len[d], P.nel[d]);
    }
    return HH_OK;
    HH_CATCH
}

hh_status hh_export_csr(const hh_problem* pr, int which, long long* nnz, long long* row_ptr, int* col_idx,
                        double* val, long long capacity) {
    HH_TRY
    if (!pr || !nnz) throw Err{HH_EINVAL, "NULL argument"};
    if (which < 0 || which > 2) throw Err{HH_EINVAL, "which must be 0 (K), 1 (M_k) or 2 (A)"};
    const ProblemImpl& P = pr->impl;
    if (P.somm && which == 2) throw Err{HH_EINVAL, "A is complex under the radiation condition (export K and M_k)"};
    const bool const_k = P.k_mode == 0;
    std::vector<double> S;
    if (!const_k) galerkin_mass_stencil(P.ax0, P.ay0, P.k2, S);
    const double k2c = const_k ? P.k * P.k : 0.0;
    const long long N = P.N();
    // rows of the tensor-product band (2D / 1D: visit_row; the cube: visit_row3)
    auto row = [&](long long I, auto&& f) {
        if (P.dim == 3)
            visit_row3(P.ax0, P.ay0, P.az0, k2c, I, f);
        else
            visit_row(P.ax0, P.ay0, const_k, k2c, S, I, f);
    };
    long long count = 0;
    for (long long I = 0; I < N; ++I) row(I, [&](long long, double, double) { ++count; });
    *nnz = count;
    if (!row_ptr) return HH_OK;
    if (!col_idx || !val) throw Err{HH_EINVAL, "NULL col_idx or val"};
    if (capacity < count) throw Err{HH_EINVAL, "capacity below the number of entries"};
    long long k = 0;
    for (long long I = 0; I < N; ++I) {
        row_ptr[I] = k;
        row(I, [&](long long J, double kv, double mv) {
            col_idx[k] = (int)J;
            val[k] = which == 0 ? kv : which == 1 ? mv : kv - mv;
            ++k;
        });
    }
    row_ptr[N] = k;
    return HH_OK;
    HH_CATCH
}

hh_status hh_rhs_point_source(const hh_problem* pr, const double* x0, double amp, void* f_dev, void* stream) {
    HH_TRY
    if (!pr || !x0 || !f_dev) throw Err{HH_EINVAL, "NULL argument"};
    rhs_point_source(pr->impl, x0, amp, (cx<double>*)f_dev, (hipStream_t)stream);
    return HH_OK;
    HH_CATCH
}

hh_status hh_rhs_dirichlet_lift(const hh_problem* pr, double u0, void* f_dev, void* stream) {
    HH_TRY
    if (!pr || !f_dev) throw Err{HH_EINVAL, "NULL argument"};
    rhs_dirichlet_lift(pr->impl, u0, (cx<double>*)f_dev, (hipStream_t)stream);
    return HH_OK;
    HH_CATCH
}

hh_status hh_rhs_point_source_noalloc(const hh_problem* pr, const double* x0, double amp, void* f_dev,
                                      void* stream) {
    HH_TRY
    if (!pr || !x0 || !f_dev) throw Err{HH_EINVAL, "NULL argument"};
    rhs_point_source_noalloc(pr->impl, x0, amp, (cx<double>*)f_dev, (hipStream_t)stream);
    return HH_OK;
    HH_CATCH
}

hh_status hh_setup(const hh_problem* pr, const hh_solver_opts* o, void* stream, hh_solver** out) {
    HH_TRY
    if (!pr || !out) throw Err{HH_EINVAL, "NULL argument"};
    *out = nullptr;
    auto impl = std::make_unique<SolverImpl>();
    impl->prob = &pr->impl;
    if (o)
        impl->o = *o;
    else
        hh_default_opts(&impl->o);
    impl->setup((hipStream_t)stream);
    auto* h = new hh_solver();
    h->impl = std::move(impl);
    *out = h;
    set_error("");
    return HH_OK;
    HH_CATCH
}

hh_status hh_solver_destroy(hh_solver* s) {
    delete s;
    return HH_OK;
}

hh_status hh_solve(hh_solver* s, const void* f_dev, void* u_dev, int use_u0, hh_solve_info* info, void* stream) {
    HH_TRY
    if (!s || !f_dev || !u_dev) throw Err{HH_EINVAL, "NULL argument"};
    if (f_dev == u_dev) throw Err{HH_EINVAL, "f and u must not alias"};
    return s->impl->solve((const cx<double>*)f_dev, (cx<double>*)u_dev, use_u0, info, (hipStream_t)stream);
    HH_CATCH
}

// Stream pool of the batched solve (default priority; created on first use and
// kept for the life of the process: the handles are reclaimed with the HIP
// runtime at exit, and destroying them from a static destructor would run after
// the runtime's own teardown).
static std::vector<hipStream_t> g_pool;
static std::mutex g_pool_mu;
// Host workers of a batched solve, one per pool stream: as many as the hardware
// queues a process gets by default (four), measured best on the 64-problem
// batch (2 workers 294 ms, 4: 259 ms, 8: 264 ms, one after another: 510 ms).
constexpr int kBatchWorkers = 4;

// An event released on every path (a HIP call that throws between creation and
// use must not leak it).
struct Event {
    hipEvent_t e = nullptr;
    Event() { HH_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming)); }
    ~Event() {
        if (e) (void)hipEventDestroy(e);
    }
    Event(const Event&) = delete;
    Event& operator=(const Event&) = delete;
};

static std::vector<hipStream_t> pool_streams(int n) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    while ((int)g_pool.size() < n) {
        hipStream_t st;
        HH_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        g_pool.push_back(st);
    }
    return std::vector<hipStream_t>(g_pool.begin(), g_pool.begin() + n);
}

hh_status hh_solve_batched(hh_solver* const* s, int n, const void* const* f, void* const* u,
                           hh_solve_info* infos, void* stream) {
    HH_TRY
    if (!s || !f || !u || !infos || n < 1) throw Err{HH_EINVAL, "NULL argument or n < 1"};
    {
        std::set<const hh_solver*> seen;
        for (int i = 0; i < n; ++i) {
            if (!s[i] || !f[i] || !u[i]) throw Err{HH_EINVAL, "NULL solver or vector in the batch"};
            if (!seen.insert(s[i]).second) throw Err{HH_EINVAL, "a solver appears twice in the batch"};
            if (f[i] == u[i]) throw Err{HH_EINVAL, "f and u must not alias"};
        }
    }
    hipStream_t cs = (hipStream_t)stream;
    int dev = 0;
    HH_HIP(hipGetDevice(&dev));
    const int ns = std::min(n, kBatchWorkers);
    const std::vector<hipStream_t> st = pool_streams(ns);
    // the pool streams start after the work already on the caller's stream
    {
        Event fork;
        HH_HIP(hipEventRecord(fork.e, cs));
        for (int k = 0; k < ns; ++k) HH_HIP(hipStreamWaitEvent(st[k], fork.e, 0));
    }
    // largest problems first: each worker takes the next unsolved one, so the
    // long solves start early and the short ones fill in around them
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return s[a]->impl->lev[0]->N > s[b]->impl->lev[0]->N; });
    // no cooperative launches from the workers: a grid-wide Arnoldi kernel runs
    // as a resident grid sized for four concurrent solves, or as the
    // per-projection kernels when it does not fit (runs whose workers launched
    // cooperative grids on the pool streams ended in a segmentation fault at
    // process exit)
    // nor step graphs: four workers replaying graphs measured slower than the
    // same steps launched one by one (64 point-source problems, k 50..400,
    // p 2..4: 321 ms against 261 ms)
    for (int i = 0; i < n; ++i) {
        s[i]->impl->allow_coop = false;
        s[i]->impl->in_batch = true;
    }
    std::vector<int> status(n, HH_OK);
    std::vector<std::string> errs(n);
    std::atomic<int> next{0};
    auto worker = [&](int w) {
        if (hipSetDevice(dev) != hipSuccess) return;
        for (;;) {
            const int k = next.fetch_add(1);
            if (k >= n) break;
            const int i = order[k];
            try {
                hh_solve_info inf{};
                status[i] = s[i]->impl->solve((const cx<double>*)f[i], (cx<double>*)u[i], 0, &inf, st[w]);
                infos[i] = inf;
            } catch (const Err& e) {
                status[i] = e.code;
                errs[i] = e.msg;
            } catch (const std::exception& e) {
                status[i] = HH_EINVAL;
                errs[i] = e.what();
            }
        }
    };
    {
        std::vector<std::thread> pool;
        for (int w = 1; w < ns; ++w) pool.emplace_back(worker, w);
        worker(0);
        for (auto& t : pool) t.join();
    }
    for (int i = 0; i < n; ++i) {
        s[i]->impl->allow_coop = true;
        s[i]->impl->in_batch = false;
    }
    // the caller's stream continues after every pool stream
    for (int k = 0; k < ns; ++k) {
        Event join;
        HH_HIP(hipEventRecord(join.e, st[k]));
        HH_HIP(hipStreamWaitEvent(cs, join.e, 0));
    }
    HH_HIP(hipStreamSynchronize(cs));
    int ret = HH_OK;
    for (int i = 0; i < n; ++i) {
        if (status[i] < 0) infos[i] = hh_solve_info{};
        infos[i].status = status[i];
        if (status[i] < 0 && ret >= 0) {
            ret = status[i];
            set_error("problem " + std::to_string(i) + ": " + errs[i]);
        }
        if (status[i] == HH_ENOCONV && ret == HH_OK) ret = HH_ENOCONV;
    }
    return ret;
    HH_CATCH
}

hh_status hh_cnn_create(unsigned long long seed, hh_cnn** out) {
    HH_TRY
    if (!out) throw Err{HH_EINVAL, "out is NULL"};
    *out = nullptr;
    auto* c = new hh_cnn();
    try {
        c->impl = std::make_unique<CnnImpl>(seed);
    } catch (...) {
        delete c;
        throw;
    }
    *out = c;
    return HH_OK;
    HH_CATCH
}

hh_status hh_cnn_destroy(hh_cnn* c) {
    delete c;
    return HH_OK;
}

hh_status hh_cnn_num_params(const hh_cnn* c, int* n) {
    HH_TRY
    if (!c || !n) throw Err{HH_EINVAL, "NULL argument"};
    *n = 2 * c->impl->nparam;
    return HH_OK;
    HH_CATCH
}

hh_status hh_cnn_get_params(const hh_cnn* c, float* host, int n) {
    HH_TRY
    if (!c || !host) throw Err{HH_EINVAL, "NULL argument"};
    if (n != 2 * c->impl->nparam) throw Err{HH_EINVAL, "parameter count mismatch"};
    HH_HIP(hipDeviceSynchronize());
    HH_HIP(hipMemcpy(host, c->impl->theta.p, (size_t)n * 4, hipMemcpyDeviceToHost));
    return HH_OK;
    HH_CATCH
}

hh_status hh_cnn_set_params(hh_cnn* c, const float* host, int n) {
    HH_TRY
    if (!c || !host) throw Err{HH_EINVAL, "NULL argument"};
    c->impl->set_params(host, n);
    return HH_OK;
    HH_CATCH
}

hh_status hh_cnn_set_fused(hh_cnn* c, int fused) {
    HH_TRY
    if (!c) throw Err{HH_EINVAL, "NULL argument"};
    c->impl->fused = fused != 0;
    return HH_OK;
    HH_CATCH
}

static MbetaFn finest_mbeta(SolverImpl& S, hipStream_t st) {
    return [&S, st](const cx<double>* x, const cx<double>* b, cx<double>* y, int conj) {
        if (conj)
            S.op_alpha<double>(0, MODE_APPLY, S.o.beta[0], -S.o.beta[1], x, nullptr, y, st);
        else
            S.op_alpha<double>(0, MODE_RESID, S.o.beta[0], S.o.beta[1], x, b, y, st);
    };
}

hh_status hh_cnn_loss_grad(hh_cnn* c, hh_solver* s, const void* r_dev, double* loss, float* grad_host, int n,
                           void* stream) {
    HH_TRY
    if (!c || !s || !r_dev || !loss) throw Err{HH_EINVAL, "NULL argument"};
    if (grad_host && n != 2 * c->impl->nparam) throw Err{HH_EINVAL, "parameter count mismatch"};
    SolverImpl& S = *s->impl;
    hipStream_t st = (hipStream_t)stream;
    const LevelDev& l0 = *S.lev[0];
    *loss = c->impl->loss_grad(l0.n2, l0.n1, (const cx<double>*)r_dev, S.feat.as<float>(),
                               l0.Dinv64.as<cx<double>>(), l0.omega, finest_mbeta(S, st), st);
    if (grad_host) {
        HH_HIP(hipMemcpyAsync(grad_host, c->impl->grad.p, (size_t)n * 4, hipMemcpyDeviceToHost, st));
        HH_HIP(hipStreamSynchronize(st));
    }
    return HH_OK;
    HH_CATCH
}

hh_status hh_cnn_train_step(hh_cnn* c, hh_solver* s, const void* r_dev, double lr, double* loss, void* stream) {
    HH_TRY
    if (!c || !s || !r_dev) throw Err{HH_EINVAL, "NULL argument"};
    if (!(lr > 0.0) || !std::isfinite(lr)) throw Err{HH_EINVAL, "learning rate must be positive"};
    SolverImpl& S = *s->impl;
    hipStream_t st = (hipStream_t)stream;
    const LevelDev& l0 = *S.lev[0];
    const double L = c->impl->loss_grad(l0.n2, l0.n1, (const cx<double>*)r_dev, S.feat.as<float>(),
                                        l0.Dinv64.as<cx<double>>(), l0.omega, finest_mbeta(S, st), st);
    if (!std::isfinite(L)) throw Err{HH_ENUMERIC, "training loss is not finite"};
    c->impl->adam_step(lr, st);
    HH_HIP(hipStreamSynchronize(st));
    if (loss) *loss = L;
    return HH_OK;
    HH_CATCH
}

namespace {
// SplitMix64 step (a counter-based generator: state += golden gamma, then mix)
uint64_t splitmix64(uint64_t& st) {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t fnv1a(const unsigned char* p, size_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 0x100000001b3ull;
    return h;
}

const char kWeightMagic[8] = {'H', 'H', 'C', 'N', 'N', 'v', '1', '\0'};

void save_weights(const CnnImpl& c, const char* path) {
    std::vector<float> v((size_t)2 * c.nparam);
    HH_HIP(hipDeviceSynchronize());
    HH_HIP(hipMemcpy(v.data(), c.theta.p, v.size() * 4, hipMemcpyDeviceToHost));
    const int32_t n = (int32_t)v.size();
    const uint64_t sum = fnv1a((const unsigned char*)v.data(), v.size() * 4);
    FILE* f = std::fopen(path, "wb");
    if (!f) throw Err{HH_EINVAL, std::string("cannot open ") + path + " for writing"};
    const bool ok = std::fwrite(kWeightMagic, 1, 8, f) == 8 && std::fwrite(&n, 4, 1, f) == 1 &&
                    std::fwrite(v.data(), 4, v.size(), f) == v.size() && std::fwrite(&sum, 8, 1, f) == 1;
    const bool closed = std::fclose(f) == 0;
    if (!ok || !closed) throw Err{HH_EINVAL, std::string("write to ") + path + " failed"};
}
}  // namespace

hh_status hh_cnn_train(hh_cnn* c, const hh_cnn_train_opts* o, hh_solver* const* solvers,
                       const void* const* samples, const int* counts, int n, double* loss_before, double* loss_after,
                       const char* out_weights, void* stream) {
    HH_TRY
    if (!c || !o || !solvers || !samples || !counts || n < 1) throw Err{HH_EINVAL, "NULL argument or n < 1"};
    const int steps = o->steps > 0 ? o->steps : 800;
    const double lr = o->lr > 0.0 ? o->lr : 3e-4;
    if (!std::isfinite(lr)) throw Err{HH_EINVAL, "learning rate must be finite"};
    hipStream_t st = (hipStream_t)stream;
    // every (problem, sample) pair, visited in a seeded order (Fisher-Yates)
    std::vector<std::pair<int, int>> pairs;
    for (int i = 0; i < n; ++i) {
        if (!solvers[i] || (counts[i] > 0 && !samples[i])) throw Err{HH_EINVAL, "NULL solver or sample buffer"};
        if (counts[i] < 0) throw Err{HH_EINVAL, "negative sample count"};
        for (int j = 0; j < counts[i]; ++j) pairs.emplace_back(i, j);
    }
    if (pairs.empty()) throw Err{HH_EINVAL, "no training samples"};
    std::vector<int> order(pairs.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    uint64_t rs = o->seed;
    for (size_t i = order.size() - 1; i > 0; --i) std::swap(order[i], order[splitmix64(rs) % (i + 1)]);
    CnnImpl& net = *c->impl;
    auto loss_of = [&](const std::pair<int, int>& pr) {
        SolverImpl& S = *solvers[pr.first]->impl;
        const LevelDev& l0 = *S.lev[0];
        const cx<double>* r = (const cx<double>*)samples[pr.first] + (size_t)pr.second * l0.N;
        return net.loss_grad(l0.n2, l0.n1, r, S.feat.as<float>(), l0.Dinv64.as<cx<double>>(), l0.omega,
                             finest_mbeta(S, st), st);
    };
    auto mean_loss = [&]() {
        double sum = 0.0;
        for (const auto& pr : pairs) sum += loss_of(pr);
        return sum / (double)pairs.size();
    };
    const double l0 = mean_loss();
    for (int it = 0; it < steps; ++it) {
        const double L = loss_of(pairs[order[it % order.size()]]);
        if (!std::isfinite(L)) throw Err{HH_ENUMERIC, "training loss is not finite"};
        net.adam_step(lr, st);
    }
    const double l1 = mean_loss();
    HH_HIP(hipStreamSynchronize(st));
    if (loss_before) *loss_before = l0;
    if (loss_after) *loss_after = l1;
    if (out_weights) save_weights(net, out_weights);
    return HH_OK;
    HH_CATCH
}

hh_status hh_cnn_save(const hh_cnn* c, const char* path) {
    HH_TRY
    if (!c || !path) throw Err{HH_EINVAL, "NULL argument"};
    save_weights(*c->impl, path);
    return HH_OK;
    HH_CATCH
}

hh_status hh_cnn_load(const char* path, hh_cnn** out) {
    HH_TRY
    if (!path || !out) throw Err{HH_EINVAL, "NULL argument"};
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) throw Err{HH_EINVAL, std::string("cannot open ") + path};
    char magic[8] = {0};
    int32_t n = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kWeightMagic, 8) == 0 &&
              std::fread(&n, 4, 1, f) == 1 && n > 0 && n <= (1 << 24);
    std::vector<float> v(ok ? (size_t)n : 0);
    uint64_t sum = 0;
    ok = ok && std::fread(v.data(), 4, v.size(), f) == v.size() && std::fread(&sum, 8, 1, f) == 1 &&
         std::fgetc(f) == EOF;
    std::fclose(f);
    if (!ok) throw Err{HH_EINVAL, std::string(path) + " is not a weight file of this library"};
    if (fnv1a((const unsigned char*)v.data(), v.size() * 4) != sum)
        throw Err{HH_EINVAL, std::string(path) + ": checksum mismatch"};
    auto net = std::make_unique<CnnImpl>(0ull);
    if (n != 2 * net->nparam) throw Err{HH_EINVAL, std::string(path) + ": parameter count of another network"};
    net->set_params(v.data(), n);
    auto* c = new hh_cnn();
    c->impl = std::move(net);
    *out = c;
    return HH_OK;
    HH_CATCH
}

hh_status hh_solver_set_smoother(hh_solver* s, hh_cnn* c) {
    HH_TRY
    if (!s) throw Err{HH_EINVAL, "NULL solver"};
    if (c && s->impl->prob->dim == 3) throw Err{HH_EINVAL, "the learned smoother is built for 1D and 2D problems"};
    s->impl->cnn = c ? c->impl.get() : nullptr;
    s->impl->drop_graphs();   // the smoother changes the captured step
    return HH_OK;
    HH_CATCH
}

hh_status hh_solver_capture(hh_solver* s, void* buf, int max_samples) {
    HH_TRY
    if (!s) throw Err{HH_EINVAL, "NULL solver"};
    if (buf && max_samples < 1) throw Err{HH_EINVAL, "max_samples must be >= 1"};
    s->impl->cap_buf = (cx<double>*)buf;
    s->impl->cap_max = buf ? max_samples : 0;
    if (buf) s->impl->cap_n = 0;  // a new capture starts empty; stopping keeps the count
    return HH_OK;
    HH_CATCH
}

hh_status hh_solver_captured(const hh_solver* s, int* n) {
    HH_TRY
    if (!s || !n) throw Err{HH_EINVAL, "NULL argument"};
    *n = s->impl->cap_n;
    return HH_OK;
    HH_CATCH
}

hh_status hh_set_kernel_timing(hh_solver* s, int cls) {
    HH_TRY
    if (!s) throw Err{HH_EINVAL, "NULL solver"};
    if (cls < 0 || cls > 5) throw Err{HH_EINVAL, "timing class must be 0..5"};
    s->impl->o.time_kernels = cls;
    return HH_OK;
    HH_CATCH
}

hh_status hh_debug_set_spin_limit(hh_solver* s, int spins) {
    HH_TRY
    if (!s) throw Err{HH_EINVAL, "NULL solver"};
    if (spins < 0) throw Err{HH_EINVAL, "spins must be >= 0"};
    s->impl->set_spin_limit(spins == 0 ? kSpinLimit : spins);
    return HH_OK;
    HH_CATCH
}

hh_status hh_solve_history(const hh_solver* s, double* out, int capacity, int* n) {
    HH_TRY
    if (!s || !n) throw Err{HH_EINVAL, "NULL argument"};
    if (capacity < 0) throw Err{HH_EINVAL, "capacity must be >= 0"};
    const std::vector<double>& h = s->impl->last_hist;
    *n = (int)h.size();
    if (out) std::copy(h.begin(), h.begin() + std::min<size_t>(h.size(), (size_t)capacity), out);
    return HH_OK;
    HH_CATCH
}

hh_status hh_level_info(const hh_solver* s, int level, hh_level_stats* out) {
    HH_TRY
    if (!s || !out) throw Err{HH_EINVAL, "NULL argument"};
    const SolverImpl& S = *s->impl;
    if (level < 0 || (level > S.L && !(S.zadp && level == S.Lz))) throw Err{HH_EINVAL, "level out of range"};
    const LevelDev& lv = *S.lev[level];
    out->n[0] = lv.n1;
    out->n[1] = lv.n2;
    out->n_el[0] = lv.ax.nel;
    out->n_el[1] = lv.ay.nel;
    out->N = lv.N;
    out->omega = lv.omega;
    out->gersh = lv.gersh;
    out->n_levels = S.L + 1;
    out->defl_direct_level = S.Lz;
    out->op_rows[0] = lv.ty64;
    out->op_rows[1] = lv.ty32;
    const bool sub_here = S.sub && level == S.Lz;
    out->defl_sub[0] = sub_here ? S.sub->bx : 0;
    out->defl_sub[1] = sub_here ? S.sub->by : 0;
    out->defl_sep = sub_here ? S.sub->nS : 0;
    out->defl_check = sub_here ? S.sub->self_check : -1.0;
    out->defl_refine = sub_here ? S.sub->refine : 0;
    out->n_z = lv.n3;
    out->n_el_z = lv.az.nel;
    return HH_OK;
    HH_CATCH
}

hh_status hh_apply(hh_solver* s, int op, int level, const void* x_dev, void* y_dev, void* stream) {
    HH_TRY
    if (!s || !x_dev || !y_dev) throw Err{HH_EINVAL, "NULL argument"};
    if (x_dev == y_dev) throw Err{HH_EINVAL, "x and y must not alias"};
    SolverImpl& S = *s->impl;
    hipStream_t st = (hipStream_t)stream;
    // the ADP deflation level (outside the multigrid hierarchy) takes its own
    // operators and E^-1 only
    const bool adp_level = S.zadp && level == S.Lz;
    if (level < 0 || (level > S.L && !adp_level)) throw Err{HH_EINVAL, "level out of range"};
    if (adp_level && op != HH_OP_A && op != HH_OP_K && op != HH_OP_MK && op != HH_OP_EINV)
        throw Err{HH_EINVAL, "the ADP deflation level takes A, K, M_k and E^-1 only"};
    auto x = (const cx<double>*)x_dev;
    auto y = (cx<double>*)y_dev;
    LevelDev& lv = *S.lev[level];
    switch (op) {
        case HH_OP_A: S.op<double>(level, MODE_APPLY, false, x, nullptr, y, st); break;
        case HH_OP_MBETA: S.op<double>(level, MODE_APPLY, true, x, nullptr, y, st); break;
        case HH_OP_JACOBI0:
            launch_jacobi0<double>(lv.N, lv.Dinv64.as<cx<double>>(), lv.omega, x, y, st);
            break;
        case HH_OP_RESTRICT:
            if (level >= S.L) throw Err{HH_EINVAL, "no coarser level"};
            launch_restrict<double>(lv.tr, x, y, st);
            break;
        case HH_OP_PROLONG:
            if (level >= S.L) throw Err{HH_EINVAL, "no coarser level"};
            launch_prolong<double>(lv.tr, x, y, 0, st);
            break;
        case HH_OP_VCYCLE: S.precond_vcycle(level, x, y, st); break;
        case HH_OP_T: S.T_apply(level, x, y, st); break;
        case HH_OP_K: S.op_alpha<double>(level, MODE_APPLY, 0.0, 0.0, x, nullptr, y, st, nullptr, nullptr, false); break;
        case HH_OP_MK:
            S.op_alpha<double>(level, MODE_APPLY, -1.0, 0.0, x, nullptr, y, st, nullptr, nullptr, false, true);
            break;
        case HH_OP_ZT:
        case HH_OP_Z: {
            if (S.Lz == 0 || level >= S.defl_end()) throw Err{HH_EINVAL, "no deflation level below this one"};
            const Transfer& tr = S.zadp ? S.ztr : lv.tr;
            if (op == HH_OP_ZT)
                launch_restrict<double>(tr, x, y, st);
            else
                launch_prolong<double>(tr, x, y, 0, st);
            break;
        }
        case HH_OP_EINV:
            if (S.Lz == 0 || level < 1 || level > S.Lz || (S.zadp && level != S.Lz))
                throw Err{HH_EINVAL, "not a deflation level"};
            S.coarse_solve(level, x, y, st);
            break;
        default: throw Err{HH_EINVAL, "unknown operator"};
    }
    HH_HIP(hipGetLastError());
    HH_HIP(hipStreamSynchronize(st));
    return HH_OK;
    HH_CATCH
}

}  // extern "C"
