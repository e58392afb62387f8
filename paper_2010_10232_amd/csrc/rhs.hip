// Point-source load on the device (MP 1-B, MP 2-A, MP 2-B: the Galerkin load of
// amp * delta(x - x0) is f_i = amp * Phi_i(x0), section 2.3).  Phi_i is a tensor
// product, so the host evaluates the p + 1 nonzero B-splines per direction at
// x0 (a few flops), stages the 1D factor vectors fx[n1], fy[n2] (and fz[n3] on
// the unit cube) in device memory, and one kernel writes
// f[i3][i2][i1] = ((amp * fz[i3]) * fy[i2]) * fx[i1] over the whole grid (fz = 1
// without a z direction).  Only n1 + n2 (+ n3) values cross the host link
// instead of N.
#include <cmath>
#include <mutex>

#include "solver.h"

namespace hh {

namespace {

__global__ void __launch_bounds__(256) point_source_kernel(int n1, int n2, int has_z, long long N,
                                                            const double* __restrict__ stage, double amp,
                                                            cx<double>* __restrict__ f) {
    const double* fx = stage;
    const double* fy = stage + n1;
    const double* fz = stage + n1 + n2;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const long long i23 = i / n1;
        const int i1 = (int)(i - i23 * n1);
        const int i3 = (int)(i23 / n2);
        const int i2 = (int)(i23 - (long long)i3 * n2);
        const double az = has_z ? amp * fz[i3] : amp;
        f[i] = cx<double>{az * fy[i2] * fx[i1], 0.0};
    }
}

int span_of(double x, int nel) {
    int e = (int)std::floor(x * nel);
    return e < nel - 1 ? e : nel - 1;
}

// Staged values: n1 + n2, and n3 more on the unit cube.
int stage_size(const ProblemImpl& P) { return P.ax0.n + P.ay0.n + (P.dim == 3 ? P.az0.n : 0); }

// The 1D factors of Phi(x0) over the interior unknowns: stage[0..n1) in x,
// stage[n1..n1+n2) in y (1D problems: fy = [1]), stage[n1+n2..n1+n2+n3) in z on
// the unit cube.  stage must hold stage_size(P) doubles; everything but the
// p + 1 supported entries per direction is zero.
void point_factors(const ProblemImpl& P, const double* x0, double* stage) {
    const int n1 = P.ax0.n, n2 = P.ay0.n, p = P.p;
    for (int i = 0; i < stage_size(P); ++i) stage[i] = 0.0;
    double Nv[8];
    const int s1 = span_of(x0[0] / P.len[0], P.nel[0]);
    basis_values(P.ax0.U, p, s1 + p, x0[0], Nv, nullptr);
    for (int a = 0; a <= p; ++a) {
        const int i = s1 + a - 1;
        if (i >= 0 && i < n1) stage[i] = Nv[a];
    }
    if (P.dim >= 2) {
        const int s2 = span_of(x0[1] / P.len[1], P.nel[1]);
        basis_values(P.ay0.U, p, s2 + p, x0[1], Nv, nullptr);
        for (int a = 0; a <= p; ++a) {
            const int i = s2 + a - 1;
            if (i >= 0 && i < n2) stage[n1 + i] = Nv[a];
        }
    } else {
        stage[n1] = 1.0;
    }
    if (P.dim == 3) {
        const int n3 = P.az0.n;
        const int s3 = span_of(x0[2] / P.len[2], P.nel[2]);
        basis_values(P.az0.U, p, s3 + p, x0[2], Nv, nullptr);
        for (int a = 0; a <= p; ++a) {
            const int i = s3 + a - 1;
            if (i >= 0 && i < n3) stage[n1 + n2 + i] = Nv[a];
        }
    }
}

void check_point(const ProblemImpl& P, const double* x0) {
    for (int d = 0; d < P.dim; ++d)
        HH_REQUIRE(x0[d] >= 0.0 && x0[d] <= P.len[d], "source point outside the domain");
}

void launch_point_source(const ProblemImpl& P, const double* stage_dev, double amp, cx<double>* f,
                         hipStream_t s) {
    const long long N = P.N();
    const int blocks = (int)std::min<long long>((N + 255) / 256, 8192);
    point_source_kernel<<<blocks, 256, 0, s>>>(P.ax0.n, P.ay0.n, P.dim == 3 ? 1 : 0, N, stage_dev, amp, f);
    HH_HIP(hipGetLastError());
}

// ---- allocation-free variant: the staging lives in a fixed device array ----
// Capacity of the staging array in doubles (n1 + n2 (+ n3) of the finest level).
constexpr int kStageMax = 65536;
static __device__ __align__(256) double scratch[kStageMax];
// In host code `scratch` names a host-side stand-in; its device address is
// looked up once per device and kept here.
constexpr int kMaxDevices = 64;
double* g_scratch_dev[kMaxDevices] = {};
std::mutex g_scratch_mu;           // guards the lookup table and the host staging below
double g_stage_host[kStageMax];    // host staging of the no-alloc path (no heap use)

double* scratch_on_current_device() {
    int dev = -1;
    HH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Err{HH_EINVAL, "device index beyond the supported range"};
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        HH_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Err{HH_EHIP, "no device address for the staging array"};
        g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_dev[dev];
}

}  // namespace

// Regular path: the staging buffer is allocated by the library for the call.
void rhs_point_source(const ProblemImpl& P, const double* x0, double amp, cx<double>* f, hipStream_t s) {
    check_point(P, x0);
    const int n = stage_size(P);
    std::vector<double> stage((size_t)n);
    point_factors(P, x0, stage.data());
    DevBuf d;
    d.alloc((size_t)n * sizeof(double));
    HH_HIP(hipMemcpyAsync(d.p, stage.data(), (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
    launch_point_source(P, d.as<double>(), amp, f, s);
    HH_HIP(hipStreamSynchronize(s));
}

// No-alloc path: the same kernel reading the fixed array; no device or heap
// allocation.  Calls overlapping on one device share the array and race.
void rhs_point_source_noalloc(const ProblemImpl& P, const double* x0, double amp, cx<double>* f, hipStream_t s) {
    check_point(P, x0);
    const int n = stage_size(P);
    if (n > kStageMax)
        throw Err{HH_EINVAL, "n1 + n2 (+ n3) = " + std::to_string(n) + " exceeds the staging capacity of " +
                                 std::to_string(kStageMax) + " values"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    double* stage_dev = scratch_on_current_device();
    point_factors(P, x0, g_stage_host);
    HH_HIP(hipMemcpyAsync(stage_dev, g_stage_host, (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
    launch_point_source(P, stage_dev, amp, f, s);
    HH_HIP(hipStreamSynchronize(s));
}

// MP 1-A: the boundary value u(0) = u0 carried by the eliminated first basis
// function, moved to the right-hand side: f_{j-1} = -u0 (K - k^2 M)_{j,0} for the
// functions j = 1..p that share the first element with it (zero elsewhere).
void rhs_dirichlet_lift(const ProblemImpl& P, double u0, cx<double>* f, hipStream_t s) {
    if (!P.somm) throw Err{HH_EINVAL, "the Dirichlet lift is defined for problems with bc_right = 1"};
    if (!std::isfinite(u0)) throw Err{HH_EINVAL, "u0 must be finite"};
    const Axis& a = P.ax0;
    std::vector<cx<double>> h((size_t)a.n, cx<double>{0.0, 0.0});
    const double k2 = P.k * P.k;
    for (int j = 1; j <= P.p && j - 1 < a.n; ++j) h[j - 1] = {-u0 * (a.K0[j] - k2 * a.M0[j]), 0.0};
    HH_HIP(hipMemcpyAsync(f, h.data(), h.size() * sizeof(cx<double>), hipMemcpyHostToDevice, s));
    HH_HIP(hipStreamSynchronize(s));
}

}  // namespace hh
