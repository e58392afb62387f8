// HIP kernels for gfx950 (CDNA4, wave64): knot-insertion transfers, pointwise
// updates, dense products of the direct coarse solves, and the deterministic
// reductions of the Arnoldi process.  The level-operator kernels are in
// op_kernel.h.
#include <algorithm>
#include <climits>
#include <map>
#include <mutex>
#include <type_traits>

#include "hh_internal.h"

namespace hh {

template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// --------------------------------------------------------------------------
// Level operator: kernels live in op_kernel.h, one translation unit per degree.
// --------------------------------------------------------------------------
template <class T>
void launch_op(int kind, int mode, int px, int py, const OpArgs<T>& a, hipStream_t s) {
    if (a.n3 > 0) {
        if (kind != KIND_SEP || py != px) throw Err{HH_EINVAL, "3D levels are constant-k with one degree"};
        return launch_op3d<T>(mode, px, a, s);
    }
    if (a.n1 <= 0 || a.n2 <= 0) return;
    if (py != 0 && py != px) throw Err{HH_EINVAL, "unsupported degree pair"};
    switch (px) {
        case 1: return launch_op_deg<1, T>(kind, mode, py, a, s);
        case 2: return launch_op_deg<2, T>(kind, mode, py, a, s);
        case 3: return launch_op_deg<3, T>(kind, mode, py, a, s);
        case 4: return launch_op_deg<4, T>(kind, mode, py, a, s);
        case 5: return launch_op_deg<5, T>(kind, mode, py, a, s);
    }
    throw Err{HH_EINVAL, "unsupported degree"};
}
template void launch_op<double>(int, int, int, int, const OpArgs<double>&, hipStream_t);
template void launch_op<float>(int, int, int, int, const OpArgs<float>&, hipStream_t);

// --------------------------------------------------------------------------
// Knot-insertion transfers: restriction c = P^T r, prolongation x (+)= P e,
// P = P_y (x) P_x stored as per-row / per-column runs.
// --------------------------------------------------------------------------
// W = 0: loops over the run widths as stored.  W > 0 (a bound on the widths,
// known at compile time): unrolled loops over W entries with clamped,
// always-valid addresses and zero weights past the run, so the loads of a
// thread can be in flight at once; the terms are added in the same order.
// FULL = false unrolls the inner loop only (fewer registers, for the
// 1024-thread tail workgroup).
template <class T, int W = 0, bool FULL = true>
__device__ __forceinline__ cx<T> restrict_one(const Transfer& t, const cx<T>* __restrict__ r, int idx) {
    const int J1 = idx % t.nc1, J2 = idx / t.nc1;
    const int i0x = t.pcol0x[J1], i0y = t.pcol0y[J2];
    T sr = 0, si = 0;
    if constexpr (W == 0) {
        for (int a2 = 0; a2 < t.rw2; ++a2) {
            const T wy = (T)t.pcoly[(size_t)J2 * t.rw2 + a2];
            if (wy == T(0)) continue;
            const cx<T>* row = r + (size_t)(i0y + a2) * t.nf1 + i0x;
            T rr = 0, ri = 0;
            for (int a1 = 0; a1 < t.rw1; ++a1) {
                const T wx = (T)t.pcolx[(size_t)J1 * t.rw1 + a1];
                const cx<T> v = row[a1];
                rr += wx * v.re;
                ri += wx * v.im;
            }
            sr += wy * rr;
            si += wy * ri;
        }
    } else {
        T wx[W], wy[W];
#pragma unroll
        for (int a = 0; a < W; ++a) {
            const T vx = (T)t.pcolx[(size_t)J1 * t.rw1 + min(a, t.rw1 - 1)];
            const T vy = (T)t.pcoly[(size_t)J2 * t.rw2 + min(a, t.rw2 - 1)];
            wx[a] = a < t.rw1 ? vx : T(0);
            wy[a] = a < t.rw2 ? vy : T(0);
        }
#pragma unroll FULL ? W : 1
        for (int a2 = 0; a2 < W; ++a2) {
            const cx<T>* row = r + (size_t)(i0y + min(a2, t.rw2 - 1)) * t.nf1 + i0x;
            T rr = 0, ri = 0;
#pragma unroll
            for (int a1 = 0; a1 < W; ++a1) {
                const cx<T> v = row[min(a1, t.rw1 - 1)];
                rr += wx[a1] * v.re;
                ri += wx[a1] * v.im;
            }
            sr += wy[a2] * rr;
            si += wy[a2] * ri;
        }
    }
    return {sr, si};
}

template <class T, int W = 0, bool FULL = true>
__device__ __forceinline__ cx<T> prolong_one(const Transfer& t, const cx<T>* __restrict__ e, int idx) {
    const int I1 = idx % t.nf1, I2 = idx / t.nf1;
    const int j0x = t.prow0x[I1], j0y = t.prow0y[I2];
    T sr = 0, si = 0;
    if constexpr (W == 0) {
        for (int b2 = 0; b2 < t.pw2; ++b2) {
            const T wy = (T)t.prowy[(size_t)I2 * t.pw2 + b2];
            if (wy == T(0)) continue;
            const cx<T>* row = e + (size_t)(j0y + b2) * t.nc1 + j0x;
            T rr = 0, ri = 0;
            for (int b1 = 0; b1 < t.pw1; ++b1) {
                const T wx = (T)t.prowx[(size_t)I1 * t.pw1 + b1];
                const cx<T> v = row[b1];
                rr += wx * v.re;
                ri += wx * v.im;
            }
            sr += wy * rr;
            si += wy * ri;
        }
    } else {
        T wx[W], wy[W];
#pragma unroll
        for (int b = 0; b < W; ++b) {
            const T vx = (T)t.prowx[(size_t)I1 * t.pw1 + min(b, t.pw1 - 1)];
            const T vy = (T)t.prowy[(size_t)I2 * t.pw2 + min(b, t.pw2 - 1)];
            wx[b] = b < t.pw1 ? vx : T(0);
            wy[b] = b < t.pw2 ? vy : T(0);
        }
#pragma unroll FULL ? W : 1
        for (int b2 = 0; b2 < W; ++b2) {
            const cx<T>* row = e + (size_t)(j0y + min(b2, t.pw2 - 1)) * t.nc1 + j0x;
            T rr = 0, ri = 0;
#pragma unroll
            for (int b1 = 0; b1 < W; ++b1) {
                const cx<T> v = row[min(b1, t.pw1 - 1)];
                rr += wx[b1] * v.re;
                ri += wx[b1] * v.im;
            }
            sr += wy[b2] * rr;
            si += wy[b2] * ri;
        }
    }
    return {sr, si};
}

// (level sizes below 2^31 unknowns, checked by the launchers: 32-bit indices)
// dinv != nullptr: also the coarse level's first damped Jacobi sweep from zero,
// xs = omega D^-1 c, formed exactly as jacobi0_kernel forms it.
template <class T, int W>
__global__ void restrict_kernel(Transfer t, const cx<T>* __restrict__ r, cx<T>* __restrict__ c,
                                const cx<T>* __restrict__ dinv, T omega, cx<T>* __restrict__ xs) {
    const int idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= t.nc1 * t.nc2) return;
    const cx<T> v = restrict_one<T, W>(t, r, idx);
    c[idx] = v;
    if (dinv) {
        const cx<T> d = dinv[idx];
        xs[idx] = {omega * (d.re * v.re - d.im * v.im), omega * (d.re * v.im + d.im * v.re)};
    }
}

// x = xin + P e (xin may alias x; xin == nullptr: x = P e)
template <class T, int W>
__global__ void prolong_kernel(Transfer t, const cx<T>* __restrict__ e, const cx<T>* xin, cx<T>* x) {
    const int idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= t.nf1 * t.nf2) return;
    const cx<T> v = prolong_one<T, W>(t, e, idx);
    if (xin) {
        const cx<T> o = xin[idx];
        x[idx] = {o.re + v.re, o.im + v.im};
    } else {
        x[idx] = v;
    }
}

static inline unsigned grid1d(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// The unrolled forms for run widths up to 7 (degree 5: restriction runs of
// p + 2, prolongation runs of p + 1); wider runs take the loop form.
template <class T>
static const void* restrict_fn(int w) {
    switch (w) {
        case 1: return (const void*)restrict_kernel<T, 1>;
        case 2: return (const void*)restrict_kernel<T, 2>;
        case 3: return (const void*)restrict_kernel<T, 3>;
        case 4: return (const void*)restrict_kernel<T, 4>;
        case 5: return (const void*)restrict_kernel<T, 5>;
        case 6: return (const void*)restrict_kernel<T, 6>;
        case 7: return (const void*)restrict_kernel<T, 7>;
    }
    return (const void*)restrict_kernel<T, 0>;
}
template <class T>
static const void* prolong_fn(int w) {
    switch (w) {
        case 1: return (const void*)prolong_kernel<T, 1>;
        case 2: return (const void*)prolong_kernel<T, 2>;
        case 3: return (const void*)prolong_kernel<T, 3>;
        case 4: return (const void*)prolong_kernel<T, 4>;
        case 5: return (const void*)prolong_kernel<T, 5>;
        case 6: return (const void*)prolong_kernel<T, 6>;
        case 7: return (const void*)prolong_kernel<T, 7>;
    }
    return (const void*)prolong_kernel<T, 0>;
}

thread_local Meter* g_meter = nullptr;

template <class T>
void launch_restrict(const Transfer& t, const cx<T>* r, cx<T>* c, hipStream_t s, const cx<T>* dinv, T omega,
                     cx<T>* xs) {
    if (t.nf3 > 0) return launch_restrict3<T>(t, r, c, s, dinv, omega, xs);
    const long long Nc = (long long)t.nc1 * t.nc2;
    if (Nc <= 0) return;
    meter(sizeof(cx<T>) * ((double)t.nf1 * t.nf2 + Nc * (dinv ? 3.0 : 1.0)),
          4.0 * t.rw1 * t.rw2 * (double)Nc + (dinv ? 8.0 * Nc : 0.0));
    if (Nc > INT_MAX || (long long)t.nf1 * t.nf2 > INT_MAX) throw Err{HH_EINVAL, "level too large for a transfer"};
    void* args[] = {(void*)&t, (void*)&r, (void*)&c, (void*)&dinv, (void*)&omega, (void*)&xs};
    HH_HIP(hipLaunchKernel(restrict_fn<T>(std::max(t.rw1, t.rw2)), dim3(grid1d(Nc, 256)), dim3(256), args, 0, s));
}
template <class T>
void launch_prolong_add(const Transfer& t, const cx<T>* e, const cx<T>* xin, cx<T>* xout, hipStream_t s) {
    if (t.nf3 > 0) return launch_prolong_add3<T>(t, e, xin, xout, s);
    const long long Nf = (long long)t.nf1 * t.nf2;
    if (Nf <= 0) return;
    meter(sizeof(cx<T>) * ((double)t.nc1 * t.nc2 + Nf * (xin ? 2.0 : 1.0)),
          4.0 * t.pw1 * t.pw2 * (double)Nf + (xin ? 2.0 * Nf : 0.0));
    if (Nf > INT_MAX || (long long)t.nc1 * t.nc2 > INT_MAX) throw Err{HH_EINVAL, "level too large for a transfer"};
    void* args[] = {(void*)&t, (void*)&e, (void*)&xin, (void*)&xout};
    HH_HIP(hipLaunchKernel(prolong_fn<T>(std::max(t.pw1, t.pw2)), dim3(grid1d(Nf, 256)), dim3(256), args, 0, s));
}
template <class T>
void launch_prolong(const Transfer& t, const cx<T>* e, cx<T>* x, int add, hipStream_t s) {
    launch_prolong_add<T>(t, e, add ? x : nullptr, x, s);
}
template void launch_restrict<double>(const Transfer&, const cx<double>*, cx<double>*, hipStream_t, const cx<double>*,
                                      double, cx<double>*);
template void launch_restrict<float>(const Transfer&, const cx<float>*, cx<float>*, hipStream_t, const cx<float>*,
                                     float, cx<float>*);
template void launch_prolong<double>(const Transfer&, const cx<double>*, cx<double>*, int, hipStream_t);
template void launch_prolong_add<double>(const Transfer&, const cx<double>*, const cx<double>*, cx<double>*, hipStream_t);
template void launch_prolong<float>(const Transfer&, const cx<float>*, cx<float>*, int, hipStream_t);
template void launch_prolong_add<float>(const Transfer&, const cx<float>*, const cx<float>*, cx<float>*, hipStream_t);

// --------------------------------------------------------------------------
// Pointwise kernels
// --------------------------------------------------------------------------
template <class T>
__global__ void jacobi0_kernel(long long N, const cx<T>* dinv, T omega, const cx<T>* b, cx<T>* x) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const cx<T> d = dinv[i], v = b[i];
    x[i] = {omega * (d.re * v.re - d.im * v.im), omega * (d.re * v.im + d.im * v.re)};
}
template <class T>
void launch_jacobi0(long long N, const cx<T>* dinv, T omega, const cx<T>* b, cx<T>* x, hipStream_t s) {
    meter(3.0 * sizeof(cx<T>) * N, 8.0 * N);
    hipLaunchKernelGGL(jacobi0_kernel<T>, dim3(grid1d(N, 256)), dim3(256), 0, s, N, dinv, omega, b, x);
}
template void launch_jacobi0<double>(long long, const cx<double>*, double, const cx<double>*, cx<double>*, hipStream_t);
template void launch_jacobi0<float>(long long, const cx<float>*, float, const cx<float>*, cx<float>*, hipStream_t);

template <class T>
__global__ void axpy_kernel(long long N, const cx<T>* x, cx<T>* y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const cx<T> a = x[i], b = y[i];
    y[i] = {b.re + a.re, b.im + a.im};
}
template <class T>
void launch_axpy(long long N, const cx<T>* x, cx<T>* y, hipStream_t s) {
    meter(3.0 * sizeof(cx<T>) * N, 2.0 * N);
    hipLaunchKernelGGL(axpy_kernel<T>, dim3(grid1d(N, 256)), dim3(256), 0, s, N, x, y);
}
template void launch_axpy<double>(long long, const cx<double>*, cx<double>*, hipStream_t);
template void launch_axpy<float>(long long, const cx<float>*, cx<float>*, hipStream_t);

__global__ void add_kernel(long long N, const cx<double>* a, const cx<double>* b, cx<double>* y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const cx<double> u = a[i], v = b[i];
    y[i] = {u.re + v.re, u.im + v.im};
}
void launch_add(long long N, const cx<double>* a, const cx<double>* b, cx<double>* y, hipStream_t s) {
    meter(48.0 * N, 2.0 * N);
    hipLaunchKernelGGL(add_kernel, dim3(grid1d(N, 256)), dim3(256), 0, s, N, a, b, y);
}

__global__ void copy_kernel(long long N, const cx<double>* x, cx<double>* y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = x[i];
}
void launch_copy(long long N, const cx<double>* x, cx<double>* y, hipStream_t s) {
    meter(32.0 * N, 0.0);
    hipLaunchKernelGGL(copy_kernel, dim3(grid1d(N, 256)), dim3(256), 0, s, N, x, y);
}
__global__ void zero_kernel(long long N, cx<double>* y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = {0.0, 0.0};
}
void launch_zero(long long N, cx<double>* y, hipStream_t s) {
    meter(16.0 * N, 0.0);
    hipLaunchKernelGGL(zero_kernel, dim3(grid1d(N, 256)), dim3(256), 0, s, N, y);
}

__global__ void cast_d2f_kernel(long long N, const cx<double>* x, cx<float>* y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = {(float)x[i].re, (float)x[i].im};
}
__global__ void cast_f2d_kernel(long long N, const cx<float>* x, cx<double>* y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = {(double)x[i].re, (double)x[i].im};
}
void launch_cast_d2f(long long N, const cx<double>* x, cx<float>* y, hipStream_t s) {
    meter(24.0 * N, 0.0);
    hipLaunchKernelGGL(cast_d2f_kernel, dim3(grid1d(N, 256)), dim3(256), 0, s, N, x, y);
}
void launch_cast_f2d(long long N, const cx<float>* x, cx<double>* y, hipStream_t s) {
    meter(24.0 * N, 0.0);
    hipLaunchKernelGGL(cast_f2d_kernel, dim3(grid1d(N, 256)), dim3(256), 0, s, N, x, y);
}
__global__ void cast_f2d_add_kernel(long long N, const cx<float>* x, const cx<double>* q, cx<double>* y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = {(double)x[i].re + q[i].re, (double)x[i].im + q[i].im};
}
void launch_cast_f2d_add(long long N, const cx<float>* x, const cx<double>* q, cx<double>* y, hipStream_t s) {
    meter(40.0 * N, 2.0 * N);
    hipLaunchKernelGGL(cast_f2d_add_kernel, dim3(grid1d(N, 256)), dim3(256), 0, s, N, x, q, y);
}

// --------------------------------------------------------------------------
// Dense matrix-vector product y = A x (A row-major n x n): one wave per row.
// --------------------------------------------------------------------------
template <class TV>
__device__ __forceinline__ void mac(const double& a, const cx<TV>& x, TV& sr, TV& si) {
    sr += (TV)a * x.re;
    si += (TV)a * x.im;
}
template <class TV, class TA>
__device__ __forceinline__ void mac(const cx<TA>& a, const cx<TV>& x, TV& sr, TV& si) {
    sr += (TV)a.re * x.re - (TV)a.im * x.im;
    si += (TV)a.re * x.im + (TV)a.im * x.re;
}

template <class TM, class TV>
__global__ __launch_bounds__(256) void gemv_kernel(int n, long long ld, const TM* __restrict__ A,
                                                   const cx<TV>* __restrict__ x, cx<TV>* __restrict__ y) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row = blockIdx.x * 4 + wave;
    if (row >= n) return;
    TV sr = 0, si = 0;
    const TM* a = A + (size_t)row * ld;
    for (int j = lane; j < n; j += 64) mac(a[j], x[j], sr, si);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sr += __shfl_xor(sr, o, 64);
        si += __shfl_xor(si, o, 64);
    }
    if (lane == 0) y[row] = {sr, si};
}
// Real FP64 matrix (leading dimension ld, even) times complex vector for
// large n (the dense E^-1 of a variable-k deflation level): each wave streams
// four rows at once with 16-byte loads (two columns per lane and step), so
// every load of x feeds four rows; per row, lane-strided partial sums then a
// butterfly (fixed order).
constexpr int GEMV_RPW = 4;
__global__ __launch_bounds__(256) void gemv4_kernel(int n, long long ld, const double* __restrict__ A,
                                                    const cx<double>* __restrict__ x, cx<double>* __restrict__ y) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long r0 = ((long long)blockIdx.x * 4 + wave) * GEMV_RPW;
    if (r0 >= n) return;
    const double* a[GEMV_RPW];
#pragma unroll
    for (int q = 0; q < GEMV_RPW; ++q) a[q] = A + (size_t)min(r0 + q, (long long)n - 1) * ld;
    double sr[GEMV_RPW], si[GEMV_RPW];
#pragma unroll
    for (int q = 0; q < GEMV_RPW; ++q) sr[q] = si[q] = 0.0;
    const int n2 = n & ~1;   // columns handled in pairs; an odd last column separately
#pragma unroll 2
    for (int j = 2 * lane; j < n2; j += 128) {
        const cx<double> x0 = x[j], x1 = x[j + 1];
#pragma unroll
        for (int q = 0; q < GEMV_RPW; ++q) {
            const double2 v = *(const double2*)(a[q] + j);
            sr[q] += v.x * x0.re + v.y * x1.re;
            si[q] += v.x * x0.im + v.y * x1.im;
        }
    }
    if ((n & 1) && lane == 0) {
        const cx<double> xl = x[n - 1];
#pragma unroll
        for (int q = 0; q < GEMV_RPW; ++q) {
            sr[q] += a[q][n - 1] * xl.re;
            si[q] += a[q][n - 1] * xl.im;
        }
    }
#pragma unroll
    for (int q = 0; q < GEMV_RPW; ++q) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            sr[q] += __shfl_xor(sr[q], o, 64);
            si[q] += __shfl_xor(si[q], o, 64);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < GEMV_RPW; ++q)
            if (r0 + q < n) y[r0 + q] = {sr[q], si[q]};
    }
}

template <class TM, class TV>
void launch_gemv(int n, const TM* A, const cx<TV>* x, cx<TV>* y, hipStream_t s) {
    meter((double)sizeof(TM) * n * n + 2.0 * sizeof(cx<TV>) * n, 8.0 * n * (double)n);
    hipLaunchKernelGGL((gemv_kernel<TM, TV>), dim3((n + 3) / 4), dim3(256), 0, s, n, (long long)n, A, x, y);
}
void launch_gemv_real(int n, long long ld, const double* A, const cx<double>* x, cx<double>* y, hipStream_t s) {
    meter(8.0 * n * (double)n + 32.0 * n, 4.0 * n * (double)n);
    if (n >= 1024 && ld % 2 == 0) {
        const long long rows_per_block = 4LL * GEMV_RPW;
        hipLaunchKernelGGL(gemv4_kernel, dim3((unsigned)((n + rows_per_block - 1) / rows_per_block)), dim3(256), 0,
                           s, n, ld, A, x, y);
    } else {
        hipLaunchKernelGGL((gemv_kernel<double, double>), dim3((n + 3) / 4), dim3(256), 0, s, n, ld, A, x, y);
    }
}
template void launch_gemv<double, double>(int, const double*, const cx<double>*, cx<double>*, hipStream_t);
template void launch_gemv<cx<double>, double>(int, const cx<double>*, const cx<double>*, cx<double>*, hipStream_t);
template void launch_gemv<cx<float>, float>(int, const cx<float>*, const cx<float>*, cx<float>*, hipStream_t);

// Exact inverse of a separable level operator E = My (x) Kx + Ky (x) Mx - k^2 My (x) Mx
// by fast diagonalisation: with Kx Vx = Mx Vx diag(lx), Vx^T Mx Vx = I (and
// likewise in y), (Vy (x) Vx)^T E (Vy (x) Vx) = diag(ly_a + lx_b - k^2), so
// E^-1 c = Vy [ (Vy^T C Vx) ./ D ] Vx^T for c viewed as the [n2][n1] matrix C.
// Four small dense passes; each output sums in a fixed order (deterministic).
// Each pass is a small complex x real matrix product Y = A B (one operand real),
// tiled 32 x 32 outputs per workgroup with K in chunks of 64 staged through
// LDS (every thread issues all of its tile loads before the first is used);
// every output sums k in increasing order.  Operand element (r, c) sits at
// base[r * sr + c * sc], which expresses the transposes.
constexpr int FDM_KC = 64;
template <bool LEFT_REAL>
__global__ __launch_bounds__(256) void fdm_gemm_kernel(int M, int N, int K, const double* __restrict__ W, int wsr,
                                                       int wsc, const cx<double>* __restrict__ X, int xsr, int xsc,
                                                       const double* __restrict__ scale,
                                                       const cx<double>* __restrict__ cscale, cx<double>* __restrict__ Y) {
    // LEFT_REAL: Ws[m][k] (32 x KC), Xs[k][n] (KC x 32); else Xs[m][k], Ws[k][n]
    constexpr int WR = LEFT_REAL ? 32 : FDM_KC, WC = LEFT_REAL ? FDM_KC : 32;
    constexpr int XR = LEFT_REAL ? FDM_KC : 32, XC = LEFT_REAL ? 32 : FDM_KC;
    __shared__ double Ws[WR][WC + 1];
    __shared__ cx<double> Xs[XR][XC + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
    double ar[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, ai[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    constexpr int PER = 32 * FDM_KC / 256;   // tile elements per thread and operand
    // tile coordinates of element e: the operand's unit-stride index runs fastest
    auto wpos = [&](int e, int& r, int& c) {
        r = (wsc == 1) ? e / WC : e % WR;
        c = (wsc == 1) ? e % WC : e / WR;
    };
    auto xpos = [&](int e, int& r, int& c) {
        r = (xsc == 1) ? e / XC : e % XR;
        c = (xsc == 1) ? e % XC : e / XR;
    };
    for (int k0 = 0; k0 < K; k0 += FDM_KC) {
        double wv[PER];
        cx<double> xv[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + 256 * q;
            int r, c;
            wpos(e, r, c);
            int gr = (LEFT_REAL ? m0 : k0) + r, gc = (LEFT_REAL ? k0 : n0) + c;
            bool ok = LEFT_REAL ? (gr < M && gc < K) : (gr < K && gc < N);
            wv[q] = ok ? W[(size_t)gr * wsr + (size_t)gc * wsc] : 0.0;
            xpos(e, r, c);
            gr = (LEFT_REAL ? k0 : m0) + r;
            gc = (LEFT_REAL ? n0 : k0) + c;
            ok = LEFT_REAL ? (gr < K && gc < N) : (gr < M && gc < K);
            xv[q] = ok ? X[(size_t)gr * xsr + (size_t)gc * xsc] : cx<double>{0.0, 0.0};
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = threadIdx.x + 256 * q;
            int r, c;
            wpos(e, r, c);
            Ws[r][c] = wv[q];
            xpos(e, r, c);
            Xs[r][c] = xv[q];
        }
        __syncthreads();
        const int kn = min(FDM_KC, K - k0);
        for (int kk = 0; kk < kn; ++kk) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int jj = 0; jj < 2; ++jj) {
                    const int m = ty + 16 * i, n = tx + 16 * jj;
                    const double a = LEFT_REAL ? Ws[m][kk] : Ws[kk][n];
                    const cx<double> x = LEFT_REAL ? Xs[kk][n] : Xs[m][kk];
                    ar[i][jj] += a * x.re;
                    ai[i][jj] += a * x.im;
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
            const int m = m0 + ty + 16 * i, n = n0 + tx + 16 * jj;
            if (m >= M || n >= N) continue;
            const size_t o = (size_t)m * N + n;
            if (cscale) {
                const cx<double> d = cscale[o];
                Y[o] = {ar[i][jj] * d.re - ai[i][jj] * d.im, ar[i][jj] * d.im + ai[i][jj] * d.re};
            } else {
                const double d = scale ? scale[o] : 1.0;
                Y[o] = {ar[i][jj] * d, ai[i][jj] * d};
            }
        }
}

// Small levels (both sides at most 128): two passes, each a pair of products
// Y[r][:] = scale[r][:] * (sum_k L(r, k) X[k][:]) R for a block of FDM2_RB
// output rows per workgroup, L and R real.  Every thread issues all its
// global loads (its column of X over a 32-long k range, its column of R over a
// 32-long j range, one element of the L rows) before any arithmetic, so a
// pass costs one memory round trip; partial sums of the k (j) ranges are
// added in range order in LDS (deterministic).
constexpr int FDM2_TB = 512, FDM2_RB = 2, FDM2_CH = 32, FDM2_NMAX = 128;
__global__ __launch_bounds__(FDM2_TB) void fdm_pass_kernel(int n2, int n1, const double* __restrict__ Lm, int lsr,
                                                           int lsc, const cx<double>* __restrict__ X,
                                                           const double* __restrict__ R,
                                                           const double* __restrict__ scale,
                                                           const cx<double>* __restrict__ cscale,
                                                           cx<double>* __restrict__ Y) {
    __shared__ double Ls[FDM2_RB][FDM2_NMAX];
    __shared__ cx<double> P[FDM2_NMAX / FDM2_CH][FDM2_RB][FDM2_NMAX];
    __shared__ cx<double> U[FDM2_RB][FDM2_NMAX];
    const int tid = threadIdx.x, r0 = blockIdx.x * FDM2_RB;
    const int g = tid / n1, col = tid % n1;               // k (or j) range g, column col
    const int G2 = (n2 + FDM2_CH - 1) / FDM2_CH, G1 = (n1 + FDM2_CH - 1) / FDM2_CH;
    cx<double> xv[FDM2_CH];
    double rv[FDM2_CH];
#pragma unroll
    for (int q = 0; q < FDM2_CH; ++q) {
        const int k = g * FDM2_CH + q;
        xv[q] = (g < G2 && k < n2) ? X[(size_t)k * n1 + col] : cx<double>{0.0, 0.0};
        rv[q] = (g < G1 && k < n1) ? R[(size_t)k * n1 + col] : 0.0;
    }
    for (int e = tid; e < FDM2_RB * FDM2_NMAX; e += FDM2_TB) {
        const int r = e / FDM2_NMAX, k = e % FDM2_NMAX, row = r0 + r;
        Ls[r][k] = (row < n2 && k < n2) ? Lm[(size_t)row * lsr + (size_t)k * lsc] : 0.0;
    }
    __syncthreads();
    if (g < G2) {
#pragma unroll
        for (int r = 0; r < FDM2_RB; ++r) {
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int q = 0; q < FDM2_CH; ++q) {
                const double l = Ls[r][g * FDM2_CH + q];
                ar += l * xv[q].re;
                ai += l * xv[q].im;
            }
            P[g][r][col] = {ar, ai};
        }
    }
    __syncthreads();
    for (int e = tid; e < FDM2_RB * FDM2_NMAX; e += FDM2_TB) {
        const int r = e / FDM2_NMAX, c = e % FDM2_NMAX;
        double ar = 0.0, ai = 0.0;
        if (c < n1)
            for (int gg = 0; gg < G2; ++gg) {
                ar += P[gg][r][c].re;
                ai += P[gg][r][c].im;
            }
        U[r][c] = {ar, ai};
    }
    __syncthreads();
    if (g < G1) {
#pragma unroll
        for (int r = 0; r < FDM2_RB; ++r) {
            double ar = 0.0, ai = 0.0;
#pragma unroll
            for (int q = 0; q < FDM2_CH; ++q) {
                const cx<double> u = U[r][g * FDM2_CH + q];
                ar += u.re * rv[q];
                ai += u.im * rv[q];
            }
            P[g][r][col] = {ar, ai};
        }
    }
    __syncthreads();
    for (int e = tid; e < FDM2_RB * FDM2_NMAX; e += FDM2_TB) {
        const int r = e / FDM2_NMAX, c = e % FDM2_NMAX, row = r0 + r;
        if (c < n1 && row < n2) {
            double ar = 0.0, ai = 0.0;
            for (int gg = 0; gg < G1; ++gg) {
                ar += P[gg][r][c].re;
                ai += P[gg][r][c].im;
            }
            const size_t o = (size_t)row * n1 + c;
            if (cscale) {
                const cx<double> d = cscale[o];
                Y[o] = {ar * d.re - ai * d.im, ar * d.im + ai * d.re};
            } else {
                const double d = scale ? scale[o] : 1.0;
                Y[o] = {ar * d, ai * d};
            }
        }
    }
}

void launch_fdm_solve(int n2, int n1, const double* Vx, const double* VxT, const double* Vy, const double* dinv,
                      const cx<double>* c, cx<double>* t1, cx<double>* t2, cx<double>* e, hipStream_t s,
                      const cx<double>* cdinv) {
    // c, e, 1/D (complex: twice the bytes) and both eigenvector matrices once
    meter((cdinv ? 48.0 : 40.0) * n1 * (double)n2 + 8.0 * ((double)n1 * n1 + (double)n2 * n2),
          8.0 * n1 * (double)n2 * (n1 + n2) + (cdinv ? 16.0 : 8.0) * n1 * (double)n2);
    const double* rd = cdinv ? nullptr : dinv;
    if (n1 <= FDM2_NMAX && n2 <= FDM2_NMAX) {
        const dim3 g((unsigned)((n2 + FDM2_RB - 1) / FDM2_RB)), b(FDM2_TB);
        // T2 = (Vy^T C Vx) ./ D
        hipLaunchKernelGGL(fdm_pass_kernel, g, b, 0, s, n2, n1, Vy, 1, n2, c, Vx, rd, cdinv, t2);
        // e = Vy T2 Vx^T
        hipLaunchKernelGGL(fdm_pass_kernel, g, b, 0, s, n2, n1, Vy, n2, 1, t2, VxT, nullptr, nullptr, e);
        return;
    }
    const dim3 g((unsigned)((n1 + 31) / 32), (unsigned)((n2 + 31) / 32)), b(256);
    // T1 = C Vx
    hipLaunchKernelGGL(fdm_gemm_kernel<false>, g, b, 0, s, n2, n1, n1, Vx, n1, 1, c, n1, 1, nullptr, nullptr, t1);
    // T2 = (Vy^T T1) ./ D
    hipLaunchKernelGGL(fdm_gemm_kernel<true>, g, b, 0, s, n2, n1, n2, Vy, 1, n2, t1, n1, 1, rd, cdinv, t2);
    // T1 = T2 Vx^T
    hipLaunchKernelGGL(fdm_gemm_kernel<false>, g, b, 0, s, n2, n1, n1, Vx, 1, n1, t2, n1, 1, nullptr, nullptr, t1);
    // e = Vy T1
    hipLaunchKernelGGL(fdm_gemm_kernel<true>, g, b, 0, s, n2, n1, n2, Vy, n2, 1, t1, n1, 1, nullptr, nullptr, e);
}

// --------------------------------------------------------------------------
// Coarse tail of the V-cycle in one workgroup.  On levels with a few thousand
// unknowns or fewer every kernel of the V-cycle is a handful of waves and its
// cost is launch latency.  Here one 1024-thread workgroup runs the whole
// descent (Jacobi sweeps, residual, restriction), the dense coarsest solve and
// the ascent (prolongation, Jacobi sweeps) with the right-hand side, iterate
// and spare vector of every level in LDS, and a block barrier between phases.
// The 1D bands and transfer weights of every tail level are copied into LDS
// at the start from one image prepared at setup; D^-1, the variable-k stencils
// and the coarsest inverse are read through the caches.  Each stencil sum runs over the (2px+1)(2py+1) neighbours in a fixed
// order (deterministic).
// --------------------------------------------------------------------------
constexpr int TAIL_TB = 1024;
// the tail workgroup's dynamic LDS: coefficient image, then the level vectors
// (declared here so that every helper forms LDS addresses from it directly)
extern __shared__ __align__(16) unsigned char tail_smem[];

// Stencil rows r0, r0 + rstep, ... (offsets d2 = r - P) of (K - alpha M_k) x at
// unknown (I2, I1) of a 2D tail level of degree P (x in LDS): K and M_k parts
// summed separately.  The loop over a row is unrolled; out-of-range
// neighbours read a valid entry and get a zero coefficient, so the loads of a
// row do not wait for each other.
template <class T, int P, bool SEP>
__device__ __forceinline__ void tail_rows(const TailLevel<T>& L, double k2c, const cx<T>* x, int I2, int I1, int r0,
                                          int rstep, T& kr, T& ki, T& mr, T& mi) {
    constexpr int B = 2 * P + 1;
    const int n1 = L.n1, N = L.n1 * L.n2, I = I2 * n1 + I1;
    T kx[B], mx[B];   // this column's x bands, the same for every stencil row
#pragma unroll
    for (int d = 0; d < B; ++d) {
        kx[d] = (T)L.Kx[I1 * B + d];
        mx[d] = (T)L.Mx[I1 * B + d];
    }
    for (int r = r0; r < B; r += rstep) {
        const int d2 = r - P;
        const bool ok2 = (unsigned)(I2 + d2) < (unsigned)L.n2;
        const T myv = (T)L.My[I2 * B + r], kyv = (T)L.Ky[I2 * B + r];
        const cx<T>* row = x + (ok2 ? I2 + d2 : I2) * n1;
        if constexpr (SEP) {
            // separable row: u1 = Kx-band sum, u2 = Mx-band sum of the row's values;
            // K part my u1 + ky u2, mass part k^2 my u2.  The 1D bands are zero
            // at neighbours outside the level, so an out-of-range neighbour (read
            // at a clamped, valid address: a finite value) adds zero unmasked.
            T u1r = 0, u1i = 0, u2r = 0, u2i = 0;
#pragma unroll
            for (int d1 = -P; d1 <= P; ++d1) {
                const bool ok = (unsigned)(I1 + d1) < (unsigned)n1;
                const cx<T> v = row[ok ? I1 + d1 : I1];
                u1r += kx[d1 + P] * v.re;
                u1i += kx[d1 + P] * v.im;
                u2r += mx[d1 + P] * v.re;
                u2i += mx[d1 + P] * v.im;
            }
            const T km = (T)k2c * myv;
            kr += myv * u1r + kyv * u2r;
            ki += myv * u1i + kyv * u2i;
            mr += km * u2r;
            mi += km * u2i;
        } else {
#pragma unroll
            for (int d1 = -P; d1 <= P; ++d1) {
                const bool ok = ok2 && (unsigned)(I1 + d1) < (unsigned)n1;
                const cx<T> v = row[ok ? I1 + d1 : I1];
                T kc = myv * kx[d1 + P] + kyv * mx[d1 + P];
                T mc = L.S[(size_t)(r * B + d1 + P) * N + I];
                kc = ok ? kc : T(0);
                mc = ok ? mc : T(0);
                kr += kc * v.re;
                ki += kc * v.im;
                mr += mc * v.re;
                mi += mc * v.im;
            }
        }
    }
}

// (K - alpha M_k) x at unknown (I2, I1) of one level (x in LDS), any shape:
// the loops run over the in-range neighbours only.
template <class T>
__device__ __forceinline__ cx<T> tail_apply(const TailLevel<T>& L, double k2c, T are, T aim, const cx<T>* x, int I2,
                                            int I1, long long N) {
    const int bx = 2 * L.px + 1, by = 2 * L.py + 1;
    T kr = 0, ki = 0, mr = 0, mi = 0;
    const int d2a = max(-L.py, -I2), d2b = min(L.py, L.n2 - 1 - I2);
    const int d1a = max(-L.px, -I1), d1b = min(L.px, L.n1 - 1 - I1);
    const double* kxr = L.Kx + (size_t)I1 * bx + L.px;
    const double* mxr = L.Mx + (size_t)I1 * bx + L.px;
    for (int d2 = d2a; d2 <= d2b; ++d2) {
        const T myv = (T)L.My[(size_t)I2 * by + d2 + L.py], kyv = (T)L.Ky[(size_t)I2 * by + d2 + L.py];
        const cx<T>* row = x + (size_t)(I2 + d2) * L.n1 + I1;
        for (int d1 = d1a; d1 <= d1b; ++d1) {
            const T kxv = (T)kxr[d1], mxv = (T)mxr[d1];
            const cx<T> v = row[d1];
            const T kc = myv * kxv + kyv * mxv;
            const T mc = (L.kind == KIND_SEP) ? (T)k2c * myv * mxv
                                              : L.S[(size_t)((d2 + L.py) * bx + d1 + L.px) * N + (size_t)I2 * L.n1 + I1];
            kr += kc * v.re;
            ki += kc * v.im;
            mr += mc * v.re;
            mi += mc * v.im;
        }
    }
    return {kr - (are * mr - aim * mi), ki - (are * mi + aim * mr)};
}

// y = b - M_beta x (RESID) or y = x + omega D^-1 (b - M_beta x) (SMOOTH), then a
// block barrier.  P > 0: G = 1, 2, 4 or 8 adjacent lanes share an unknown (the
// most that the level's size allows in one pass of the workgroup), each takes
// every G-th stencil row, and the partial sums meet in a butterfly over the G
// lanes (a fixed order, so the result is reproducible).
template <class T, int P>
__device__ __forceinline__ void tail_op(const TailLevel<T>& L, const TailDesc<T>& D, int mode, const cx<T>* x,
                                        const cx<T>* b, cx<T>* y) {
    const int n1 = L.n1, N = L.n1 * L.n2;
    if constexpr (P > 0) {
        const int G = N <= TAIL_TB / 8 ? 8 : N <= TAIL_TB / 4 ? 4 : N <= TAIL_TB / 2 ? 2 : 1;
        const int sub = threadIdx.x & (G - 1);
        for (int I = threadIdx.x / G; I < N; I += TAIL_TB / G) {
            const int I1 = I % n1, I2 = I / n1;
            T kr = 0, ki = 0, mr = 0, mi = 0;
            if (L.kind == KIND_SEP)
                tail_rows<T, P, true>(L, D.k2c, x, I2, I1, sub, G, kr, ki, mr, mi);
            else
                tail_rows<T, P, false>(L, D.k2c, x, I2, I1, sub, G, kr, ki, mr, mi);
            for (int o = G >> 1; o > 0; o >>= 1) {
                kr += __shfl_xor(kr, o, 64);
                ki += __shfl_xor(ki, o, 64);
                mr += __shfl_xor(mr, o, 64);
                mi += __shfl_xor(mi, o, 64);
            }
            if (sub == 0) {
                const cx<T> bv = b[I];
                const T rr = bv.re - (kr - (D.are * mr - D.aim * mi)), ri = bv.im - (ki - (D.are * mi + D.aim * mr));
                if (mode == MODE_RESID) {
                    y[I] = {rr, ri};
                } else {
                    const cx<T> dv = L.dinv[I], xv = x[I];
                    y[I] = {xv.re + L.omega * (dv.re * rr - dv.im * ri), xv.im + L.omega * (dv.re * ri + dv.im * rr)};
                }
            }
        }
    } else {
        for (int I = threadIdx.x; I < N; I += TAIL_TB) {
            const int I1 = I % n1, I2 = I / n1;
            const cx<T> a = tail_apply<T>(L, D.k2c, D.are, D.aim, x, I2, I1, N);
            const cx<T> bv = b[I];
            const T rr = bv.re - a.re, ri = bv.im - a.im;
            if (mode == MODE_RESID) {
                y[I] = {rr, ri};
            } else {
                const cx<T> dv = L.dinv[I], xv = x[I];
                y[I] = {xv.re + L.omega * (dv.re * rr - dv.im * ri), xv.im + L.omega * (dv.re * ri + dv.im * rr)};
            }
        }
    }
    __syncthreads();
}

// A level's descriptor (a level above the coarsest) with its bands and
// transfer tables redirected to the LDS copies.  Every redirected pointer is
// formed from tail_smem, so the compiler addresses them as LDS.
template <class T>
__device__ __forceinline__ TailLevel<T> tail_level(const TailDesc<T>& D, int l) {
    TailLevel<T> v = D.lv[l];
    v.Kx = (const double*)(tail_smem + v.o_kx);
    v.Mx = (const double*)(tail_smem + v.o_mx);
    v.Ky = (const double*)(tail_smem + v.o_ky);
    v.My = (const double*)(tail_smem + v.o_my);
    v.tr.prow0x = (const int*)(tail_smem + v.o_prow0x);
    v.tr.prowx = (const double*)(tail_smem + v.o_prowx);
    v.tr.prow0y = (const int*)(tail_smem + v.o_prow0y);
    v.tr.prowy = (const double*)(tail_smem + v.o_prowy);
    v.tr.pcol0x = (const int*)(tail_smem + v.o_pcol0x);
    v.tr.pcolx = (const double*)(tail_smem + v.o_pcolx);
    v.tr.pcol0y = (const int*)(tail_smem + v.o_pcol0y);
    v.tr.pcoly = (const double*)(tail_smem + v.o_pcoly);
    return v;
}

// P = 0: any level shapes; P > 0: 2D levels of degree P (unrolled stencils and
// transfers; restriction runs <= P + 2, prolongation runs <= P + 1)
template <class T, int P>
__global__ __launch_bounds__(TAIL_TB) void vcycle_tail_kernel(const TailDesc<T>* __restrict__ Dp, int l0,
                                                              const uint4* __restrict__ img, int n16,
                                                              const cx<T>* __restrict__ minv,
                                                              const cx<T>* __restrict__ b0, cx<T>* __restrict__ x0) {
    constexpr int WR = P > 0 ? P + 2 : 0, WP = P > 0 ? P + 1 : 0;
    const TailDesc<T>& D = *Dp;
    const int L = D.L;
    auto vb = [&](int l) { return (cx<T>*)(tail_smem + D.offb[l]); };
    auto vx = [&](int l) { return (cx<T>*)(tail_smem + D.offx[l]); };
    auto vt = [&](int l) { return (cx<T>*)(tail_smem + D.offt[l]); };
    {
        // the coefficient image (the tables of every tail level, prepared at
        // setup in their LDS layout) and the level-l0 right-hand side
        const int N0 = D.lv[l0].n1 * D.lv[l0].n2;
        cx<T>* b = vb(l0);
        uint4* dst = (uint4*)tail_smem;
#pragma unroll 4
        for (int I = threadIdx.x; I < n16; I += TAIL_TB) dst[I] = img[I];
        for (int I = threadIdx.x; I < N0; I += TAIL_TB) b[I] = b0[I];
        if (D.o_minv >= 0) {   // the coarsest inverse, transposed (MT[c][r] = Minv[r][c])
            cx<T>* MT = (cx<T>*)(tail_smem + D.o_minv);
            const int nL = D.nL;
            for (int i = threadIdx.x; i < nL * nL; i += TAIL_TB) MT[(i % nL) * nL + i / nL] = minv[i];
        }
        __syncthreads();
    }
    // descent
    for (int l = l0; l < L; ++l) {
        const TailLevel<T> lv = tail_level<T>(D, l);
        const int N = lv.n1 * lv.n2;
        const cx<T>* b = vb(l);
        cx<T>* x = vx(l);
        cx<T>* t = vt(l);
        cx<T>* cur = ((D.nu_pre - 1) & 1) ? t : x;
        cx<T>* oth = ((D.nu_pre - 1) & 1) ? x : t;
        for (int I = threadIdx.x; I < N; I += TAIL_TB) {
            const cx<T> dv = lv.dinv[I], bv = b[I];
            cur[I] = {lv.omega * (dv.re * bv.re - dv.im * bv.im), lv.omega * (dv.re * bv.im + dv.im * bv.re)};
        }
        __syncthreads();
        for (int i = 1; i < D.nu_pre; ++i) {
            tail_op<T, P>(lv, D, MODE_SMOOTH, cur, b, oth);
            cx<T>* tmp = cur;
            cur = oth;
            oth = tmp;
        }
        tail_op<T, P>(lv, D, MODE_RESID, x, b, t);   // the spare vector holds the residual
        const int Nc = lv.tr.nc1 * lv.tr.nc2;
        cx<T>* bc = vb(l + 1);
        for (int I = threadIdx.x; I < Nc; I += TAIL_TB) bc[I] = restrict_one<T, WR, false>(lv.tr, t, I);
        __syncthreads();
    }
    // coarsest level: x = M_beta^-1 b, one wave per row (lane-strided sums, butterfly)
    {
        const cx<T>* b = vb(L);
        cx<T>* x = vx(L);
        const int nL = D.nL;
        if (D.o_minv >= 0) {
            // transposed copy in LDS: one thread per row, j in increasing order
            const cx<T>* MT = (const cx<T>*)(tail_smem + D.o_minv);
            for (int r = threadIdx.x; r < nL; r += TAIL_TB) {
                T sr = 0, si = 0;
                for (int j = 0; j < nL; ++j) {
                    const cx<T> av = MT[j * nL + r], xv = b[j];
                    sr += av.re * xv.re - av.im * xv.im;
                    si += av.re * xv.im + av.im * xv.re;
                }
                x[r] = {sr, si};
            }
        } else {
            // one wave per row (lane-strided sums, butterfly)
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            for (int row = wave; row < nL; row += TAIL_TB / 64) {
                T sr = 0, si = 0;
                const cx<T>* a = minv + (size_t)row * nL;
                for (int j = lane; j < nL; j += 64) {
                    const cx<T> av = a[j], xv = b[j];
                    sr += av.re * xv.re - av.im * xv.im;
                    si += av.re * xv.im + av.im * xv.re;
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    sr += __shfl_xor(sr, o, 64);
                    si += __shfl_xor(si, o, 64);
                }
                if (lane == 0) x[row] = {sr, si};
            }
        }
        __syncthreads();
    }
    // ascent
    for (int l = L - 1; l >= l0; --l) {
        const TailLevel<T> lv = tail_level<T>(D, l);
        const int N = lv.n1 * lv.n2;
        const cx<T>* b = vb(l);
        cx<T>* x = vx(l);
        cx<T>* t = vt(l);
        const cx<T>* xc = vx(l + 1);
        cx<T>* cur = (D.nu_post & 1) ? t : x;
        cx<T>* oth = (D.nu_post & 1) ? x : t;
        for (int I = threadIdx.x; I < N; I += TAIL_TB) {
            const cx<T> v = prolong_one<T, WP, false>(lv.tr, xc, I), o = x[I];
            cur[I] = {o.re + v.re, o.im + v.im};
        }
        __syncthreads();
        for (int i = 0; i < D.nu_post; ++i) {
            tail_op<T, P>(lv, D, MODE_SMOOTH, cur, b, oth);
            cx<T>* tmp = cur;
            cur = oth;
            oth = tmp;
        }
    }
    {
        const int N0 = D.lv[l0].n1 * D.lv[l0].n2;
        const cx<T>* x = vx(l0);
        for (int I = threadIdx.x; I < N0; I += TAIL_TB) x0[I] = x[I];
    }
}

template <class T>
static const void* tail_fn(int P) {
    switch (P) {
        case 1: return (const void*)vcycle_tail_kernel<T, 1>;
        case 2: return (const void*)vcycle_tail_kernel<T, 2>;
        case 3: return (const void*)vcycle_tail_kernel<T, 3>;
        case 4: return (const void*)vcycle_tail_kernel<T, 4>;
        case 5: return (const void*)vcycle_tail_kernel<T, 5>;
    }
    return (const void*)vcycle_tail_kernel<T, 0>;
}

template <class T>
void tail_prepare(int lds_bytes) {
    for (int P = 0; P <= 5; ++P)
        HH_HIP(hipFuncSetAttribute(tail_fn<T>(P), hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes));
}
template void tail_prepare<double>(int);
template void tail_prepare<float>(int);

template <class T>
void launch_vcycle_tail(const TailDesc<T>* desc, const void* img, int img16, const cx<T>* minv, int P, int l0,
                        int lds_bytes, const cx<T>* b, cx<T>* x, hipStream_t s) {
    void* args[] = {(void*)&desc, (void*)&l0, (void*)&img, (void*)&img16, (void*)&minv, (void*)&b, (void*)&x};
    HH_HIP(hipLaunchKernel(tail_fn<T>(P), dim3(1), dim3(TAIL_TB), args, (size_t)lds_bytes, s));
}
template void launch_vcycle_tail<double>(const TailDesc<double>*, const void*, int, const cx<double>*, int, int, int,
                                         const cx<double>*, cx<double>*, hipStream_t);
template void launch_vcycle_tail<float>(const TailDesc<float>*, const void*, int, const cx<float>*, int, int, int,
                                        const cx<float>*, cx<float>*, hipStream_t);

// --------------------------------------------------------------------------
// Symmetric dense E^-1 (variable-k deflation level): only the upper triangle
// is stored, as 128 x 128 tiles (I <= J) packed in row order of the tile grid,
// each tile row-major and zero-padded past n.  A product reads every stored
// entry once and uses it twice (row sums of tile (I, J) go to block I, column
// sums to block J), halving the bytes of a full-matrix product.  Tile partial
// sums go to per-tile slots and are added per block in a fixed order, so the
// result is deterministic.
// --------------------------------------------------------------------------
constexpr int SYT = 128;
constexpr long long SYM_STRIDE = (long long)SYT * SYT;   // tile stride (doubles)
__device__ __host__ inline long long sym_tile_index(long long I, long long J, long long nt) {
    return I * nt - I * (I - 1) / 2 + (J - I);
}
long long sym_tiles(int n) {
    const long long nt = (n + SYT - 1) / SYT;
    return nt * (nt + 1) / 2;
}
long long sym_packed_doubles(int n) { return sym_tiles(n) * SYM_STRIDE; }

__global__ __launch_bounds__(256) void sym_pack_kernel(int n, long long ld, const double* __restrict__ D,
                                                       double* __restrict__ P) {
    const int I = blockIdx.y, J = blockIdx.x;
    if (J < I) return;
    const long long nt = (n + SYT - 1) / SYT;
    double* T = P + sym_tile_index(I, J, nt) * SYM_STRIDE;
    for (int e = threadIdx.x; e < SYT * SYT; e += 256) {
        const int rr = e / SYT, cc = e % SYT;
        const long long r = (long long)I * SYT + rr, c = (long long)J * SYT + cc;
        T[e] = (r < n && c < n) ? D[r * ld + c] : 0.0;
    }
}
void launch_sym_pack(int n, long long ld, const double* D, double* P, hipStream_t s) {
    const unsigned nt = (unsigned)((n + SYT - 1) / SYT);
    hipLaunchKernelGGL(sym_pack_kernel, dim3(nt, nt), dim3(256), 0, s, n, ld, D, P);
}

// One workgroup per stored tile (I, J): wave w takes rows 32w .. 32w+31 of
// the tile, lane l columns 2l, 2l+1 (16-byte loads).  Row sums: every lane
// keeps its partial for each of the 32 rows, then one reduce-scatter over the
// wave (five halving exchanges, lane l ends with row l/2, a last exchange adds
// the lane pair) -- 32 shuffles per lane instead of a butterfly per row.
// Column sums (off-diagonal tiles): per lane over its rows, then the four
// waves in order.
typedef double dbl2v __attribute__((ext_vector_type(2)));

// One workgroup per stored tile, in storage order (a 1D grid over the
// triangle: no idle workgroups), the tile streamed with nontemporal loads.
__global__ __launch_bounds__(256) void symv_tiles_kernel(int n, const double* __restrict__ P,
                                                         const cx<double>* __restrict__ x,
                                                         cx<double>* __restrict__ rowpart,
                                                         cx<double>* __restrict__ colpart) {
    __shared__ cx<double> xs[SYT];
    __shared__ cx<double> us[SYT];
    __shared__ double vs[4][SYT][2];
    const long long nt = (n + SYT - 1) / SYT;
    const long long tidx = blockIdx.x;
    // tile row I: the last row whose first tile index I nt - I (I - 1) / 2 is <= tidx
    long long I = (long long)((2.0 * nt + 1.0 - sqrt((2.0 * nt + 1.0) * (2.0 * nt + 1.0) - 8.0 * (double)tidx)) / 2.0);
    I = I < 0 ? 0 : (I >= nt ? nt - 1 : I);
    while (I > 0 && sym_tile_index(I, I, nt) > tidx) --I;
    while (I + 1 < nt && sym_tile_index(I + 1, I + 1, nt) <= tidx) ++I;
    const long long J = I + (tidx - sym_tile_index(I, I, nt));
    const double* T = P + tidx * SYM_STRIDE;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x < SYT) {
        const long long r = (long long)I * SYT + threadIdx.x;
        xs[threadIdx.x] = r < n ? x[r] : cx<double>{0.0, 0.0};
    }
    const long long c0 = (long long)J * SYT + 2 * lane;
    const cx<double> xj0 = c0 < n ? x[c0] : cx<double>{0.0, 0.0};
    const cx<double> xj1 = c0 + 1 < n ? x[c0 + 1] : cx<double>{0.0, 0.0};
    __syncthreads();
    double vr0 = 0.0, vi0 = 0.0, vr1 = 0.0, vi1 = 0.0;
    const bool off = (I != J);
    double ur[32], ui[32];
    const double* Tw = T + (size_t)(32 * w) * SYT + 2 * lane;
    // all 32 row loads of the wave are issued before any is used (the empty
    // asm with a memory clobber keeps the compiler from interleaving them with
    // the arithmetic, which left one or two loads in flight)
    dbl2v av[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) av[q] = __builtin_nontemporal_load((const dbl2v*)(Tw + (size_t)q * SYT));
    asm volatile("" ::: "memory");
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const dbl2v a = av[q];
        ur[q] = a.x * xj0.re + a.y * xj1.re;
        ui[q] = a.x * xj0.im + a.y * xj1.im;
        if (off) {
            const cx<double> xi = xs[32 * w + q];
            vr0 += a.x * xi.re;
            vi0 += a.x * xi.im;
            vr1 += a.y * xi.re;
            vi1 += a.y * xi.im;
        }
    }
#pragma unroll
    for (int lvl = 0; lvl < 5; ++lvl) {
        const int o = 32 >> lvl, cnt = 16 >> lvl;
        const bool hi = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < cnt; ++i) {
            const double sr = hi ? ur[i] : ur[i + cnt], si = hi ? ui[i] : ui[i + cnt];
            const double kr = hi ? ur[i + cnt] : ur[i], ki = hi ? ui[i + cnt] : ui[i];
            ur[i] = kr + __shfl_xor(sr, o, 64);
            ui[i] = ki + __shfl_xor(si, o, 64);
        }
    }
    ur[0] += __shfl_xor(ur[0], 1, 64);
    ui[0] += __shfl_xor(ui[0], 1, 64);
    if ((lane & 1) == 0) us[32 * w + (lane >> 1)] = {ur[0], ui[0]};
    if (off) {
        vs[w][2 * lane][0] = vr0;
        vs[w][2 * lane][1] = vi0;
        vs[w][2 * lane + 1][0] = vr1;
        vs[w][2 * lane + 1][1] = vi1;
    }
    __syncthreads();
    if (threadIdx.x < SYT) {
        const int c = threadIdx.x;
        rowpart[tidx * SYT + c] = us[c];
        if (off)
            colpart[tidx * SYT + c] = {vs[0][c][0] + vs[1][c][0] + vs[2][c][0] + vs[3][c][0],
                                       vs[0][c][1] + vs[1][c][1] + vs[2][c][1] + vs[3][c][1]};
    }
}

// y for block I: sum over J = 0 .. nt-1 of (J < I: column sums of tile (J, I),
// J >= I: row sums of tile (I, J)).  SYR_G lane groups of SYT threads take
// J = g, g + SYR_G, ... in increasing order (four partials loaded at a time),
// and the group sums are added in group order: a fixed order, deterministic.
constexpr int SYR_G = 8;
__global__ __launch_bounds__(SYT * SYR_G) void symv_reduce_kernel(int n, const cx<double>* __restrict__ rowpart,
                                                                   const cx<double>* __restrict__ colpart,
                                                                   cx<double>* __restrict__ y) {
    __shared__ double sr_s[SYR_G][SYT], si_s[SYR_G][SYT];
    const int I = blockIdx.x, r = threadIdx.x % SYT, grp = threadIdx.x / SYT;
    const long long nt = (n + SYT - 1) / SYT;
    auto part = [&](long long J) -> cx<double> {
        return (J < I) ? colpart[sym_tile_index(J, I, nt) * SYT + r] : rowpart[sym_tile_index(I, J, nt) * SYT + r];
    };
    double sr = 0.0, si = 0.0;
    long long J = grp;
    for (; J + 3 * SYR_G < nt; J += 4 * SYR_G) {
        const cx<double> v0 = part(J), v1 = part(J + SYR_G), v2 = part(J + 2 * SYR_G), v3 = part(J + 3 * SYR_G);
        sr += v0.re;
        si += v0.im;
        sr += v1.re;
        si += v1.im;
        sr += v2.re;
        si += v2.im;
        sr += v3.re;
        si += v3.im;
    }
    for (; J < nt; J += SYR_G) {
        const cx<double> v = part(J);
        sr += v.re;
        si += v.im;
    }
    sr_s[grp][r] = sr;
    si_s[grp][r] = si;
    __syncthreads();
    const long long gr = (long long)I * SYT + threadIdx.x;
    if (threadIdx.x < SYT && gr < n) {
        double tr = 0.0, ti = 0.0;
#pragma unroll
        for (int g = 0; g < SYR_G; ++g) {
            tr += sr_s[g][threadIdx.x];
            ti += si_s[g][threadIdx.x];
        }
        y[gr] = {tr, ti};
    }
}

void launch_symv(int n, const double* P, const cx<double>* x, cx<double>* rowpart, cx<double>* colpart,
                 cx<double>* y, hipStream_t s) {
    const unsigned nt = (unsigned)((n + SYT - 1) / SYT);
    meter(8.0 * SYM_STRIDE * (double)sym_tiles(n) + 32.0 * n, 4.0 * n * (double)n);
    hipLaunchKernelGGL(symv_tiles_kernel, dim3((unsigned)sym_tiles(n)), dim3(256), 0, s, n, P, x, rowpart, colpart);
    hipLaunchKernelGGL(symv_reduce_kernel, dim3(nt), dim3(SYT * SYR_G), 0, s, n, rowpart, colpart, y);
}

// Dense-matrix set-up helpers: y[idx[i]] = val[i] (distinct indices), and
// the diagonal of an n x n zero matrix set to one.
__global__ void scatter_kernel(long long n, const long long* __restrict__ idx, const double* __restrict__ val,
                               double* __restrict__ y) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[idx[i]] = val[i];
}
void launch_scatter(long long n, const long long* idx, const double* val, double* y, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(scatter_kernel, dim3(grid1d(n, 256)), dim3(256), 0, s, n, idx, val, y);
}
__global__ void set_identity_kernel(long long n, long long ld, double* __restrict__ a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i * ld + i] = 1.0;
}
void launch_set_identity(int n, long long ld, double* a, hipStream_t s) {
    hipLaunchKernelGGL(set_identity_kernel, dim3(grid1d(n, 256)), dim3(256), 0, s, (long long)n, ld, a);
}

// --------------------------------------------------------------------------
// Krylov: deterministic two-stage reductions.  Every block writes its partial
// sum; the last block to finish (device-scope atomic ticket) sums the partials
// in index order, so results do not depend on block scheduling.
// --------------------------------------------------------------------------
constexpr int RB = 256;  // threads per reduction block

int reduction_blocks(long long N) {
    long long b = (N + 4 * RB - 1) / (4 * RB);
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
    const int t = threadIdx.x;
    sh[t] = a;
    sh[RB + t] = b;
    __syncthreads();
#pragma unroll
    for (int o = RB / 2; o > 0; o >>= 1) {
        if (t < o) {
            sh[t] += sh[t + o];
            sh[RB + t] += sh[RB + t + o];
        }
        __syncthreads();
    }
    a = sh[0];
    b = sh[RB];
}

// Returns true in the one block that sees all partials (after its block_sum2).
// Memory model: the partial is released with an agent-scope fence before the
// ticket, and the last block acquires with another fence before it reads the
// partials (the L2 caches of the XCDs are not coherent with each other
// otherwise).
__device__ __forceinline__ bool last_block(int* counter, bool* flag) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ticket = atomicAdd(counter, 1);
        *flag = (ticket == (int)gridDim.x - 1);
    }
    __syncthreads();
    if (*flag) __threadfence();
    return *flag;
}

__device__ __forceinline__ void sum_partials(const cx<double>* partials, int nb, double& re, double& im,
                                             double* sh) {
    re = 0.0;
    im = 0.0;
    for (int i = threadIdx.x; i < nb; i += RB) {
        const cx<double> v = partials[i];
        re += v.re;
        im += v.im;
    }
    block_sum2(re, im, sh);
}

__device__ __forceinline__ cx<double> hload(const cx<double>* p) {
    // device-scope coherent read of a value written by another block of an
    // earlier kernel (plain load; kernels on one stream are ordered)
    return *p;
}

// w -= h_{i-1} V[i-1] (i > 0), then H[i, j] = V[i]^H w.
__global__ __launch_bounds__(RB) void mgs_kernel(long long N, int i, int j, cx<double>* __restrict__ w,
                                                 const cx<double>* __restrict__ V, long long ldv, KrylovDev k) {
    __shared__ double sh[2 * RB];
    __shared__ bool flag;
    const int ldh = k.m + 1;
    cx<double> h = {0.0, 0.0};
    if (i > 0) h = hload(&k.H[(size_t)j * ldh + (i - 1)]);
    const cx<double>* vp = V + (size_t)(i > 0 ? i - 1 : 0) * ldv;
    const cx<double>* vc = V + (size_t)i * ldv;
    double sr = 0.0, si = 0.0;
    const long long stride = (long long)gridDim.x * RB;
    for (long long t = (long long)blockIdx.x * RB + threadIdx.x; t < N; t += stride) {
        cx<double> wv = w[t];
        if (i > 0) {
            const cx<double> pv = vp[t];
            wv.re -= h.re * pv.re - h.im * pv.im;
            wv.im -= h.re * pv.im + h.im * pv.re;
            w[t] = wv;
        }
        const cx<double> cv = vc[t];
        sr += cv.re * wv.re + cv.im * wv.im;   // conj(v) w
        si += cv.re * wv.im - cv.im * wv.re;
    }
    block_sum2(sr, si, sh);
    if (threadIdx.x == 0) k.partials[blockIdx.x] = {sr, si};
    if (!last_block(&k.ints[2], &flag)) return;
    double tr, ti;
    sum_partials(k.partials, gridDim.x, tr, ti, sh);
    if (threadIdx.x == 0) {
        k.H[(size_t)j * ldh + i] = {tr, ti};
        k.ints[2] = 0;
    }
}

void launch_mgs(long long N, int i, int j, cx<double>* w, const cx<double>* V, long long ldv, KrylovDev& k,
                hipStream_t s) {
    hipLaunchKernelGGL(mgs_kernel, dim3(reduction_blocks(N)), dim3(RB), 0, s, N, i, j, w, V, ldv, k);
}

__device__ void givens_rot(cx<double> a, cx<double> b, double& c, cx<double>& s) {
    const double ab = hypot(a.re, a.im), bb = hypot(b.re, b.im);
    if (bb == 0.0) {
        c = 1.0;
        s = {0.0, 0.0};
    } else if (ab == 0.0) {
        c = 0.0;
        s = {b.re / bb, -b.im / bb};
    } else {
        const double t = sqrt(ab * ab + bb * bb);
        c = ab / t;
        const cx<double> u = {a.re / ab, a.im / ab};
        const cx<double> cb = {b.re / t, -b.im / t};
        s = cmul(u, cb);
    }
}

// Givens update of a Hessenberg column Hc[0..j+1] with H[j+1, j] = hn: the
// previous rotations (cs, sn) in order, then the new one annihilating
// H[j+1, j], returned in c, s.  Single thread; the same operations wherever
// the column and the rotations are held (device memory or LDS).
__device__ __forceinline__ void givens_rotate(cx<double>* Hc, const double* cs, const cx<double>* sn, int j,
                                              double hn, double& c, cx<double>& s) {
    // rotation ii acts on entries ii and ii + 1; the rotated entry ii + 1 is
    // carried to the next rotation in a register
    cx<double> a = Hc[0];
    for (int ii = 0; ii < j; ++ii) {
        const double ci = cs[ii];
        const cx<double> si = sn[ii];
        const cx<double> b = Hc[ii + 1];
        const cx<double> sb = cmul(si, b);
        const cx<double> t = {ci * a.re + sb.re, ci * a.im + sb.im};
        const cx<double> cs_ = {si.re, -si.im};
        const cx<double> ca = cmul(cs_, a);
        Hc[ii] = t;
        a = {-ca.re + ci * b.re, -ca.im + ci * b.im};
    }
    const cx<double> b = {hn, 0.0};
    givens_rot(a, b, c, s);
    const cx<double> sb = cmul(s, b);
    Hc[j] = {c * a.re + sb.re, c * a.im + sb.im};
    Hc[j + 1] = {0.0, 0.0};
}

// The rest of step j's update: rotation j stored, g rotated, |g_{j+1}|, the
// step count and the breakdown flag (gj = g[j], broke = the flag on entry).
__device__ __forceinline__ double givens_finish(KrylovDev& k, int j, double hn, double c, cx<double> s,
                                                cx<double> gj, int broke) {
    k.scal[1] = hn;
    k.cs[j] = c;
    k.sn[j] = s;
    const cx<double> cs_ = {s.re, -s.im};
    const cx<double> ng = cmul(cs_, gj);
    const cx<double> g1 = {-ng.re, -ng.im};
    k.g[j + 1] = g1;
    k.g[j] = {c * gj.re, c * gj.im};
    const double gabs = hypot(g1.re, g1.im);
    k.scal[2] = gabs;
    if (!broke) k.ints[0] = j + 1;
    if (hn == 0.0) k.ints[1] = 1;
    return gabs;
}

// What the host reads after step j, stored by the thread that finished the
// step straight into the pinned slot j & 1 (when the Krylov state has one):
// |g_{j+1}| at double 2, the breakdown flag at int 1 and the grid-exchange
// timeout flag (tmo, read before the Givens update) at int 5 of the slot's
// integers, which start at byte 64.
__device__ __forceinline__ void publish_step(KrylovDev& k, int j, double gabs, int breakdown, int tmo) {
    unsigned char* slot = k.hstep + 128 * (j & 1);
    ((double*)slot)[2] = gabs;
    ((int*)(slot + 64))[1] = breakdown;
    ((int*)(slot + 64))[5] = tmo;
}

// Givens update of Hessenberg column j and of the residual vector g, all in
// device memory; single thread.
__device__ void givens_column(KrylovDev& k, int j, double hn) {
    double c;
    cx<double> s;
    givens_rotate(k.H + (size_t)j * (k.m + 1), k.cs, k.sn, j, hn, c, s);
    givens_finish(k, j, hn, c, s, k.g[j], k.ints[1]);
}

// w -= H[j,j] V[j]; hn = ||w||; H[j+1,j] = hn; Givens update of column j and g.
__global__ __launch_bounds__(RB) void norm_givens_kernel(long long N, int j, cx<double>* __restrict__ w,
                                                         const cx<double>* __restrict__ V, long long ldv,
                                                         KrylovDev k) {
    __shared__ double sh[2 * RB];
    __shared__ bool flag;
    const int ldh = k.m + 1;
    const cx<double> h = hload(&k.H[(size_t)j * ldh + j]);
    const cx<double>* vp = V + (size_t)j * ldv;
    double sr = 0.0, dummy = 0.0;
    const long long stride = (long long)gridDim.x * RB;
    for (long long t = (long long)blockIdx.x * RB + threadIdx.x; t < N; t += stride) {
        cx<double> wv = w[t];
        const cx<double> pv = vp[t];
        wv.re -= h.re * pv.re - h.im * pv.im;
        wv.im -= h.re * pv.im + h.im * pv.re;
        w[t] = wv;
        sr += wv.re * wv.re + wv.im * wv.im;
    }
    block_sum2(sr, dummy, sh);
    if (threadIdx.x == 0) k.partials[blockIdx.x] = {sr, 0.0};
    if (!last_block(&k.ints[2], &flag)) return;
    double tr, ti;
    sum_partials(k.partials, gridDim.x, tr, ti, sh);
    if (threadIdx.x != 0) return;
    k.ints[2] = 0;
    givens_column(k, j, sqrt(tr));
}

void launch_norm_givens(long long N, int j, cx<double>* w, const cx<double>* V, long long ldv, KrylovDev& k,
                        hipStream_t s) {
    hipLaunchKernelGGL(norm_givens_kernel, dim3(reduction_blocks(N)), dim3(RB), 0, s, N, j, w, V, ldv, k);
}

// One whole Arnoldi step on a short vector in a single workgroup: modified
// Gram-Schmidt of w against V[0..j] (h_ij = V_i^H w, w -= h_ij V_i, in order),
// hn = ||w||, the Givens update, and w /= hn.  Each thread owns a fixed strided
// subset of the entries, so only the reductions need barriers.
constexpr int SB = 1024;
__global__ __launch_bounds__(SB) void arnoldi_small_kernel(long long N, int j, cx<double>* __restrict__ w,
                                                           const cx<double>* __restrict__ V, long long ldv,
                                                           KrylovDev k) {
    __shared__ double sh[2 * SB];
    const int tid = threadIdx.x;
    const int ldh = k.m + 1;
    for (int i = 0; i <= j; ++i) {
        const cx<double>* vi = V + (size_t)i * ldv;
        double sr = 0.0, si = 0.0;
        for (long long t = tid; t < N; t += SB) {
            const cx<double> cv = vi[t], wv = w[t];
            sr += cv.re * wv.re + cv.im * wv.im;
            si += cv.re * wv.im - cv.im * wv.re;
        }
        sh[tid] = sr;
        sh[SB + tid] = si;
        __syncthreads();
        for (int o = SB / 2; o > 0; o >>= 1) {
            if (tid < o) {
                sh[tid] += sh[tid + o];
                sh[SB + tid] += sh[SB + tid + o];
            }
            __syncthreads();
        }
        const cx<double> h = {sh[0], sh[SB]};
        __syncthreads();
        if (tid == 0) k.H[(size_t)j * ldh + i] = h;
        for (long long t = tid; t < N; t += SB) {
            const cx<double> cv = vi[t];
            cx<double> wv = w[t];
            wv.re -= h.re * cv.re - h.im * cv.im;
            wv.im -= h.re * cv.im + h.im * cv.re;
            w[t] = wv;
        }
    }
    double nr = 0.0;
    for (long long t = tid; t < N; t += SB) {
        const cx<double> wv = w[t];
        nr += wv.re * wv.re + wv.im * wv.im;
    }
    sh[tid] = nr;
    __syncthreads();
    for (int o = SB / 2; o > 0; o >>= 1) {
        if (tid < o) sh[tid] += sh[tid + o];
        __syncthreads();
    }
    const double hn = sqrt(sh[0]);
    if (tid == 0) {
        givens_column(k, j, hn);
        if (k.hstep) {
            const int tmo = __hip_atomic_load(&k.ints[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            publish_step(k, j, k.scal[2], k.ints[1], tmo);
        }
    }
    for (long long t = tid; t < N; t += SB) {
        const cx<double> wv = w[t];
        w[t] = hn == 0.0 ? cx<double>{0.0, 0.0} : cx<double>{wv.re / hn, wv.im / hn};
    }
}

void launch_arnoldi_small(long long N, int j, cx<double>* w, const cx<double>* V, long long ldv, KrylovDev& k,
                          hipStream_t s) {
    hipLaunchKernelGGL(arnoldi_small_kernel, dim3(1), dim3(SB), 0, s, N, j, w, V, ldv, k);
}

// Sum over a wave into lane 63 with DPP lane moves (no LDS traffic): pairs and
// quads (quad permutations), half rows and rows (mirrors), then row 0 into row
// 1 and row 2 into row 3 (broadcast of lanes 15 and 47), then rows 0-1 into
// rows 2-3 (broadcast of lane 31).  Fixed order; only lane 63 holds the total.
// All 64 lanes must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_last(double v) {
    v += dpp_f64<0xb1, 0xf>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4e, 0xf>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141, 0xf>(v);   // row_half_mirror
    v += dpp_f64<0x140, 0xf>(v);   // row_mirror
    v += dpp_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return v;
}
__device__ __forceinline__ void wave_sum_last4(double& a, double& b, double& c, double& d) {
    a = wave_sum_last(a);
    b = wave_sum_last(b);
    c = wave_sum_last(c);
    d = wave_sum_last(d);
}
__device__ __forceinline__ double lane63(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over a wave with the same bits in every lane (lane 63's total, read by
// all lanes).  All 64 lanes must be active.
__device__ __forceinline__ void wave_sum2(double& a, double& b) {
    a = lane63(wave_sum_last(a));
    b = lane63(wave_sum_last(b));
}

// Deterministic grid-wide complex sum for a cooperatively launched grid
// (all workgroups resident), without a barrier.  Each block publishes its
// partial as four 64-bit words, each holding 32 bits of the value in its high
// half and, in its low half, a tag unique to (launch, round).  Wave 0 of every
// block polls the words of all blocks until every tag matches, adds the
// partials in block order (lane-strided, then a fixed-order wave sum, so every block gets
// identical bits) and hands the sum to the other waves through LDS.  The words
// are written and read as single-copy-atomic 64-bit accesses at device scope,
// so a matching tag implies the value bits beside it are current; no other
// memory is exchanged during the step, so no fence is needed.  Slots are
// double-buffered by round parity: a block cannot overwrite round r's slot
// with round r + 2 before every block has published round r + 1, which each
// does only after reading round r.  The wait is bounded: after ~2^20 polls the
// lane sets the timeout flag and stops waiting, and every wait that sees the
// flag stops too, so every wave always finishes.
constexpr int kSlotBlocks = 256;   // slots per parity (the grid limit of the cooperative kernels)

// rounds per launch <= restart + 1 <= 201 fit the 8-bit round field
__device__ __forceinline__ unsigned step_tag(int epoch, int round) {
    return 0x80000000u | (((unsigned)epoch & 0x7fffffu) << 8) | (unsigned)round;
}

__device__ __forceinline__ cx<double> exchange_sum(double tr, double ti, unsigned tag, KrylovDev& k, double* shb) {
    unsigned long long* buf = k.slots + (size_t)(tag & 1u) * (4 * kSlotBlocks);
    if (threadIdx.x == 0) {
        const unsigned long long br = (unsigned long long)__double_as_longlong(tr);
        const unsigned long long bi = (unsigned long long)__double_as_longlong(ti);
        unsigned long long* w = buf + 4 * blockIdx.x;
        __hip_atomic_store(w + 0, (br & 0xffffffff00000000ull) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(w + 1, (br << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(w + 2, (bi & 0xffffffff00000000ull) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(w + 3, (bi << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (threadIdx.x < 64) {
        double sr = 0.0, si = 0.0;
        for (int b = threadIdx.x; b < (int)gridDim.x; b += 64) {
            const unsigned long long* w = buf + 4 * b;
            unsigned long long q0, q1, q2, q3;
            int spins = 0;
            for (;;) {
                q0 = __hip_atomic_load(w + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                q1 = __hip_atomic_load(w + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                q2 = __hip_atomic_load(w + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                q3 = __hip_atomic_load(w + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((unsigned)q0 == tag && (unsigned)q1 == tag && (unsigned)q2 == tag && (unsigned)q3 == tag) break;
                __builtin_amdgcn_s_sleep(1);
                if (++spins > k.spin_limit) {
                    atomicExch(&k.ints[5], 1);
                    break;
                }
                // after a timeout anywhere, later waits end quickly too
                if ((spins & 1023) == 0 && __hip_atomic_load(&k.ints[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    break;
            }
            sr += __longlong_as_double((long long)((q0 & 0xffffffff00000000ull) | (q1 >> 32)));
            si += __longlong_as_double((long long)((q2 & 0xffffffff00000000ull) | (q3 >> 32)));
        }
        wave_sum2(sr, si);
        if (threadIdx.x == 0) {
            shb[0] = sr;
            shb[1] = si;
        }
    }
    __syncthreads();
    return {shb[0], shb[1]};
}

// Launch epoch of the cooperative Arnoldi kernels: read once at the start
// (atomically, so it is never re-read), bumped by block 0 after its last
// round; every block has read it before block 0 can pass round 0.
__device__ __forceinline__ int step_epoch(KrylovDev& k) {
    return __hip_atomic_load(&k.ints[6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void next_epoch(KrylovDev& k, int epoch) {
    if (blockIdx.x == 0 && threadIdx.x == 0)
        __hip_atomic_store(&k.ints[6], epoch + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block partial (tree in LDS) followed by the grid-wide exchange.
__device__ __forceinline__ cx<double> grid_sum(double sr, double si, unsigned tag, KrylovDev& k, double* sh,
                                               double* shb) {
    block_sum2(sr, si, sh);
    return exchange_sum(sr, si, tag, k, shb);
}

// One whole Arnoldi step across a cooperatively launched grid: modified
// Gram-Schmidt of w against V[0..j] (one grid-wide reduction per basis
// vector, in order), hn = ||w||, the Givens update (block 0) and w /= hn.
__global__ __launch_bounds__(RB) void arnoldi_coop_kernel(long long N, int j, cx<double>* __restrict__ w,
                                                          const cx<double>* __restrict__ V, long long ldv,
                                                          KrylovDev k) {
    __shared__ double sh[2 * RB];
    __shared__ double shb[2];
    const long long stride = (long long)gridDim.x * RB;
    const long long t0 = (long long)blockIdx.x * RB + threadIdx.x;
    const int ldh = k.m + 1;
    const int epoch = step_epoch(k);
    int round = 0;
    for (int i = 0; i <= j; ++i, ++round) {
        const cx<double>* vi = V + (size_t)i * ldv;
        double sr = 0.0, si = 0.0;
        for (long long t = t0; t < N; t += stride) {
            const cx<double> cv = vi[t], wv = w[t];
            sr += cv.re * wv.re + cv.im * wv.im;
            si += cv.re * wv.im - cv.im * wv.re;
        }
        const cx<double> h = grid_sum(sr, si, step_tag(epoch, round), k, sh, shb);
        if (blockIdx.x == 0 && threadIdx.x == 0) k.H[(size_t)j * ldh + i] = h;
        for (long long t = t0; t < N; t += stride) {
            const cx<double> cv = vi[t];
            cx<double> wv = w[t];
            wv.re -= h.re * cv.re - h.im * cv.im;
            wv.im -= h.re * cv.im + h.im * cv.re;
            w[t] = wv;
        }
    }
    double nr = 0.0;
    for (long long t = t0; t < N; t += stride) {
        const cx<double> wv = w[t];
        nr += wv.re * wv.re + wv.im * wv.im;
    }
    const double hn = sqrt(grid_sum(nr, 0.0, step_tag(epoch, round), k, sh, shb).re);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int tmo = __hip_atomic_load(&k.ints[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        givens_column(k, j, hn);
        if (k.hstep) publish_step(k, j, k.scal[2], k.ints[1], tmo);
    }
    next_epoch(k, epoch);
    for (long long t = t0; t < N; t += stride) {
        const cx<double> wv = w[t];
        w[t] = hn == 0.0 ? cx<double>{0.0, 0.0} : cx<double>{wv.re / hn, wv.im / hn};
    }
}

// Register-resident variant for N <= 256 * RB * R: every thread keeps its R
// entries of w and of the current basis vector in registers, prefetches the
// next basis vector before the grid-wide exchange (it does not depend on h),
// and forms its block partial with wave sums plus one ordered pass over
// the four waves.  Same MGS order and one grid-wide exchange per projection as
// arnoldi_coop_kernel.

__device__ __forceinline__ cx<double> grid_sum_reg(double sr, double si, unsigned tag, KrylovDev& k, double* sh,
                                                   double* shb) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    sr = wave_sum_last(sr);
    si = wave_sum_last(si);
    if (lane == 63) {
        sh[2 * wave] = sr;
        sh[2 * wave + 1] = si;
    }
    __syncthreads();
    double tr = 0.0, ti = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < RB / 64; ++w) {
            tr += sh[2 * w];
            ti += sh[2 * w + 1];
        }
    }
    return exchange_sum(tr, ti, tag, k, shb);
}

template <int R>
__global__ __launch_bounds__(RB) void arnoldi_reg_kernel(long long N, int j, cx<double>* __restrict__ w,
                                                         const cx<double>* __restrict__ V, long long ldv,
                                                         KrylovDev k) {
    __shared__ double sh[2 * (RB / 64)];
    __shared__ double shb[2];
    __shared__ cx<double> shc[kMaxRestart + 1];   // block 0: column j of H
    __shared__ double scs[kMaxRestart];            // block 0: rotations 0..j-1
    __shared__ cx<double> ssn[kMaxRestart];
    const long long stride = (long long)gridDim.x * RB;
    const long long t0 = (long long)blockIdx.x * RB + threadIdx.x;
    const int ldh = k.m + 1;
    const int epoch = step_epoch(k);
    cx<double> gj = {0.0, 0.0};
    int broke = 0;
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < j; i += RB) {
            scs[i] = k.cs[i];
            ssn[i] = k.sn[i];
        }
        if (threadIdx.x == 0) {
            gj = k.g[j];
            broke = k.ints[1];
        }
    }
    cx<double> wr[R], vr[R], vn[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const long long t = t0 + r * stride;
        wr[r] = t < N ? w[t] : cx<double>{0.0, 0.0};
        vr[r] = t < N ? V[t] : cx<double>{0.0, 0.0};
    }
    int round = 0;
    for (int i = 0; i <= j; ++i, ++round) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            sr += vr[r].re * wr[r].re + vr[r].im * wr[r].im;
            si += vr[r].re * wr[r].im - vr[r].im * wr[r].re;
        }
        if (i < j) {
            const cx<double>* vi1 = V + (size_t)(i + 1) * ldv;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const long long t = t0 + r * stride;
                vn[r] = t < N ? vi1[t] : cx<double>{0.0, 0.0};
            }
        }
        const cx<double> h = grid_sum_reg(sr, si, step_tag(epoch, round), k, sh, shb);
        if (blockIdx.x == 0 && threadIdx.x == 0) shc[i] = h;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            wr[r].re -= h.re * vr[r].re - h.im * vr[r].im;
            wr[r].im -= h.re * vr[r].im + h.im * vr[r].re;
            vr[r] = vn[r];
        }
    }
    double nr = 0.0, zero = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) nr += wr[r].re * wr[r].re + wr[r].im * wr[r].im;
    const double hn = sqrt(grid_sum_reg(nr, zero, step_tag(epoch, round), k, sh, shb).re);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int tmo = __hip_atomic_load(&k.ints[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        double c;
        cx<double> sg;
        givens_rotate(shc, scs, ssn, j, hn, c, sg);
        for (int i = 0; i <= j + 1; ++i) k.H[(size_t)j * ldh + i] = shc[i];
        const double gabs = givens_finish(k, j, hn, c, sg, gj, broke);
        if (k.hstep) publish_step(k, j, gabs, (broke || hn == 0.0) ? 1 : 0, tmo);
    }
    next_epoch(k, epoch);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const long long t = t0 + r * stride;
        if (t < N) w[t] = hn == 0.0 ? cx<double>{0.0, 0.0} : cx<double>{wr[r].re / hn, wr[r].im / hn};
    }
}

// LDS-resident variant for the vectors past the register kernels (N up to
// 256 * RB * R): every thread keeps its R entries of w in the LDS of its block
// (dynamic, R * RB complex) and the current basis vector in registers; the next
// basis vector is loaded after w's update (no room for a second register
// copy).  Same MGS order and one grid-wide exchange per projection as
// arnoldi_coop_kernel, but V and w cross HBM once per step instead of V twice
// and w three times per projection.
constexpr int kLdsR = 36;
template <int R>
__global__ __launch_bounds__(RB) void arnoldi_lds_kernel(long long N, int j, cx<double>* __restrict__ w,
                                                         const cx<double>* __restrict__ V, long long ldv,
                                                         KrylovDev k) {
    extern __shared__ cx<double> wl[];            // [R][RB]: this block's entries of w
    __shared__ double sh[2 * (RB / 64)];
    __shared__ double shb[2];
    __shared__ cx<double> shc[kMaxRestart + 1];   // block 0: column j of H
    __shared__ double scs[kMaxRestart];            // block 0: rotations 0..j-1
    __shared__ cx<double> ssn[kMaxRestart];
    const long long stride = (long long)gridDim.x * RB;
    const long long t0 = (long long)blockIdx.x * RB + threadIdx.x;
    const int ldh = k.m + 1;
    const int epoch = step_epoch(k);
    cx<double> gj = {0.0, 0.0};
    int broke = 0;
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < j; i += RB) {
            scs[i] = k.cs[i];
            ssn[i] = k.sn[i];
        }
        if (threadIdx.x == 0) {
            gj = k.g[j];
            broke = k.ints[1];
        }
    }
    cx<double> vr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const long long t = t0 + r * stride;
        wl[r * RB + threadIdx.x] = t < N ? w[t] : cx<double>{0.0, 0.0};
        vr[r] = t < N ? V[t] : cx<double>{0.0, 0.0};
    }
    int round = 0;
    for (int i = 0; i <= j; ++i, ++round) {
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const cx<double> wv = wl[r * RB + threadIdx.x];
            sr += vr[r].re * wv.re + vr[r].im * wv.im;
            si += vr[r].re * wv.im - vr[r].im * wv.re;
        }
        const cx<double> h = grid_sum_reg(sr, si, step_tag(epoch, round), k, sh, shb);
        if (blockIdx.x == 0 && threadIdx.x == 0) shc[i] = h;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cx<double> wv = wl[r * RB + threadIdx.x];
            wv.re -= h.re * vr[r].re - h.im * vr[r].im;
            wv.im -= h.re * vr[r].im + h.im * vr[r].re;
            wl[r * RB + threadIdx.x] = wv;
        }
        if (i < j) {
            const cx<double>* vi1 = V + (size_t)(i + 1) * ldv;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const long long t = t0 + r * stride;
                vr[r] = t < N ? vi1[t] : cx<double>{0.0, 0.0};
            }
        }
    }
    double nr = 0.0, zero = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const cx<double> wv = wl[r * RB + threadIdx.x];
        nr += wv.re * wv.re + wv.im * wv.im;
    }
    const double hn = sqrt(grid_sum_reg(nr, zero, step_tag(epoch, round), k, sh, shb).re);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int tmo = __hip_atomic_load(&k.ints[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        double c;
        cx<double> sg;
        givens_rotate(shc, scs, ssn, j, hn, c, sg);
        for (int i = 0; i <= j + 1; ++i) k.H[(size_t)j * ldh + i] = shc[i];
        const double gabs = givens_finish(k, j, hn, c, sg, gj, broke);
        if (k.hstep) publish_step(k, j, gabs, (broke || hn == 0.0) ? 1 : 0, tmo);
    }
    next_epoch(k, epoch);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const long long t = t0 + r * stride;
        const cx<double> wv = wl[r * RB + threadIdx.x];
        if (t < N) w[t] = hn == 0.0 ? cx<double>{0.0, 0.0} : cx<double>{wv.re / hn, wv.im / hn};
    }
}

// One Arnoldi step in the one-reduction form of modified Gram-Schmidt (the
// inverse compact-WY form of Swirydowicz, Langou, Ananthan, Yang and Thomas,
// 2020).  MGS subtracts the projections in order, so its coefficients satisfy
// h_i = v_i^H w - sum_{k<i} (v_i^H v_k) h_k, that is (I + L) h = V^H w with L
// the strictly lower part of V^H V; this holds for the computed, not exactly
// orthonormal, basis too, so solving that triangular system gives the MGS
// projection w - V h without a chain of j + 1 dependent reductions.  Per step:
//   pass 1: c = V^H w and the new Gram row v_j^H v_k (k < j), block partials
//           (each wave takes every fourth basis vector over the block's 1024
//           entries, w and v_j staged in LDS);
//   one grid-wide exchange of those 2j + 1 values (tagged words as in
//           exchange_sum, summed in block order by groups of eight);
//   forward substitution for h with rows 1..j-1 of L kept from earlier steps
//           (same operations in every block: identical h everywhere);
//   pass 2: w -= sum_i h_i v_i in order of i;
//   hn = ||w|| (scalar exchange), the Givens update, w /= hn.
// Block 0 stores column j of H and row j of L.  A launch writes the 2j + 1
// exchange slots it uses and, when 2^20 launches have passed since the last
// such write, zeros in the rest, so no slot read holds an older launch's word
// with a matching tag.
constexpr int OR_R = 4;                 // entries of w per thread
constexpr int OR_CH = RB * OR_R;        // entries per block
constexpr int OR_QMAX = 2 * kOneRedMaxM - 1;

__global__ __launch_bounds__(RB) void arnoldi_onered_kernel(long long N, int j, cx<double>* __restrict__ w,
                                                            const cx<double>* __restrict__ V, long long ldv,
                                                            KrylovDev k) {
    __shared__ cx<double> sw[OR_CH];    // w's entries of this block; later the group partials
    __shared__ cx<double> sv[OR_CH];    // v_j's entries of this block
    __shared__ cx<double> sL[kOneRedMaxM * (kOneRedMaxM - 1) / 2];
    __shared__ cx<double> sq[OR_QMAX];  // block partials, then grid sums
    __shared__ cx<double> shh[kOneRedMaxM + 1];  // h, then the rotated column j of H
    __shared__ double scs[kOneRedMaxM];            // block 0: rotations 0..j-1
    __shared__ cx<double> ssn[kOneRedMaxM];
    __shared__ double sh[2 * (RB / 64)];
    __shared__ double shb[2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long stride = (long long)gridDim.x * RB;
    const long long base = (long long)blockIdx.x * RB;
    const int ldh = k.m + 1;
    const int epoch = step_epoch(k);
    const bool refresh = (unsigned)(epoch - __hip_atomic_load(&k.ints[7], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >=
                         (1u << 20) || epoch == 0;
    const int Q = 2 * j + 1;
    const cx<double>* vj = V + (size_t)j * ldv;
    // pass 1 reads: wave `wave` takes v_i for i = wave, wave + 4, ...; lane
    // covers the block positions p = lane + 64 q (q = 0..15)
    constexpr int PQ = OR_CH / 64;
    auto load_vec = [&](int i, cx<double>* dst) {
        const cx<double>* vi = V + (size_t)i * ldv;
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            const int p = lane + 64 * q;
            const long long t = base + (p & (RB - 1)) + (long long)(p / RB) * stride;
            dst[q] = vi[t < N ? t : N - 1];
        }
    };
    cx<double> cur[PQ], nxt[PQ];
    if (wave <= j) load_vec(wave, cur);   // in flight with the loads below
    // block 0, for the Givens update at the end: rotations, g[j] and the flag
    cx<double> gj = {0.0, 0.0};
    int broke = 0;
    if (blockIdx.x == 0) {
        for (int i = tid; i < j; i += RB) {
            scs[i] = k.cs[i];
            ssn[i] = k.sn[i];
        }
        if (tid == 0) {
            gj = k.g[j];
            broke = k.ints[1];
        }
    }
    // own entries (p = tid + RB r), clamped reads of valid addresses, zero beyond N
    cx<double> wr[OR_R];
#pragma unroll
    for (int r = 0; r < OR_R; ++r) {
        const long long t = base + tid + r * stride;
        const long long tc = t < N ? t : N - 1;
        const cx<double> a = w[tc], b = vj[tc];
        wr[r] = t < N ? a : cx<double>{0.0, 0.0};
        sw[tid + RB * r] = wr[r];
        sv[tid + RB * r] = t < N ? b : cx<double>{0.0, 0.0};
    }
    // rows 1..j-1 of L (packed) for the substitution
    const int nL = j * (j - 1) / 2;
    for (int i = tid; i < nL; i += RB) sL[i] = k.gram[i];
    __syncthreads();

    // pass 1
    for (int i = wave; i <= j; i += 4) {
        if (i + 4 <= j) load_vec(i + 4, nxt);
        double cr = 0.0, ci = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            // entries beyond N: w and v_j are zero there
            const int p = lane + 64 * q;
            const cx<double> a = cur[q], ww = sw[p], vv = sv[p];
            cr += a.re * ww.re + a.im * ww.im;   // v_i^H w
            ci += a.re * ww.im - a.im * ww.re;
            gr += vv.re * a.re + vv.im * a.im;   // v_j^H v_i
            gi += vv.re * a.im - vv.im * a.re;
        }
        wave_sum_last4(cr, ci, gr, gi);
        if (lane == 63) {
            sq[i] = {cr, ci};
            if (i < j) sq[j + 1 + i] = {gr, gi};
        }
#pragma unroll
        for (int q = 0; q < PQ; ++q) cur[q] = nxt[q];
    }
    __syncthreads();

    // publish this block's 2j + 1 values, four tagged words each; slot (q, b) at
    // q Gp + b (Gp: the grid rounded up to eight blocks)
    const unsigned tag = step_tag(epoch, 0);
    const int qcap = k.qcap;
    const int G = gridDim.x, Gp = (G + 7) & ~7, NG = Gp / 8;
    auto publish = [&](int q, cx<double> v) {
        const unsigned long long br = (unsigned long long)__double_as_longlong(v.re);
        const unsigned long long bi = (unsigned long long)__double_as_longlong(v.im);
        unsigned long long* wd = k.vslots + ((size_t)q * Gp + blockIdx.x) * 4;
        __hip_atomic_store(wd + 0, (br & 0xffffffff00000000ull) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(wd + 1, (br << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(wd + 2, (bi & 0xffffffff00000000ull) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(wd + 3, (bi << 32) | tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    for (int q = tid; q < Q; q += RB) publish(q, sq[q]);
    // pass 2 reads its first eight basis vectors now (they do not depend on h)
    cx<double> vb[8][OR_R];
    auto load_batch = [&](int i0) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + u <= j) {
                const cx<double>* vi = V + (size_t)(i0 + u) * ldv;
#pragma unroll
                for (int r = 0; r < OR_R; ++r) {
                    const long long t = base + tid + r * stride;
                    vb[u][r] = vi[t < N ? t : N - 1];
                }
            }
    };
    load_batch(0);
    // collect: thread t reads slot it = t + RB u (consecutive lanes, consecutive
    // blocks of one value: contiguous words), up to eight slots in flight; the
    // eight lanes of a group of eight blocks then sum them (quad swaps and the
    // half-row mirror: block order fixed, the same bits in all eight lanes), and
    // the groups are added in order below
    const int items = Q * Gp;
    cx<double>* sp = sw;   // [q][8] group partials (sw is no longer needed)
    for (int it0 = 0; it0 < items; it0 += RB * 8) {
        double vr[8], vi[8];
        unsigned todo = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int it = it0 + tid + RB * u;
            vr[u] = 0.0;
            vi[u] = 0.0;
            if (it < items && it % Gp < G) todo |= 1u << u;
        }
        int spins = 0;
        while (todo) {
            unsigned long long x[8][4];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (todo & (1u << u)) {
                    const unsigned long long* wd = k.vslots + (size_t)(it0 + tid + RB * u) * 4;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        x[u][e] = __hip_atomic_load(wd + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if ((todo & (1u << u)) && (unsigned)x[u][0] == tag && (unsigned)x[u][1] == tag &&
                    (unsigned)x[u][2] == tag && (unsigned)x[u][3] == tag) {
                    vr[u] = __longlong_as_double((long long)((x[u][0] & 0xffffffff00000000ull) | (x[u][1] >> 32)));
                    vi[u] = __longlong_as_double((long long)((x[u][2] & 0xffffffff00000000ull) | (x[u][3] >> 32)));
                    todo &= ~(1u << u);
                }
            if (!todo) break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > k.spin_limit) {
                atomicExch(&k.ints[5], 1);
                break;
            }
            if ((spins & 1023) == 0 && __hip_atomic_load(&k.ints[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                break;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            double ar = vr[u], ai = vi[u];
            ar += dpp_f64<0xb1, 0xf>(ar);    // quad_perm [1,0,3,2]
            ai += dpp_f64<0xb1, 0xf>(ai);
            ar += dpp_f64<0x4e, 0xf>(ar);    // quad_perm [2,3,0,1]
            ai += dpp_f64<0x4e, 0xf>(ai);
            ar += dpp_f64<0x141, 0xf>(ar);   // row_half_mirror
            ai += dpp_f64<0x141, 0xf>(ai);
            const int it = it0 + tid + RB * u;
            if ((tid & 7) == 0 && it < items) {
                const int q = it / Gp;
                sp[q * 8 + (it - q * Gp) / 8] = {ar, ai};
            }
        }
    }
    __syncthreads();
    for (int q = tid; q < Q; q += RB) {
        double ar = 0.0, ai = 0.0;
        for (int g = 0; g < NG; ++g) {
            ar += sp[q * 8 + g].re;
            ai += sp[q * 8 + g].im;
        }
        sq[q] = {ar, ai};
    }
    // Once 2^20 launches have passed since the last full write (ints[7]; any
    // Arnoldi launch advances the epoch), the slots this step does not use get
    // this launch's tag too (zero values): no slot then goes unwritten for 2^23
    // launches (the epoch field of the tag), so a launch never reads a word that
    // carries its own tag from an older launch.
    if (refresh)
        for (int q = Q + tid; q < qcap; q += RB) publish(q, cx<double>{0.0, 0.0});
    __syncthreads();

    // (I + L) h = c by forward substitution in wave 0, lane i holding row i
    // (row j from the sums); the row entries are read eight columns ahead
    if (wave == 0) {
        const bool row = lane <= j;
        cx<double> x = row ? sq[lane] : cx<double>{0.0, 0.0};
        const cx<double>* Lrow = lane < j ? sL + lane * (lane - 1) / 2 : sq + j + 1;
        for (int k0 = 0; k0 < j; k0 += 8) {
            cx<double> lv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int kk = k0 + u;
                lv[u] = (row && kk < lane) ? Lrow[kk] : cx<double>{0.0, 0.0};
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int kk = k0 + u;
                if (kk >= j) break;
                const long long hr = __double_as_longlong(x.re), hi = __double_as_longlong(x.im);
                const double h_re = __longlong_as_double(
                    ((long long)__builtin_amdgcn_readlane((int)(hr >> 32), kk) << 32) |
                    (unsigned)__builtin_amdgcn_readlane((int)hr, kk));
                const double h_im = __longlong_as_double(
                    ((long long)__builtin_amdgcn_readlane((int)(hi >> 32), kk) << 32) |
                    (unsigned)__builtin_amdgcn_readlane((int)hi, kk));
                if (row && lane > kk) {
                    const cx<double> l = lv[u];
                    x.re -= l.re * h_re - l.im * h_im;
                    x.im -= l.re * h_im + l.im * h_re;
                }
            }
        }
        if (row) shh[lane] = x;
    }
    __syncthreads();
    if (blockIdx.x == 0)
        for (int kk = tid; kk < j; kk += RB) k.gram[j * (j - 1) / 2 + kk] = sq[j + 1 + kk];

    // pass 2: w -= sum_i h_i v_i over this thread's entries, eight vectors at a time
    for (int i0 = 0; i0 <= j; i0 += 8) {
        if (i0 > 0) load_batch(i0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + u <= j) {
                const cx<double> h = shh[i0 + u];
#pragma unroll
                for (int r = 0; r < OR_R; ++r) {
                    wr[r].re -= h.re * vb[u][r].re - h.im * vb[u][r].im;
                    wr[r].im -= h.re * vb[u][r].im + h.im * vb[u][r].re;
                }
            }
    }
    double nr = 0.0, zero = 0.0;
#pragma unroll
    for (int r = 0; r < OR_R; ++r) {
        const long long t = base + tid + r * stride;
        if (t < N) nr += wr[r].re * wr[r].re + wr[r].im * wr[r].im;
    }
    const double hn = sqrt(grid_sum_reg(nr, zero, step_tag(epoch, 1), k, sh, shb).re);
    if (blockIdx.x == 0 && tid == 0) {
        const int tmo = __hip_atomic_load(&k.ints[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        double c;
        cx<double> sg;
        givens_rotate(shh, scs, ssn, j, hn, c, sg);
        for (int i = 0; i <= j + 1; ++i) k.H[(size_t)j * ldh + i] = shh[i];
        const double gabs = givens_finish(k, j, hn, c, sg, gj, broke);
        if (k.hstep) publish_step(k, j, gabs, (broke || hn == 0.0) ? 1 : 0, tmo);
        // every block read ints[7] before publishing (block 0 is past the exchange)
        if (refresh) __hip_atomic_store(&k.ints[7], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    next_epoch(k, epoch);
#pragma unroll
    for (int r = 0; r < OR_R; ++r) {
        const long long t = base + tid + r * stride;
        if (t < N) w[t] = hn == 0.0 ? cx<double>{0.0, 0.0} : cx<double>{wr[r].re / hn, wr[r].im / hn};
    }
}

// Blocks of RB threads of kernel fn that the current device holds at once
// (cached per device and kernel).
static long long resident_capacity(const void* fn, size_t shm = 0) {
    static std::mutex mu;
    static std::map<std::pair<int, const void*>, long long> cache;
    int dev = 0;
    HH_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({dev, fn});
    if (it != cache.end()) return it->second;
    if (shm > 0)   // dynamic LDS beyond the default limit, allowed once per kernel and device
        HH_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    int per_cu = 0, cus = 0;
    HH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, RB, shm));
    HH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const long long cap = (long long)per_cu * cus;
    cache[{dev, fn}] = cap;
    return cap;
}

int coop_blocks(long long N) {
    long long b = (N + 8 * RB - 1) / (8 * RB);
    if (b < 1) b = 1;
    if (b > 256) b = 256;
    return (int)b;
}

bool launch_arnoldi_grid(long long N, int j, cx<double>* w, const cx<double>* V, long long ldv, KrylovDev& k,
                         hipStream_t s, int concurrent, bool coop_ok, bool one_reduce) {
    void* args[] = {&N, &j, &w, &V, &ldv, &k};
    if (one_reduce && k.qcap > 0 && j < k.m && k.m <= kOneRedMaxM) {
        const long long b1 = (N + OR_CH - 1) / OR_CH;
        const void* f1 = (const void*)arnoldi_onered_kernel;
        if (b1 <= kOneRedMaxBlocks && b1 * concurrent <= resident_capacity(f1)) {
            HH_HIP(hipLaunchKernel(f1, dim3((unsigned)b1), dim3(RB), args, 0, s));
            return true;
        }
    }
    const void* fn = (const void*)arnoldi_coop_kernel;
    long long blocks = coop_blocks(N);
    // register-resident kernel: R entries per thread, at most 256 blocks
    auto pick = [&](int R, const void* f) {
        if (fn != (const void*)arnoldi_coop_kernel || N > 256LL * RB * R) return;
        fn = f;
        blocks = std::max(1LL, (N + (long long)RB * R - 1) / ((long long)RB * R));
    };
    pick(4, (const void*)arnoldi_reg_kernel<4>);
    pick(8, (const void*)arnoldi_reg_kernel<8>);
    pick(16, (const void*)arnoldi_reg_kernel<16>);
    // past the register kernels: w in LDS, kLdsR entries per thread, one block per CU
    size_t shm = 0;
    if (fn == (const void*)arnoldi_coop_kernel && N <= 256LL * RB * kLdsR) {
        fn = (const void*)arnoldi_lds_kernel<kLdsR>;
        blocks = std::max(1LL, (N + (long long)RB * kLdsR - 1) / ((long long)RB * kLdsR));
        shm = (size_t)RB * kLdsR * sizeof(cx<double>);
    }
    if (blocks > kSlotBlocks) throw Err{HH_EINVAL, "cooperative Arnoldi grid exceeds the exchange slots"};
    // A cooperative launch guarantees that all blocks are resident, but the
    // runtime serves it from a separate hardware queue: two cross-queue hand-offs
    // per step.  A grid small enough that `concurrent` such grids (at most that
    // many Arnoldi steps run at once: four, the workers of a batched solve) fit
    // in the blocks the device holds at once is
    // launched on the stream's own queue instead: its blocks are placed as soon
    // as CUs are free, and since the exchange's waits are bounded a shortage of
    // CUs can only end in the timeout flag, never a hang.  Otherwise the
    // cooperative launch when allowed; else nothing is launched (false).
    const long long cap = resident_capacity(fn, shm);
    if (blocks * concurrent <= cap) {
        HH_HIP(hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(RB), args, shm, s));
        return true;
    }
    if (!coop_ok || blocks > cap) return false;
    hipError_t e = hipLaunchCooperativeKernel(fn, dim3((unsigned)blocks), dim3(RB), args, shm, s);
    if (e != hipSuccess) throw Err{HH_EHIP, std::string("cooperative Arnoldi launch: ") + hipGetErrorString(e)};
    return true;
}

// ||x||^2 into *out (plain reduction).
__global__ __launch_bounds__(RB) void norm2_kernel(long long N, const cx<double>* __restrict__ x, double* out,
                                                   int* counter, cx<double>* partials) {
    __shared__ double sh[2 * RB];
    __shared__ bool flag;
    double sr = 0.0, dummy = 0.0;
    const long long stride = (long long)gridDim.x * RB;
    for (long long t = (long long)blockIdx.x * RB + threadIdx.x; t < N; t += stride) {
        const cx<double> v = x[t];
        sr += v.re * v.re + v.im * v.im;
    }
    block_sum2(sr, dummy, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = {sr, 0.0};
    if (!last_block(counter, &flag)) return;
    double tr, ti;
    sum_partials(partials, gridDim.x, tr, ti, sh);
    if (threadIdx.x == 0) {
        *out = tr;
        *counter = 0;
    }
}

void launch_dot_norm2(long long N, const cx<double>* x, double* out, int* counter, cx<double>* partials,
                      hipStream_t s) {
    meter(16.0 * N, 4.0 * N);
    hipLaunchKernelGGL(norm2_kernel, dim3(reduction_blocks(N)), dim3(RB), 0, s, N, x, out, counter, partials);
}

// Start of an Arnoldi cycle: beta = ||r||, g = (beta, 0, ...), counters reset.
__global__ void cycle_init_kernel(KrylovDev k) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double beta = sqrt(k.scal[3]);
    k.scal[0] = beta;
    for (int i = 0; i <= k.m; ++i) k.g[i] = {0.0, 0.0};
    k.g[0] = {beta, 0.0};
    k.scal[2] = beta;
    k.ints[0] = 0;
    k.ints[1] = (beta == 0.0) ? 1 : 0;
}

void launch_norm_init(long long N, const cx<double>* r, KrylovDev& k, hipStream_t s) {
    launch_dot_norm2(N, r, &k.scal[3], &k.ints[2], k.partials, s);
    hipLaunchKernelGGL(cycle_init_kernel, dim3(1), dim3(1), 0, s, k);
}

// y = x / *by, with a zero divisor giving y = 0.
__global__ void scale_by_kernel(long long N, const cx<double>* x, cx<double>* y, const double* by) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double d = *by;
    if (d == 0.0) {
        y[i] = {0.0, 0.0};
        return;
    }
    const cx<double> v = x[i];
    y[i] = {v.re / d, v.im / d};
}
void launch_scale_by(long long N, const cx<double>* x, cx<double>* y, const double* by, hipStream_t s) {
    meter(32.0 * N, 2.0 * N);
    hipLaunchKernelGGL(scale_by_kernel, dim3(grid1d(N, 256)), dim3(256), 0, s, N, x, y, by);
}

// Back substitution R y = g on the first n rows (R: rotated Hessenberg); n is
// ncols when given (>= 0), else the device count of completed Arnoldi steps.
// One wave, column by column from the last: every lane forms y_i from the
// updated s_i, then lanes r < i subtract R[r][i] y_i from s_r (s in LDS; R's
// upper triangle staged in LDS, packed by columns, when n <= LSQ_COLS).
constexpr int LSQ_COLS = 64;
__global__ __launch_bounds__(64) void lsq_kernel(KrylovDev k, int ncols) {
    __shared__ cx<double> sR[LSQ_COLS * (LSQ_COLS + 1) / 2];
    __shared__ cx<double> sS[kMaxRestart];
    const int lane = threadIdx.x;
    const int n = ncols >= 0 ? ncols : k.ints[0], ldh = k.m + 1;
    for (int r = lane; r < n; r += 64) sS[r] = k.g[r];
    const bool staged = n <= LSQ_COLS;
    if (staged) {
        // entry (r, c), r <= c, at c(c+1)/2 + r; eight loads in flight per lane
        const int T = n * (n + 1) / 2;
        for (int i0 = 0; i0 < T; i0 += 64 * 8) {
            cx<double> v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = i0 + lane + 64 * u;
                if (idx < T) {
                    int c = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
                    if ((c + 1) * (c + 2) / 2 <= idx) ++c;
                    if (c * (c + 1) / 2 > idx) --c;
                    v[u] = k.H[(size_t)c * ldh + (idx - c * (c + 1) / 2)];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = i0 + lane + 64 * u;
                if (idx < T) sR[idx] = v[u];
            }
        }
    }
    __syncthreads();
    for (int i = n - 1; i >= 0; --i) {
        const cx<double> si = sS[i];
        const cx<double> d = staged ? sR[i * (i + 1) / 2 + i] : k.H[(size_t)i * ldh + i];
        const double den = d.re * d.re + d.im * d.im;
        const cx<double> y = {(si.re * d.re + si.im * d.im) / den, (si.im * d.re - si.re * d.im) / den};
        if (lane == 0) k.y[i] = y;
        for (int r = lane; r < i; r += 64) {
            const cx<double> h = staged ? sR[i * (i + 1) / 2 + r] : k.H[(size_t)i * ldh + r];
            const cx<double> p = cmul(h, y);
            cx<double> t = sS[r];
            t.re -= p.re;
            t.im -= p.im;
            sS[r] = t;
        }
    }
}
void launch_lsq(KrylovDev& k, hipStream_t s, int ncols) {
    hipLaunchKernelGGL(lsq_kernel, dim3(1), dim3(64), 0, s, k, ncols);
}

// u (+)= sum_{i < n} Z_i y_i, accumulated in increasing i (n as in lsq_kernel).
__global__ void update_kernel(long long N, const cx<double>* __restrict__ Z, long long ldz, KrylovDev k,
                              cx<double>* __restrict__ u, int accumulate, int ncols) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    const int n = ncols >= 0 ? ncols : k.ints[0];
    double dr = 0.0, di = 0.0;
#pragma unroll 8
    for (int i = 0; i < n; ++i) {
        const cx<double> z = Z[(size_t)i * ldz + t];
        const cx<double> y = k.y[i];
        dr += z.re * y.re - z.im * y.im;
        di += z.re * y.im + z.im * y.re;
    }
    if (accumulate) {
        const cx<double> o = u[t];
        u[t] = {o.re + dr, o.im + di};
    } else {
        u[t] = {dr, di};
    }
}
void launch_update(long long N, const cx<double>* Z, long long ldz, KrylovDev& k, cx<double>* u, int accumulate,
                   hipStream_t s, int ncols) {
    const double n = ncols >= 0 ? ncols : k.m;
    meter(16.0 * N * (n + (accumulate ? 2.0 : 1.0)), 8.0 * N * n);
    hipLaunchKernelGGL(update_kernel, dim3(grid1d(N, 256)), dim3(256), 0, s, N, Z, ldz, k, u, accumulate, ncols);
}

}  // namespace hh
