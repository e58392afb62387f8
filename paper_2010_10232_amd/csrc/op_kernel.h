// HIP kernels for gfx950 (CDNA4, wave64).
//
// Level operator y = K x - alpha M_k x (section 2.3: stiffness plus
// k^2-weighted mass; alpha = 1 gives A, alpha = beta1 + i beta2 the CSLP of
// section 3) on tensor-product B-splines, with fused epilogues for the residual
// b - Op x and the damped Jacobi sweep x + omega D^-1 (b - Op x).
//
// Layout: complex vectors interleaved (re, im), row-major [n2][n1] (x fastest).
// One workgroup = one wave of 64 lanes owns a 64-column x TY-row output tile.
// The input tile plus a p-wide halo is staged in LDS with coalesced row loads;
// each lane then walks the tile rows, applying the x-direction bands of its own
// column from LDS and scattering into TY register accumulators through the
// y-direction bands (separable apply of My (x) Kx + Ky (x) Mx).  The mass part is
//   KIND_SEP      constant k:  k^2 My (x) Mx, folded into the same pass;
//   KIND_VARFINE  finest level, k^2 per element: per element row e2 the lane
//                 builds the k^2-weighted x-band of its column from the element
//                 mass blocks, applies it to the p+1 rows of that element row
//                 and scatters through the y element block (sum factorisation);
//   KIND_STENCIL  coarse level, k^2 per finest element: stored Galerkin stencil,
//                 (2p+1)^2 coefficients per unknown in SoA order (coalesced).
#pragma once
#include "hh_internal.h"

namespace hh {

template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// --------------------------------------------------------------------------
// Level operator
// --------------------------------------------------------------------------
template <int PX, int PY, int TY, int KIND, int MODE, class T>
__global__ __launch_bounds__(64) void op_kernel(OpArgs<T> a) {
    constexpr int TX = 64;
    constexpr int BX = 2 * PX + 1, BY = 2 * PY + 1;
    constexpr int LW = TX + 2 * PX, LH = TY + 2 * PY;
    __shared__ cx<T> xs[LH][LW];
    const int lane = threadIdx.x;
    const int C0 = blockIdx.x * TX, R0 = blockIdx.y * TY;
    const int n1 = a.n1, n2 = a.n2;

    for (int idx = lane; idx < LH * LW; idx += TX) {
        const int r = idx / LW, c = idx - r * LW;
        const int J2 = R0 - PY + r, J1 = C0 - PX + c;
        cx<T> v = {T(0), T(0)};
        if (J2 >= 0 && J2 < n2 && J1 >= 0 && J1 < n1) v = a.x[(size_t)J2 * n1 + J1];
        xs[r][c] = v;
    }
    __syncthreads();

    const int I1 = C0 + lane;
    const int I1c = I1 < n1 ? I1 : n1 - 1;
    T kx[BX], mx[BX];
#pragma unroll
    for (int d = 0; d < BX; ++d) {
        kx[d] = (T)a.Kx[(size_t)I1c * BX + d];
        mx[d] = (T)a.Mx[(size_t)I1c * BX + d];
    }
    T accr[TY], acci[TY], mr[TY], mi[TY];
#pragma unroll
    for (int t = 0; t < TY; ++t) accr[t] = acci[t] = mr[t] = mi[t] = T(0);

    const T are = a.are, aim = a.aim;
    const T k2c = (T)a.k2c;
    // stiffness part (plus the constant-k mass part)
#pragma unroll
    for (int r = 0; r < LH; ++r) {
        T u1r = 0, u1i = 0, u2r = 0, u2i = 0;
#pragma unroll
        for (int d = 0; d < BX; ++d) {
            const cx<T> v = xs[r][lane + d];
            u1r += kx[d] * v.re;
            u1i += kx[d] * v.im;
            u2r += mx[d] * v.re;
            u2i += mx[d] * v.im;
        }
#pragma unroll
        for (int t = 0; t < TY; ++t) {
            const int d2 = r - PY - t;
            if (d2 < -PY || d2 > PY) continue;
            const int I2 = R0 + t;
            if (I2 >= n2) continue;
            const T my = (T)a.My[(size_t)I2 * BY + d2 + PY];
            const T ky = (T)a.Ky[(size_t)I2 * BY + d2 + PY];
            if (KIND == KIND_SEP) {
                const T cr = u1r - k2c * (are * u2r - aim * u2i);
                const T ci = u1i - k2c * (are * u2i + aim * u2r);
                accr[t] += my * cr + ky * u2r;
                acci[t] += my * ci + ky * u2i;
            } else {
                accr[t] += my * u1r + ky * u2r;
                acci[t] += my * u1i + ky * u2i;
            }
        }
    }

    if (KIND == KIND_VARFINE) {
        constexpr int QX = PX + 1, QY = PY + 1;
        // element mass rows of this column: local index a1 in element e1 = I1 + off1 - a1
        T mex[QX][QX];
        bool ev[QX];
#pragma unroll
        for (int a1 = 0; a1 < QX; ++a1) {
            const int e1 = I1c + a.off1 - a1;
            ev[a1] = (e1 >= 0 && e1 < a.nel1);
            const int ec = ev[a1] ? e1 : 0;
#pragma unroll
            for (int c1 = 0; c1 < QX; ++c1) mex[a1][c1] = (T)a.Mex[(size_t)ec * QX * QX + a1 * QX + c1];
        }
#pragma unroll
        for (int s = 0; s < TY + PY; ++s) {
            const int e2 = R0 + a.off2 - PY + s;
            if (e2 < 0 || e2 >= a.nel2) continue;
            T B[BX];
#pragma unroll
            for (int d = 0; d < BX; ++d) B[d] = T(0);
#pragma unroll
            for (int a1 = 0; a1 < QX; ++a1) {
                if (!ev[a1]) continue;
                const T w = (T)a.k2[(size_t)e2 * a.nel1 + (I1c + a.off1 - a1)];
#pragma unroll
                for (int c1 = 0; c1 < QX; ++c1) B[c1 - a1 + PX] += w * mex[a1][c1];
            }
            T tr[QY], ti[QY];
#pragma unroll
            for (int c2 = 0; c2 < QY; ++c2) {
                T sr = 0, si = 0;
#pragma unroll
                for (int d = 0; d < BX; ++d) {
                    const cx<T> v = xs[s + c2][lane + d];
                    sr += B[d] * v.re;
                    si += B[d] * v.im;
                }
                tr[c2] = sr;
                ti[c2] = si;
            }
            const double* mey = a.Mey + (size_t)e2 * QY * QY;
#pragma unroll
            for (int a2 = 0; a2 < QY; ++a2) {
                const int t = s + a2 - PY;
                if (t < 0 || t >= TY) continue;
                T sr = 0, si = 0;
#pragma unroll
                for (int c2 = 0; c2 < QY; ++c2) {
                    const T g = (T)mey[a2 * QY + c2];
                    sr += g * tr[c2];
                    si += g * ti[c2];
                }
                mr[t] += sr;
                mi[t] += si;
            }
        }
    }

    if (KIND == KIND_STENCIL) {
        const size_t N = (size_t)n1 * n2;
#pragma unroll
        for (int t = 0; t < TY; ++t) {
            const int I2 = R0 + t;
            if (I2 >= n2) continue;
            const size_t I = (size_t)I2 * n1 + I1c;
            T sr = 0, si = 0;
#pragma unroll
            for (int d2 = 0; d2 < BY; ++d2)
#pragma unroll
                for (int d1 = 0; d1 < BX; ++d1) {
                    const T c = a.S[(size_t)(d2 * BX + d1) * N + I];
                    const cx<T> v = xs[t + d2][lane + d1];
                    sr += c * v.re;
                    si += c * v.im;
                }
            mr[t] = sr;
            mi[t] = si;
        }
    }

    if (I1 >= n1) return;
#pragma unroll
    for (int t = 0; t < TY; ++t) {
        const int I2 = R0 + t;
        if (I2 >= n2) continue;
        T yr = accr[t], yi = acci[t];
        if (KIND != KIND_SEP) {
            yr -= are * mr[t] - aim * mi[t];
            yi -= are * mi[t] + aim * mr[t];
        }
        const size_t I = (size_t)I2 * n1 + I1;
        cx<T> out;
        if (MODE == MODE_APPLY) {
            out = {yr, yi};
        } else {
            const cx<T> bv = a.b[I];
            const T rr = bv.re - yr, ri = bv.im - yi;
            if (MODE == MODE_RESID) {
                out = {rr, ri};
            } else {
                const cx<T> dv = a.dinv[I];
                const cx<T> xv = xs[t + PY][lane + PX];
                out = {xv.re + a.omega * (dv.re * rr - dv.im * ri),
                       xv.im + a.omega * (dv.re * ri + dv.im * rr)};
            }
        }
        a.y[I] = out;
    }
}

template <int PX, int PY, int KIND, int MODE, class T>
static void launch_op_t(const OpArgs<T>& a, hipStream_t s) {
    constexpr int TY = (PY == 0) ? 1 : (KIND == KIND_SEP ? 16 : 8);
    dim3 grid((a.n1 + 63) / 64, (a.n2 + TY - 1) / TY);
    hipLaunchKernelGGL((op_kernel<PX, PY, TY, KIND, MODE, T>), grid, dim3(64), 0, s, a);
}

template <int PX, int PY, class T>
static void dispatch_km(int kind, int mode, const OpArgs<T>& a, hipStream_t s) {
#define HH_KM(K, M) \
    if (kind == K && mode == M) return launch_op_t<PX, PY, K, M, T>(a, s);
    HH_KM(KIND_SEP, MODE_APPLY)
    HH_KM(KIND_SEP, MODE_RESID)
    HH_KM(KIND_SEP, MODE_SMOOTH)
    HH_KM(KIND_VARFINE, MODE_APPLY)
    HH_KM(KIND_VARFINE, MODE_RESID)
    HH_KM(KIND_VARFINE, MODE_SMOOTH)
    HH_KM(KIND_STENCIL, MODE_APPLY)
    HH_KM(KIND_STENCIL, MODE_RESID)
    HH_KM(KIND_STENCIL, MODE_SMOOTH)
#undef HH_KM
    throw Err{HH_EINVAL, "bad operator kind/mode"};
}

#ifdef HH_OP_DEGREE
template <>
void launch_op_deg<HH_OP_DEGREE, double>(int kind, int mode, int py, const OpArgs<double>& a, hipStream_t s) {
    if (py == 0) return dispatch_km<HH_OP_DEGREE, 0, double>(kind, mode, a, s);
    return dispatch_km<HH_OP_DEGREE, HH_OP_DEGREE, double>(kind, mode, a, s);
}
template <>
void launch_op_deg<HH_OP_DEGREE, float>(int kind, int mode, int py, const OpArgs<float>& a, hipStream_t s) {
    if (py == 0) return dispatch_km<HH_OP_DEGREE, 0, float>(kind, mode, a, s);
    return dispatch_km<HH_OP_DEGREE, HH_OP_DEGREE, float>(kind, mode, a, s);
}
#endif


}  // namespace hh
