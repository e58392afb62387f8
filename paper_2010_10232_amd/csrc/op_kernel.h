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
// Row-marching level operator.  A workgroup is one wave of 64 lanes; it owns
// 64 columns and `ty` output rows, and walks the ty + 2p input rows of its
// strip once, top to bottom.  Each input row is prefetched into registers one
// iteration ahead and then written into a circular LDS buffer that holds the
// last 2p+1 rows (with a p-wide column halo).  Lane c keeps 2p+1 running
// output rows in registers (a sliding window): input row r feeds output rows
// r-2p .. r through the y-bands, after which output row r-2p is complete and
// is written out (with the residual / Jacobi epilogue).
// MODE_RESID with a.xo set: the next level-solve's first damped Jacobi sweep
// from zero on the residual just formed, xo = omega D^-1 r, exactly as
// jacobi0_kernel forms it.
template <class T>
__device__ __forceinline__ cx<T> first_sweep(const OpArgs<T>& a, long long I, cx<T> r) {
    const cx<T> d = a.dinv[I];
    return {a.omega * (d.re * r.re - d.im * r.im), a.omega * (d.re * r.im + d.im * r.re)};
}

template <int PX, int PY, int KIND, int MODE, class T>
__global__ __launch_bounds__(64) void op_kernel(OpArgs<T> a, int ty) {
    constexpr int TX = 64;
    constexpr int BX = 2 * PX + 1, BY = 2 * PY + 1;
    constexpr int QX = PX + 1, QY = PY + 1;
    constexpr int LW = TX + 2 * PX;
    constexpr int W = 2 * PY + 1;                       // window rows
    constexpr int NMEX = (KIND == KIND_VARFINE) ? QX * QX : 1;
    constexpr int NMEY = (KIND == KIND_VARFINE) ? QY * QY : 1;
    __shared__ cx<T> xs[W][LW];
    __shared__ T myS[W][BY], kyS[W][BY];
    __shared__ T mexS[NMEX][TX];
    __shared__ T meyS[NMEY];

    const int lane = threadIdx.x;
    const int C0 = blockIdx.x * TX, R0 = blockIdx.y * ty;
    const int n1 = a.n1, n2 = a.n2;
    const int LH = ty + 2 * PY;
    const int I1 = C0 + lane;
    const int I1c = I1 < n1 ? I1 : n1 - 1;

    T kx[BX], mx[BX];
#pragma unroll
    for (int d = 0; d < BX; ++d) {
        kx[d] = (T)a.Kx[(size_t)I1c * BX + d];
        mx[d] = (T)a.Mx[(size_t)I1c * BX + d];
    }
    if (KIND == KIND_VARFINE) {
#pragma unroll
        for (int a1 = 0; a1 < QX; ++a1) {
            const int e1 = min(max(I1c + a.off1 - a1, 0), a.nel1 - 1);
#pragma unroll
            for (int c1 = 0; c1 < QX; ++c1) mexS[a1 * QX + c1][lane] = (T)a.Mex[(size_t)e1 * QX * QX + a1 * QX + c1];
        }
    }

    // register prefetch of one input row (two columns per lane), its band row,
    // and (VARFINE) the k^2 values / y element block of one element row
    cx<T> px0 = {T(0), T(0)}, px1 = {T(0), T(0)};
    T pband = T(0), pmey = T(0);
    T pk2[QX];
    auto fetch = [&](int r) {
        const int J2 = R0 - PY + r;
        const bool rowok = (J2 >= 0 && J2 < n2);
        const int J1a = C0 - PX + lane, J1b = J1a + TX;
        px0 = (rowok && J1a >= 0 && J1a < n1) ? a.x[(size_t)J2 * n1 + J1a] : cx<T>{T(0), T(0)};
        px1 = (rowok && lane < LW - TX && J1b < n1) ? a.x[(size_t)J2 * n1 + J1b] : cx<T>{T(0), T(0)};
        // band row of output row R0 + r (newest output row fed by input row r)
        const int I2 = R0 + r;
        pband = T(0);
        if (I2 < n2) {
            if (lane < BY) pband = (T)a.My[(size_t)I2 * BY + lane];
            else if (lane < 2 * BY) pband = (T)a.Ky[(size_t)I2 * BY + lane - BY];
        }
        if (KIND == KIND_VARFINE) {
            // element row processed at iteration r: s = r - PY
            const int e2 = R0 + a.off2 - PY + (r - PY);
            const bool eok = (r >= PY && e2 >= 0 && e2 < a.nel2);
#pragma unroll
            for (int a1 = 0; a1 < QX; ++a1) {
                const int e1 = I1 + a.off1 - a1;
                pk2[a1] = (eok && e1 >= 0 && e1 < a.nel1) ? (T)a.k2[(size_t)e2 * a.nel1 + e1] : T(0);
            }
            pmey = (eok && lane < QY * QY) ? (T)a.Mey[(size_t)e2 * QY * QY + lane] : T(0);
        }
    };

    T wr[W], wi[W], vr[W], vi[W];   // window: K part and (non-SEP) mass part
#pragma unroll
    for (int k = 0; k < W; ++k) wr[k] = wi[k] = vr[k] = vi[k] = T(0);
    const T are = a.are, aim = a.aim;
    const T k2c = (T)a.k2c;
    const size_t N = (size_t)n1 * n2;

    fetch(0);
    int slot = 0;   // LDS slot of input row r
#pragma unroll 1
    for (int r = 0; r < LH; ++r) {
        xs[slot][lane] = px0;
        if (lane < LW - TX) xs[slot][lane + TX] = px1;
        if (lane < BY) myS[slot][lane] = pband;
        else if (lane < 2 * BY) kyS[slot][lane - BY] = pband;
        T k2r[QX];
        if (KIND == KIND_VARFINE) {
#pragma unroll
            for (int a1 = 0; a1 < QX; ++a1) k2r[a1] = pk2[a1];
            if (lane < QY * QY) meyS[lane] = pmey;
        }
        __syncthreads();
        if (r + 1 < LH) fetch(r + 1);

        // stiffness part (+ constant-k mass) from input row r
        {
            T u1r = 0, u1i = 0, u2r = 0, u2i = 0;
#pragma unroll
            for (int d = 0; d < BX; ++d) {
                const cx<T> v = xs[slot][lane + d];
                u1r += kx[d] * v.re;
                u1i += kx[d] * v.im;
                u2r += mx[d] * v.re;
                u2i += mx[d] * v.im;
            }
            if (KIND == KIND_SEP) {
                const T cr = u1r - k2c * (are * u2r - aim * u2i);
                const T ci = u1i - k2c * (are * u2i + aim * u2r);
                u1r = cr;
                u1i = ci;
            }
            // window entry k is output row r - 2p + k, whose band slot is
            // that of input row r - 2p + k; the coupling offset is d2 = p - k
            int bs = slot + 1;   // slot of row r - 2p  (== (slot - 2p) mod W)
            if (bs >= W) bs -= W;
#pragma unroll
            for (int k = 0; k < W; ++k) {
                const T my = myS[bs][2 * PY - k], ky = kyS[bs][2 * PY - k];
                wr[k] += my * u1r + ky * u2r;
                wi[k] += my * u1i + ky * u2i;
                if (++bs == W) bs = 0;
            }
        }

        if (KIND == KIND_VARFINE && r >= PY) {
            // element row s = r - p: x rows r-p .. r, output rows r-2p .. r-p
            T B[BX];
#pragma unroll
            for (int d = 0; d < BX; ++d) B[d] = T(0);
#pragma unroll
            for (int a1 = 0; a1 < QX; ++a1)
#pragma unroll
                for (int c1 = 0; c1 < QX; ++c1) B[c1 - a1 + PX] += k2r[a1] * mexS[a1 * QX + c1][lane];
            T tr[QY], ti[QY];
            int xsl = slot + W - PY;   // slot of input row r - p
            if (xsl >= W) xsl -= W;
#pragma unroll
            for (int c2 = 0; c2 < QY; ++c2) {
                T sr = 0, si = 0;
#pragma unroll
                for (int d = 0; d < BX; ++d) {
                    const cx<T> v = xs[xsl][lane + d];
                    sr += B[d] * v.re;
                    si += B[d] * v.im;
                }
                tr[c2] = sr;
                ti[c2] = si;
                if (++xsl == W) xsl = 0;
            }
#pragma unroll
            for (int a2 = 0; a2 < QY; ++a2) {
                T sr = 0, si = 0;
#pragma unroll
                for (int c2 = 0; c2 < QY; ++c2) {
                    const T g = meyS[a2 * QY + c2];
                    sr += g * tr[c2];
                    si += g * ti[c2];
                }
                vr[a2] += sr;   // window entry a2 = output row r - 2p + a2
                vi[a2] += si;
            }
        }

        // output row t = r - 2p is complete
        const int t = r - 2 * PY;
        if (t >= 0 && t < ty && I1 < n1 && R0 + t < n2) {
            const int I2 = R0 + t;
            const size_t I = (size_t)I2 * n1 + I1;
            T yr = wr[0], yi = wi[0];
            if (KIND == KIND_STENCIL) {
                T sr = 0, si = 0;
                int xsl = slot + 1;   // slot of input row r - 2p (= output row t - p)
                if (xsl >= W) xsl -= W;
#pragma unroll
                for (int d2 = 0; d2 < BY; ++d2) {
#pragma unroll
                    for (int d1 = 0; d1 < BX; ++d1) {
                        const T c = a.S[(size_t)(d2 * BX + d1) * N + I];
                        const cx<T> v = xs[xsl][lane + d1];
                        sr += c * v.re;
                        si += c * v.im;
                    }
                    if (++xsl == W) xsl = 0;
                }
                vr[0] = sr;
                vi[0] = si;
            }
            if (KIND != KIND_SEP) {
                yr -= are * vr[0] - aim * vi[0];
                yi -= are * vi[0] + aim * vr[0];
            }
            if ((long long)I == a.bnd_I) {   // radiation condition: + i bnd_im x on the last unknown
                const cx<T> xb = a.x[I];
                yr -= a.bnd_im * xb.im;
                yi += a.bnd_im * xb.re;
            }
            cx<T> out;
            if (MODE == MODE_APPLY) {
                out = {yr, yi};
            } else {
                const cx<T> bv = a.b[I];
                const T rr = bv.re - yr, ri = bv.im - yi;
                if (MODE == MODE_RESID) {
                    out = {rr, ri};
                    if (a.xo) a.xo[I] = first_sweep(a, I, out);
                } else {
                    const cx<T> dv = a.dinv[I];
                    int cs = slot + W - PY;   // slot of input row r - p = output row t
                    if (cs >= W) cs -= W;
                    const cx<T> xv = xs[cs][lane + PX];
                    out = {xv.re + a.omega * (dv.re * rr - dv.im * ri),
                           xv.im + a.omega * (dv.re * ri + dv.im * rr)};
                    if (a.yadd) {
                        const cx<T> q = a.yadd[I];
                        out = {out.re + q.re, out.im + q.im};
                    }
                }
            }
            a.y[I] = out;
        }
        // slide the window
#pragma unroll
        for (int k = 0; k + 1 < W; ++k) {
            wr[k] = wr[k + 1];
            wi[k] = wi[k + 1];
            vr[k] = vr[k + 1];
            vi[k] = vi[k + 1];
        }
        wr[W - 1] = wi[W - 1] = vr[W - 1] = vi[W - 1] = T(0);
        if (++slot == W) slot = 0;
        __syncthreads();
    }
}

// Direct level operator for small levels (constant k or stored stencil): one
// thread per unknown, its bands in registers, the (2px+1)(2py+1) neighbours
// loaded together through the caches.  Same sums as op_kernel: per input row
// the x-direction band products, combined through the y bands in input-row
// order; on small grids this avoids op_kernel's sequential walk over a strip.
template <int PX, int PY, int KIND, int MODE, class T>
__global__ __launch_bounds__(256) void op_direct_kernel(OpArgs<T> a) {
    constexpr int BX = 2 * PX + 1, BY = 2 * PY + 1;
    const int n1 = a.n1, n2 = a.n2;
    const int N = n1 * n2;   // at most kOpDirectMax: 32-bit indices
    const int I = xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
    if (I >= N) return;
    const int I1 = I % n1, I2 = I / n1;
    // all (2p+1)^2 neighbour loads in flight at once, except in FP64 from degree
    // 5 (or with a stored stencil from degree 4): that many values no longer fit
    // the registers (the compiler staged them through private memory), so the
    // rows go one after another, 2p+1 loads in flight each, and the y bands are
    // read per row (a private array indexed by the row would live in memory)
    constexpr bool ROWWISE = sizeof(T) == 8 && (PY >= 5 || (KIND == KIND_STENCIL && PY >= 4));
    T kx[BX], mx[BX], ky[BY], my[BY];
#pragma unroll
    for (int d = 0; d < BX; ++d) {
        kx[d] = (T)a.Kx[(size_t)I1 * BX + d];
        mx[d] = (T)a.Mx[(size_t)I1 * BX + d];
    }
    if constexpr (!ROWWISE) {
#pragma unroll
        for (int d = 0; d < BY; ++d) {
            ky[d] = (T)a.Ky[(size_t)I2 * BY + d];
            my[d] = (T)a.My[(size_t)I2 * BY + d];
        }
    }
    const T are = a.are, aim = a.aim;
    const T k2c = (T)a.k2c;
    T wr = 0, wi = 0, vr = 0, vi = 0;
    // every neighbour is loaded from a valid (clamped) address and replaced by
    // zero when it lies outside the level, so no load waits behind a branch
#pragma unroll ROWWISE ? 1 : BY
    for (int d2 = 0; d2 < BY; ++d2) {
        const int J2 = I2 + d2 - PY;
        const bool ok2 = (unsigned)J2 < (unsigned)n2;
        const size_t row = (size_t)(ok2 ? J2 : I2) * n1;
        T u1r = 0, u1i = 0, u2r = 0, u2i = 0;
#pragma unroll
        for (int d = 0; d < BX; ++d) {
            const int J1 = I1 + d - PX;
            const bool ok = ok2 && (unsigned)J1 < (unsigned)n1;
            // (masking the value here, although the constant-k bands are zero at
            // such neighbours, measured faster: the compiler then keeps every
            // load of the thread in flight)
            const cx<T> raw = a.x[row + (ok ? J1 : I1)];
            const cx<T> v = ok ? raw : cx<T>{T(0), T(0)};
            u1r += kx[d] * v.re;
            u1i += kx[d] * v.im;
            u2r += mx[d] * v.re;
            u2i += mx[d] * v.im;
            if (KIND == KIND_STENCIL) {
                const T c = a.S[(size_t)(d2 * BX + d) * N + I];
                vr += c * v.re;
                vi += c * v.im;
            }
        }
        if (KIND == KIND_SEP) {
            const T cr = u1r - k2c * (are * u2r - aim * u2i);
            const T ci = u1i - k2c * (are * u2i + aim * u2r);
            u1r = cr;
            u1i = ci;
        }
        const T myv = ROWWISE ? (T)a.My[(size_t)I2 * BY + d2] : my[d2];
        const T kyv = ROWWISE ? (T)a.Ky[(size_t)I2 * BY + d2] : ky[d2];
        wr += myv * u1r + kyv * u2r;
        wi += myv * u1i + kyv * u2i;
    }
    T yr = wr, yi = wi;
    if (KIND == KIND_STENCIL) {
        yr -= are * vr - aim * vi;
        yi -= are * vi + aim * vr;
    }
    if (I == a.bnd_I) {   // radiation condition: + i bnd_im x on the last unknown
        const cx<T> xb = a.x[I];
        yr -= a.bnd_im * xb.im;
        yi += a.bnd_im * xb.re;
    }
    cx<T> out;
    if (MODE == MODE_APPLY) {
        out = {yr, yi};
    } else {
        const cx<T> bv = a.b[I];
        const T rr = bv.re - yr, ri = bv.im - yi;
        if (MODE == MODE_RESID) {
            out = {rr, ri};
            if (a.xo) a.xo[I] = first_sweep(a, I, out);
        } else {
            const cx<T> dv = a.dinv[I], xv = a.x[I];
            out = {xv.re + a.omega * (dv.re * rr - dv.im * ri), xv.im + a.omega * (dv.re * ri + dv.im * rr)};
            if (a.yadd) {
                const cx<T> q = a.yadd[I];
                out = {out.re + q.re, out.im + q.im};
            }
        }
    }
    a.y[I] = out;
}



// Stored-stencil level operator (coarse variable-k levels): the Galerkin mass
// stencil has (2px+1)(2py+1) FP64 coefficients per unknown, 648 B at p = 4
// against 16 B for x, so the kernel is a stream of coefficients.  A workgroup
// of four waves owns a 64-column x 4-row output tile; x of the tile and its
// p-wide halo is staged in LDS once (zero outside the level), the column and
// row bands of the tile too, and every thread issues all of its coefficient
// loads (coalesced per stencil entry across the wave) before it uses any.  The
// sums are formed in the same order as op_direct_kernel: per input row the
// band products and the stencil products, combined through the y bands.
constexpr int STC_ROWS = 4;
template <int PX, int PY, int MODE, class T>
__global__ __launch_bounds__(256) void op_stencil_kernel(OpArgs<T> a) {
    constexpr int BX = 2 * PX + 1, BY = 2 * PY + 1;
    constexpr int TX = 64, LW = TX + 2 * PX, LH = STC_ROWS + 2 * PY;
    __shared__ cx<T> xs[LH][LW];
    __shared__ T kxS[BX][TX], mxS[BX][TX];
    __shared__ T kyS[STC_ROWS][BY], myS[STC_ROWS][BY];
    const int n1 = a.n1, n2 = a.n2;
    const long long N = (long long)n1 * n2;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int tiles_x = (n1 + TX - 1) / TX;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int C0 = (b % tiles_x) * TX, R0 = (b / tiles_x) * STC_ROWS;
    const int I1 = C0 + lane, I2 = R0 + w;
    const bool active = I1 < n1 && I2 < n2;
    const long long I = active ? (long long)I2 * n1 + I1 : 0;
    // coefficients first: every load of the thread in flight at once
    T c[BY * BX];
#pragma unroll
    for (int q = 0; q < BY * BX; ++q) c[q] = a.S[(size_t)q * N + I];
    // then x of the tile and its halo, the bands and the epilogue's operands, all
    // loaded into registers before the first LDS store, so that the workgroup
    // waits for memory once rather than once per staging step
    constexpr int XPT = (LH * LW + 255) / 256, DPW = (BX + 3) / 4;
    cx<T> xv[XPT];
#pragma unroll
    for (int r = 0; r < XPT; ++r) {
        const int e = threadIdx.x + 256 * r;
        const int rr = e / LW, cc = e % LW;
        const int J2 = R0 - PY + rr, J1 = C0 - PX + cc;
        xv[r] = (e < LH * LW && J2 >= 0 && J2 < n2 && J1 >= 0 && J1 < n1) ? a.x[(size_t)J2 * n1 + J1]
                                                                           : cx<T>{T(0), T(0)};
    }
    T kxv[DPW], mxv[DPW], kyv = 0, myv = 0;
    {
        const int I1c = I1 < n1 ? I1 : n1 - 1;
#pragma unroll
        for (int r = 0; r < DPW; ++r) {
            const int d = w + 4 * r;
            kxv[r] = d < BX ? (T)a.Kx[(size_t)I1c * BX + d] : T(0);
            mxv[r] = d < BX ? (T)a.Mx[(size_t)I1c * BX + d] : T(0);
        }
        if (lane < BY) {
            const int I2c = I2 < n2 ? I2 : n2 - 1;
            kyv = (T)a.Ky[(size_t)I2c * BY + lane];
            myv = (T)a.My[(size_t)I2c * BY + lane];
        }
    }
    cx<T> bv{T(0), T(0)}, dv{T(0), T(0)};
    if (MODE != MODE_APPLY && active) {
        bv = a.b[I];
        if (MODE == MODE_SMOOTH || a.xo) dv = a.dinv[I];
    }
#pragma unroll
    for (int r = 0; r < XPT; ++r) {
        const int e = threadIdx.x + 256 * r;
        if (e < LH * LW) xs[e / LW][e % LW] = xv[r];
    }
#pragma unroll
    for (int r = 0; r < DPW; ++r) {
        const int d = w + 4 * r;
        if (d < BX) {
            kxS[d][lane] = kxv[r];
            mxS[d][lane] = mxv[r];
        }
    }
    if (lane < BY) {
        kyS[w][lane] = kyv;
        myS[w][lane] = myv;
    }
    __syncthreads();
    if (!active) return;
    const T are = a.are, aim = a.aim;
    T wr = 0, wi = 0, vr = 0, vi = 0;
#pragma unroll
    for (int d2 = 0; d2 < BY; ++d2) {
        T u1r = 0, u1i = 0, u2r = 0, u2i = 0;
#pragma unroll
        for (int d = 0; d < BX; ++d) {
            const cx<T> v = xs[w + d2][lane + d];
            const T kx = kxS[d][lane], mx = mxS[d][lane];
            u1r += kx * v.re;
            u1i += kx * v.im;
            u2r += mx * v.re;
            u2i += mx * v.im;
            const T cc = c[d2 * BX + d];
            vr += cc * v.re;
            vi += cc * v.im;
        }
        wr += myS[w][d2] * u1r + kyS[w][d2] * u2r;
        wi += myS[w][d2] * u1i + kyS[w][d2] * u2i;
    }
    const T yr = wr - (are * vr - aim * vi);
    const T yi = wi - (are * vi + aim * vr);
    cx<T> out;
    if (MODE == MODE_APPLY) {
        out = {yr, yi};
    } else {
        const T rr = bv.re - yr, ri = bv.im - yi;
        if (MODE == MODE_RESID) {
            out = {rr, ri};
            if (a.xo) a.xo[I] = {a.omega * (dv.re * rr - dv.im * ri), a.omega * (dv.re * ri + dv.im * rr)};
        } else {
            const cx<T> x0 = xs[w + PY][lane + PX];
            out = {x0.re + a.omega * (dv.re * rr - dv.im * ri), x0.im + a.omega * (dv.re * ri + dv.im * rr)};
            if (a.yadd) {
                const cx<T> q = a.yadd[I];
                out = {out.re + q.re, out.im + q.im};
            }
        }
    }
    a.y[I] = out;
}

// Strip height: the tallest of 64, 32, 16, 8, 4 rows that still gives at
// least 2048 waves (eight per CU); tall strips amortise the 2p halo rows.
inline int op_rows_per_strip(int n1, int n2, int py) {
    if (py == 0) return 1;
    const long long cols = (n1 + 63) / 64;
    int ty = 64;
    while (ty > 4 && cols * ((n2 + ty - 1) / ty) < 2048) ty >>= 1;
    return ty;
}

template <int PX, int PY, int KIND, int MODE, class T>
static void launch_op_t(const OpArgs<T>& a, hipStream_t s) {
    // stored stencils: the tiled kernel from kStencilTiledMin unknowns on (a fixed
    // size rule, not a timed choice: the two kernels round differently)
    if (KIND == KIND_STENCIL && PY > 0 && (long long)a.n1 * a.n2 >= kStencilTiledMin) {
        const long long tiles = (long long)((a.n1 + 63) / 64) * ((a.n2 + STC_ROWS - 1) / STC_ROWS);
        hipLaunchKernelGGL((op_stencil_kernel<PX, PY, MODE, T>), dim3((unsigned)tiles), dim3(256), 0, s, a);
        return;
    }
    if (KIND != KIND_VARFINE && PY > 0 && (long long)a.n1 * a.n2 <= kOpDirectMax) {
        const long long N = (long long)a.n1 * a.n2;
        hipLaunchKernelGGL((op_direct_kernel<PX, PY, KIND, MODE, T>), dim3((unsigned)((N + 255) / 256)), dim3(256), 0,
                           s, a);
        return;
    }
    // a tuned strip height (a power of two in 4..64) or the fixed rule; 1D always 1
    const int ty = (PY == 0) ? 1 : (a.ty >= 4 && a.ty <= 64 && (a.ty & (a.ty - 1)) == 0) ? a.ty
                                                                                         : op_rows_per_strip(a.n1, a.n2, PY);
    dim3 grid((a.n1 + 63) / 64, (a.n2 + ty - 1) / ty);
    hipLaunchKernelGGL((op_kernel<PX, PY, KIND, MODE, T>), grid, dim3(64), 0, s, a, ty);
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
