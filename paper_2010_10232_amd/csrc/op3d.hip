// Unit-cube kernels for gfx950 (CDNA4, wave64): the level operator, the
// knot-insertion transfers and the fast-diagonalisation E^-1 of 3D
// tensor-product B-spline levels with constant k (section 2.3 carried to three
// directions; section 3's multigrid CSLP and two-level deflation on top).
//
// Level operator.  With the 1D bands K_d, M_d of each direction,
//   y = K x - alpha k^2 M x
//     = Mz (x) [My (x) Kx + Ky (x) Mx - alpha k^2 My (x) Mx] x + Kz (x) [My (x) Mx] x,
// so every z-slice J3 of x enters through two 2D products, B2 (the bracket) and
// M2 (the 2D mass), combined through the z bands:
//   y_{i3} = sum_{J3} mz[i3][J3 - i3] B2(x_{J3}) + kz[i3][J3 - i3] M2(x_{J3}).
// A workgroup of 256 threads owns a 32 (x) by 8 (y) column tile and a run of
// tz output slices.  It walks the tz + 2p input slices once, as a three-stage
// pipeline over double-buffered LDS with one barrier per step: slice t (tile
// plus its p-wide halo) is staged from registers (slice t + 1 is already in
// flight), slice t - 1 gets its x bands once per staged row (sum
// factorisation: Kx x - alpha k^2 Mx x and Mx x per row), and for slice t - 2 every thread forms
// B2 and M2 of its column through the y bands and adds them into a window of
// 2p + 1 running output slices held in registers (mz, kz as weights).  After
// input slice J3, output slice J3 - p is complete and is written with the
// residual / Jacobi epilogue of the 2D kernels.  Per unknown and slice this is
// 2(2p+1) + 3(2p+1) + 2(2p+1) complex-by-real multiply-adds instead of the
// (2p+1)^3 of a point-wise stencil.
#include <algorithm>
#include <climits>

#include "hh_internal.h"

namespace hh {

namespace {

constexpr int O3_TX = 32, O3_TY = 8, O3_TB = O3_TX * O3_TY;
constexpr int O3_TZMAX = 32;   // output slices per workgroup, at most

template <int P, int MODE, class T>
__global__ __launch_bounds__(O3_TB) void op3d_kernel(OpArgs<T> a, int tz) {
    constexpr int B = 2 * P + 1;
    constexpr int LW = O3_TX + 2 * P, LH = O3_TY + 2 * P;
    constexpr int NL = (LH * LW + O3_TB - 1) / O3_TB;   // staged values per thread
    // double buffers: slice t is staged while slice t - 1 gets its x bands and
    // slice t - 2 its y and z bands, one barrier per step
    __shared__ cx<T> xs[2][LH][LW];
    __shared__ cx<T> us[2][2][LH][O3_TX];                // [buffer][Kx x - alpha k^2 Mx x, Mx x][row][column]
    __shared__ T mzS[O3_TZMAX][B], kzS[O3_TZMAX][B];     // z bands of the workgroup's output slices

    const int n1 = a.n1, n2 = a.n2, n3 = a.n3;
    const int tiles_x = (n1 + O3_TX - 1) / O3_TX, tiles_y = (n2 + O3_TY - 1) / O3_TY;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int bx = b % tiles_x, rest = b / tiles_x;
    const int C0 = bx * O3_TX, R0 = (rest % tiles_y) * O3_TY, Z0 = (rest / tiles_y) * tz;
    const int tid = threadIdx.x;
    const int c = tid % O3_TX, r = tid / O3_TX;
    const int I1 = C0 + c, I2 = R0 + r;
    const int I1c = I1 < n1 ? I1 : n1 - 1, I2c = I2 < n2 ? I2 : n2 - 1;
    T kx[B], mx[B], ky[B], my[B];
#pragma unroll
    for (int d = 0; d < B; ++d) {
        kx[d] = (T)a.Kx[(size_t)I1c * B + d];
        mx[d] = (T)a.Mx[(size_t)I1c * B + d];
        ky[d] = (T)a.Ky[(size_t)I2c * B + d];
        my[d] = (T)a.My[(size_t)I2c * B + d];
    }
    // the next slice in flight: every value is loaded from a valid address (its own
    // or element 0) and masked when it is staged, so no wait sits between the
    // loads and the work of the current step
    cx<T> pre[NL];
    bool pok[NL];
    auto fetch = [&](int J3) {
        const bool zok = J3 >= 0 && J3 < n3;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int e = tid + O3_TB * q;
            const int rr = e / LW, cc = e - rr * LW;
            const int J2 = R0 - P + rr, J1 = C0 - P + cc;
            const bool ok = zok && e < LH * LW && J2 >= 0 && J2 < n2 && J1 >= 0 && J1 < n1;
            pre[q] = a.x[ok ? ((size_t)J3 * n2 + J2) * n1 + J1 : 0];
            pok[q] = ok;
        }
    };
    const int zend = Z0 + tz < n3 ? Z0 + tz : n3;
    const int s0 = Z0 - P, s1 = zend - 1 + P;
    // (visible after the first barrier of the slice loop)
    for (int e = tid; e < (zend - Z0) * B; e += O3_TB) {
        const int q = e / B, d = e - q * B;
        mzS[q][d] = (T)a.Mz[(size_t)(Z0 + q) * B + d];
        kzS[q][d] = (T)a.Kz[(size_t)(Z0 + q) * B + d];
    }
    T wr[B], wi[B];
#pragma unroll
    for (int k = 0; k < B; ++k) wr[k] = wi[k] = T(0);
    const T are = a.are, aim = a.aim;
    const T k2c = (T)a.k2c;
    const bool active = I1 < n1 && I2 < n2;

    fetch(s0);
#pragma unroll 1
    for (int t = s0; t <= s1 + 2; ++t) {
        if (t <= s1) {
            // stage slice t (tile + halo), then put slice t + 1 in flight
            const int bf = t & 1;
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                const int e = tid + O3_TB * q;
                if (e < LH * LW) xs[bf][e / LW][e % LW] = pok[q] ? pre[q] : cx<T>{T(0), T(0)};
            }
            if (t < s1) fetch(t + 1);
        }
        if (t - 1 >= s0 && t - 1 <= s1) {
            // x bands of slice t - 1, once per staged row (every item of this thread has
            // column c): Kx x - alpha k^2 Mx x and Mx x
            const int bf = (t - 1) & 1;
            for (int e = tid; e < LH * O3_TX; e += O3_TB) {
                const int rr = e / O3_TX;
                T u1r = 0, u1i = 0, u2r = 0, u2i = 0;
#pragma unroll
                for (int d = 0; d < B; ++d) {
                    const cx<T> v = xs[bf][rr][c + d];
                    u1r += kx[d] * v.re;
                    u1i += kx[d] * v.im;
                    u2r += mx[d] * v.re;
                    u2i += mx[d] * v.im;
                }
                const T cr = u1r - k2c * (are * u2r - aim * u2i);
                const T ci = u1i - k2c * (are * u2i + aim * u2r);
                us[bf][0][rr][c] = {cr, ci};
                us[bf][1][rr][c] = {u2r, u2i};
            }
        }
        const int J3 = t - 2;
        if (J3 >= s0) {
            if (J3 >= 0 && J3 < n3) {
                // B2 and M2 of this column through the y bands
                const int bf = J3 & 1;
                T br = 0, bi = 0, mr = 0, mi = 0;
#pragma unroll
                for (int d2 = 0; d2 < B; ++d2) {
                    const cx<T> u1 = us[bf][0][r + d2][c], u2 = us[bf][1][r + d2][c];
                    br += my[d2] * u1.re + ky[d2] * u2.re;
                    bi += my[d2] * u1.im + ky[d2] * u2.im;
                    mr += my[d2] * u2.re;
                    mi += my[d2] * u2.im;
                }
                // window entry k is output slice J3 - p + k, coupled at offset J3 - i3 = p - k
                // (slices outside this workgroup's outputs are never written: no weight)
#pragma unroll
                for (int k = 0; k < B; ++k) {
                    const int q = J3 - P + k - Z0;
                    if (q >= 0 && q < zend - Z0) {
                        const T mz = mzS[q][2 * P - k], kz = kzS[q][2 * P - k];
                        wr[k] += mz * br + kz * mr;
                        wi[k] += mz * bi + kz * mi;
                    }
                }
            }
            // output slice J3 - p has all its input slices
            const int i3 = J3 - P;
            if (active && i3 >= Z0 && i3 < zend) {
                const size_t I = ((size_t)i3 * n2 + I2) * n1 + I1;
                const T yr = wr[0], yi = wi[0];
                cx<T> out;
                if (MODE == MODE_APPLY) {
                    out = {yr, yi};
                } else {
                    const cx<T> bv = a.b[I];
                    const T rr = bv.re - yr, ri = bv.im - yi;
                    if (MODE == MODE_RESID) {
                        out = {rr, ri};
                        if (a.xo) {
                            const cx<T> d = a.dinv[I];
                            a.xo[I] = {a.omega * (d.re * rr - d.im * ri), a.omega * (d.re * ri + d.im * rr)};
                        }
                    } else {
                        const cx<T> dv = a.dinv[I], xv = a.x[I];
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
#pragma unroll
            for (int k = 0; k + 1 < B; ++k) {
                wr[k] = wr[k + 1];
                wi[k] = wi[k + 1];
            }
            wr[B - 1] = wi[B - 1] = T(0);
        }
        __syncthreads();
    }
}

// Output slices per workgroup: a tuned value (a power of two in 2..32), else
// the longest of 16, 8, 4, 2 that still gives 1024 workgroups (four per CU).
inline int op3d_slices(int n1, int n2, int n3, int tuned) {
    if (tuned >= 2 && tuned <= O3_TZMAX && (tuned & (tuned - 1)) == 0) return tuned;
    const long long tiles = (long long)((n1 + O3_TX - 1) / O3_TX) * ((n2 + O3_TY - 1) / O3_TY);
    int tz = 16;
    while (tz > 2 && tiles * ((n3 + tz - 1) / tz) < 1024) tz >>= 1;
    return tz;
}

template <int P, class T>
void launch_op3d_p(int mode, const OpArgs<T>& a, hipStream_t s) {
    const int tz = op3d_slices(a.n1, a.n2, a.n3, a.ty);
    const long long blocks = (long long)((a.n1 + O3_TX - 1) / O3_TX) * ((a.n2 + O3_TY - 1) / O3_TY) *
                             ((a.n3 + tz - 1) / tz);
    if (blocks > INT_MAX) throw Err{HH_EINVAL, "level too large for the 3D operator"};
    switch (mode) {
        case MODE_APPLY:
            hipLaunchKernelGGL((op3d_kernel<P, MODE_APPLY, T>), dim3((unsigned)blocks), dim3(O3_TB), 0, s, a, tz);
            return;
        case MODE_RESID:
            hipLaunchKernelGGL((op3d_kernel<P, MODE_RESID, T>), dim3((unsigned)blocks), dim3(O3_TB), 0, s, a, tz);
            return;
        case MODE_SMOOTH:
            hipLaunchKernelGGL((op3d_kernel<P, MODE_SMOOTH, T>), dim3((unsigned)blocks), dim3(O3_TB), 0, s, a, tz);
            return;
    }
    throw Err{HH_EINVAL, "bad operator mode"};
}

// ------------------------------------------------------------- transfers --
// c = P^T r and x (+)= P e with P = P_z (x) P_y (x) P_x, each 1D factor stored
// as per-row / per-column runs (as in the 2D transfers), applied one direction
// at a time (sum factorisation: (p+2) + (p+2) + (p+2) terms per coarse unknown
// instead of (p+2)^3, through two intermediate grids).  One pass:
//   out[.., o, ..] = sum_{k < w} wt[o][k] in[.., i0[o] + k, ..]
// along direction `axis` of an m1 x m2 x m3 input (x fastest), n_out entries
// along that direction in the output.  The last pass of a restriction also
// forms the coarse level's first damped Jacobi sweep (xs = omega D^-1 c); the
// last pass of a prolongation adds xin.
template <class T>
__global__ void axis_pass_kernel(int m1, int m2, int m3, int axis, int n_out, const int* __restrict__ i0,
                                 const double* __restrict__ wt, int w, const cx<T>* __restrict__ in,
                                 cx<T>* __restrict__ out, const cx<T>* __restrict__ dinv, T omega,
                                 cx<T>* __restrict__ xs, const cx<T>* xin) {
    const int o1 = axis == 0 ? n_out : m1, o2 = axis == 1 ? n_out : m2, o3 = axis == 2 ? n_out : m3;
    const long long No = (long long)o1 * o2 * o3;
    const long long idx = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= No) return;
    const int j1 = (int)(idx % o1), j2 = (int)((idx / o1) % o2), j3 = (int)(idx / ((long long)o1 * o2));
    const int o = axis == 0 ? j1 : axis == 1 ? j2 : j3;
    const long long stride = axis == 0 ? 1 : axis == 1 ? m1 : (long long)m1 * m2;
    // the input entry with coordinate i0[o] along the axis and j elsewhere
    const long long base = (axis == 0 ? 0 : (long long)j1) + (axis == 1 ? 0 : (long long)j2 * m1) +
                           (axis == 2 ? 0 : (long long)j3 * m1 * m2) + (long long)i0[o] * stride;
    const cx<T>* src = in + base;
    const double* wr = wt + (size_t)o * w;
    T sr = 0, si = 0;
    for (int k = 0; k < w; ++k) {
        const T g = (T)wr[k];
        const cx<T> v = src[(size_t)k * stride];
        sr += g * v.re;
        si += g * v.im;
    }
    if (xin) {
        const cx<T> q = xin[idx];
        sr = q.re + sr;
        si = q.im + si;
    }
    out[idx] = {sr, si};
    if (dinv) {
        const cx<T> d = dinv[idx];
        xs[idx] = {omega * (d.re * sr - d.im * si), omega * (d.re * si + d.im * sr)};
    }
}

// --------------------------------------------------- fast diagonalisation --
// out = (A along one axis) in: out[.., i, ..] = sum_j A[i][j] in[.., j, ..]
// (A row-major n_a x n_a), times scale[idx] when scale is given.
__global__ void fdm3_pass_kernel(int n1, int n2, int n3, int axis, const double* __restrict__ A,
                                 const cx<double>* __restrict__ in, cx<double>* __restrict__ out,
                                 const double* __restrict__ scale) {
    const long long N = (long long)n1 * n2 * n3;
    const long long idx = (long long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const int i1 = (int)(idx % n1), i2 = (int)((idx / n1) % n2), i3 = (int)(idx / ((long long)n1 * n2));
    const int na = axis == 0 ? n1 : axis == 1 ? n2 : n3;
    const int i = axis == 0 ? i1 : axis == 1 ? i2 : i3;
    const long long stride = axis == 0 ? 1 : axis == 1 ? n1 : (long long)n1 * n2;
    const cx<double>* src = in + (idx - (long long)i * stride);
    const double* row = A + (size_t)i * na;
    double sr = 0, si = 0;
    for (int j = 0; j < na; ++j) {
        const double w = row[j];
        const cx<double> v = src[(size_t)j * stride];
        sr += w * v.re;
        si += w * v.im;
    }
    if (scale) {
        const double g = scale[idx];
        sr *= g;
        si *= g;
    }
    out[idx] = {sr, si};
}

// The same product for lines of at most FL_MAXN entries, staged in LDS: a
// workgroup takes FL_TL lines (along x: FL_TL consecutive rows; along y or z:
// FL_TL consecutive x positions at one z or y), loads them and the matrix
// once with coalesced reads, and forms every output of those lines from LDS
// (the sum over j in the same order as fdm3_pass_kernel).
constexpr int FL_TL = 16, FL_MAXN = 72;
__global__ __launch_bounds__(256) void fdm3_lines_kernel(int n1, int n2, int n3, int axis, const double* __restrict__ A,
                                                         const cx<double>* __restrict__ in,
                                                         cx<double>* __restrict__ out,
                                                         const double* __restrict__ scale) {
    __shared__ double As[FL_MAXN * FL_MAXN];
    __shared__ cx<double> ls[FL_MAXN][FL_TL];
    const int na = axis == 0 ? n1 : axis == 1 ? n2 : n3;
    const long long stride = axis == 0 ? 1 : axis == 1 ? n1 : (long long)n1 * n2;
    const int tid = threadIdx.x, b = blockIdx.x;
    long long base;   // line t starts at base + t * lstep (valid while t < nlines)
    int nlines, lstep;
    if (axis == 0) {
        const long long L0 = (long long)b * FL_TL, total = (long long)n2 * n3;
        base = L0 * n1;
        lstep = n1;
        nlines = (int)(total - L0 < FL_TL ? total - L0 : FL_TL);
    } else {
        const int xt = (n1 + FL_TL - 1) / FL_TL;
        const int x0 = (b % xt) * FL_TL, o = b / xt;   // o: z (axis 1) or y (axis 2)
        base = (axis == 1 ? (long long)o * n1 * n2 : (long long)o * n1) + x0;
        lstep = 1;
        nlines = n1 - x0 < FL_TL ? n1 - x0 : FL_TL;
    }
    for (int e = tid; e < na * na; e += 256) As[e] = A[e];
    for (int e = tid; e < na * FL_TL; e += 256) {
        // along x the entries of a row are adjacent, along y / z the lines
        const int t = axis == 0 ? e / na : e % FL_TL, j = axis == 0 ? e % na : e / FL_TL;
        ls[j][t] = t < nlines ? in[base + (long long)t * lstep + (long long)j * stride] : cx<double>{0.0, 0.0};
    }
    __syncthreads();
    for (int e = tid; e < na * FL_TL; e += 256) {
        const int t = axis == 0 ? e / na : e % FL_TL, i = axis == 0 ? e % na : e / FL_TL;
        if (t >= nlines) continue;
        const double* row = As + i * na;
        double sr = 0, si = 0;
        for (int j = 0; j < na; ++j) {
            const double w = row[j];
            const cx<double> v = ls[j][t];
            sr += w * v.re;
            si += w * v.im;
        }
        const long long idx = base + (long long)t * lstep + (long long)i * stride;
        if (scale) {
            const double g = scale[idx];
            sr *= g;
            si *= g;
        }
        out[idx] = {sr, si};
    }
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

template <class T>
void launch_op3d(int mode, int p, const OpArgs<T>& a, hipStream_t s) {
    if (a.n1 <= 0 || a.n2 <= 0 || a.n3 <= 0) return;
    switch (p) {
        case 1: return launch_op3d_p<1, T>(mode, a, s);
        case 2: return launch_op3d_p<2, T>(mode, a, s);
        case 3: return launch_op3d_p<3, T>(mode, a, s);
        case 4: return launch_op3d_p<4, T>(mode, a, s);
        case 5: return launch_op3d_p<5, T>(mode, a, s);
    }
    throw Err{HH_EINVAL, "unsupported degree"};
}
template void launch_op3d<double>(int, int, const OpArgs<double>&, hipStream_t);
template void launch_op3d<float>(int, int, const OpArgs<float>&, hipStream_t);

template <class T>
static cx<T>* tmp_a(const Transfer& t) {
    if constexpr (sizeof(T) == 8) return t.tmpa64; else return t.tmpa32;
}
template <class T>
static cx<T>* tmp_b(const Transfer& t) {
    if constexpr (sizeof(T) == 8) return t.tmpb64; else return t.tmpb32;
}
template <class T>
static void axis_pass(int m1, int m2, int m3, int axis, int n_out, const int* i0, const double* wt, int w,
                      const cx<T>* in, cx<T>* out, hipStream_t s, const cx<T>* dinv = nullptr, T omega = T(0),
                      cx<T>* xs = nullptr, const cx<T>* xin = nullptr) {
    const long long No = (long long)(axis == 0 ? n_out : m1) * (axis == 1 ? n_out : m2) * (axis == 2 ? n_out : m3);
    hipLaunchKernelGGL(axis_pass_kernel<T>, dim3(blocks_for(No, 256)), dim3(256), 0, s, m1, m2, m3, axis, n_out, i0,
                       wt, w, in, out, dinv, omega, xs, xin);
}

template <class T>
void launch_restrict3(const Transfer& t, const cx<T>* r, cx<T>* c, hipStream_t s, const cx<T>* dinv, T omega,
                      cx<T>* xs) {
    const long long Nc = (long long)t.nc1 * t.nc2 * t.nc3, Nf = (long long)t.nf1 * t.nf2 * t.nf3;
    if (Nc <= 0) return;
    if (Nc > INT_MAX || Nf > INT_MAX) throw Err{HH_EINVAL, "level too large for a transfer"};
    if (!tmp_a<T>(t) || !tmp_b<T>(t)) throw Err{HH_EINVAL, "3D transfer without its intermediate grids"};
    meter(sizeof(cx<T>) * ((double)Nf + Nc * (dinv ? 3.0 : 1.0)),
          4.0 * t.rw1 * t.rw2 * t.rw3 * (double)Nc + (dinv ? 8.0 * Nc : 0.0));
    // x: [nf3][nf2][nf1] -> [nf3][nf2][nc1]; y: -> [nf3][nc2][nc1]; z: -> [nc3][nc2][nc1]
    axis_pass<T>(t.nf1, t.nf2, t.nf3, 0, t.nc1, t.pcol0x, t.pcolx, t.rw1, r, tmp_a<T>(t), s);
    axis_pass<T>(t.nc1, t.nf2, t.nf3, 1, t.nc2, t.pcol0y, t.pcoly, t.rw2, tmp_a<T>(t), tmp_b<T>(t), s);
    axis_pass<T>(t.nc1, t.nc2, t.nf3, 2, t.nc3, t.pcol0z, t.pcolz, t.rw3, tmp_b<T>(t), c, s, dinv, omega, xs);
}
template <class T>
void launch_prolong_add3(const Transfer& t, const cx<T>* e, const cx<T>* xin, cx<T>* xout, hipStream_t s) {
    const long long Nc = (long long)t.nc1 * t.nc2 * t.nc3, Nf = (long long)t.nf1 * t.nf2 * t.nf3;
    if (Nf <= 0) return;
    if (Nc > INT_MAX || Nf > INT_MAX) throw Err{HH_EINVAL, "level too large for a transfer"};
    if (!tmp_a<T>(t) || !tmp_b<T>(t)) throw Err{HH_EINVAL, "3D transfer without its intermediate grids"};
    meter(sizeof(cx<T>) * ((double)Nc + Nf * (xin ? 2.0 : 1.0)),
          4.0 * t.pw1 * t.pw2 * t.pw3 * (double)Nf + (xin ? 2.0 * Nf : 0.0));
    // z: [nc3][nc2][nc1] -> [nf3][nc2][nc1]; y: -> [nf3][nf2][nc1]; x: -> [nf3][nf2][nf1] (+ xin)
    axis_pass<T>(t.nc1, t.nc2, t.nc3, 2, t.nf3, t.prow0z, t.prowz, t.pw3, e, tmp_b<T>(t), s);
    axis_pass<T>(t.nc1, t.nc2, t.nf3, 1, t.nf2, t.prow0y, t.prowy, t.pw2, tmp_b<T>(t), tmp_a<T>(t), s);
    axis_pass<T>(t.nc1, t.nf2, t.nf3, 0, t.nf1, t.prow0x, t.prowx, t.pw1, tmp_a<T>(t), xout, s, nullptr, T(0),
                 nullptr, xin);
}
template void launch_restrict3<double>(const Transfer&, const cx<double>*, cx<double>*, hipStream_t,
                                       const cx<double>*, double, cx<double>*);
template void launch_restrict3<float>(const Transfer&, const cx<float>*, cx<float>*, hipStream_t, const cx<float>*,
                                      float, cx<float>*);
template void launch_prolong_add3<double>(const Transfer&, const cx<double>*, const cx<double>*, cx<double>*,
                                          hipStream_t);
template void launch_prolong_add3<float>(const Transfer&, const cx<float>*, const cx<float>*, cx<float>*,
                                         hipStream_t);

void launch_fdm3_solve(int n3, int n2, int n1, const double* Vx, const double* VxT, const double* Vy,
                       const double* VyT, const double* Vz, const double* VzT, const double* dinv,
                       const cx<double>* c, cx<double>* t1, cx<double>* t2, cx<double>* e, hipStream_t s) {
    const long long N = (long long)n1 * n2 * n3;
    if (N <= 0) return;
    if (N > INT_MAX) throw Err{HH_EINVAL, "deflation level too large"};
    meter(6.0 * 32.0 * N + 8.0 * N, 4.0 * N * ((double)n1 + n2 + n3) * 2.0);
    const bool lines = std::max({n1, n2, n3}) <= FL_MAXN;
    const unsigned g = blocks_for(N, 256);
    auto pass = [&](int axis, const double* M, const cx<double>* in, cx<double>* out, const double* sc) {
        if (lines) {
            const long long nb = axis == 0 ? ((long long)n2 * n3 + FL_TL - 1) / FL_TL
                                           : (long long)((n1 + FL_TL - 1) / FL_TL) * (axis == 1 ? n3 : n2);
            hipLaunchKernelGGL(fdm3_lines_kernel, dim3((unsigned)nb), dim3(256), 0, s, n1, n2, n3, axis, M, in, out,
                               sc);
        } else {
            hipLaunchKernelGGL(fdm3_pass_kernel, dim3(g), dim3(256), 0, s, n1, n2, n3, axis, M, in, out, sc);
        }
    };
    // V^T c along x, y, z (the last scaled by 1 / D), then V along z, y, x
    pass(0, VxT, c, t1, nullptr);
    pass(1, VyT, t1, t2, nullptr);
    pass(2, VzT, t2, t1, dinv);
    pass(2, Vz, t1, t2, nullptr);
    pass(1, Vy, t2, t1, nullptr);
    pass(0, Vx, t1, e, nullptr);
}

}  // namespace hh
