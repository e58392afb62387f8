// Substructured exact solver of the deflation matrix E on a variable-k level
// (section 3: Q = Z E^-1 Z^T with E = Z^T A Z, here the Galerkin operator of
// the deflation level).  E couples control points at most p apart in each
// index direction, so bands of p grid lines cut the grid into subdomains whose
// interiors are uncoupled.  With I the interiors and S the separator bands,
//   E = [E_II E_IS; E_SI E_SS],  S = E_SS - E_SI E_II^-1 E_IS,
// and E e = c is solved exactly by
//   y_I = E_II^-1 c_I;  x_S = S^-1 (c_S - E_SI y_I);  x_I = E_II^-1 (c_I - E_IS x_S).
// E_II^-1 (one dense symmetric block per subdomain) and S^-1 are formed once at
// setup and applied as packed symmetric products; the two off-diagonal
// products come from the level operator applied to vectors that are zero off
// I (resp. S).  One application streams the stored triangles of the blocks
// twice and of S^-1 once: at 58k unknowns (p = 4) about 0.9 GB against 13.8 GB
// for the packed dense inverse of E.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <map>

#include "substruct.h"

namespace hh {

namespace {

constexpr int T128 = 128;
constexpr long long TSTRIDE = (long long)T128 * T128;

__device__ __host__ inline long long tile_index(long long I, long long J, long long nt) {
    return I * nt - I * (I - 1) / 2 + (J - I);
}

__device__ inline int find_by_tile(const SymMat* m, int nmat, long long t) {
    int lo = 0, hi = nmat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (m[mid].tile0 <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ inline int find_by_row(const SymMat* m, int nmat, int r) {
    int lo = 0, hi = nmat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (m[mid].row0 <= r) lo = mid; else hi = mid - 1;
    }
    return lo;
}

typedef double d2v __attribute__((ext_vector_type(2)));

// One workgroup per stored tile of the batch (1D grid over all tiles).  As the
// single-matrix product: wave w takes rows 32w..32w+31 of the tile, lane l the
// columns 2l, 2l+1; all 32 row loads of a wave are issued before use; row sums
// by a reduce-scatter over the wave, column sums (off-diagonal tiles) per lane
// and then over the four waves in order.  Vector entries go through the map.
__global__ __launch_bounds__(256) void symvb_tiles_kernel(const SymMat* __restrict__ mats, int nmat,
                                                          const double* __restrict__ P, const int* __restrict__ map,
                                                          const cx<double>* __restrict__ x,
                                                          cx<double>* __restrict__ rowpart,
                                                          cx<double>* __restrict__ colpart) {
    __shared__ cx<double> xs[T128];
    __shared__ cx<double> us[T128];
    __shared__ double vs[4][T128][2];
    const long long g = blockIdx.x;
    const SymMat M = mats[find_by_tile(mats, nmat, g)];
    const int n = M.n;
    const long long nt = (n + T128 - 1) / T128;
    const long long t = g - M.tile0;
    long long I = (long long)((2.0 * nt + 1.0 - sqrt((2.0 * nt + 1.0) * (2.0 * nt + 1.0) - 8.0 * (double)t)) / 2.0);
    I = I < 0 ? 0 : (I >= nt ? nt - 1 : I);
    while (I > 0 && tile_index(I, I, nt) > t) --I;
    while (I + 1 < nt && tile_index(I + 1, I + 1, nt) <= t) ++I;
    const long long J = I + (t - tile_index(I, I, nt));
    const double* T = P + g * TSTRIDE;
    const int* mp = map + M.map0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x < T128) {
        const long long r = I * T128 + threadIdx.x;
        xs[threadIdx.x] = r < n ? x[mp[r]] : cx<double>{0.0, 0.0};
    }
    const long long c0 = J * T128 + 2 * lane;
    const cx<double> xj0 = c0 < n ? x[mp[c0]] : cx<double>{0.0, 0.0};
    const cx<double> xj1 = c0 + 1 < n ? x[mp[c0 + 1]] : cx<double>{0.0, 0.0};
    __syncthreads();
    double vr0 = 0.0, vi0 = 0.0, vr1 = 0.0, vi1 = 0.0;
    const bool off = (I != J);
    double ur[32], ui[32];
    const double* Tw = T + (size_t)(32 * w) * T128 + 2 * lane;
    d2v av[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) av[q] = __builtin_nontemporal_load((const d2v*)(Tw + (size_t)q * T128));
    asm volatile("" ::: "memory");
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const d2v a = av[q];
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
    if (threadIdx.x < T128) {
        const int c = threadIdx.x;
        rowpart[g * T128 + c] = us[c];
        if (off)
            colpart[g * T128 + c] = {vs[0][c][0] + vs[1][c][0] + vs[2][c][0] + vs[3][c][0],
                                     vs[0][c][1] + vs[1][c][1] + vs[2][c][1] + vs[3][c][1]};
    }
}

// One workgroup per tile row of the batch: y for block row I of its matrix is
// the sum over J of (J < I: column sums of tile (J, I); J >= I: row sums of
// tile (I, J)); eight lane groups take J = grp, grp + 8, ... and are added in
// group order (a fixed order: deterministic).
constexpr int RG = 8;
__global__ __launch_bounds__(T128 * RG) void symvb_reduce_kernel(const SymMat* __restrict__ mats, int nmat,
                                                                 const int* __restrict__ map,
                                                                 const cx<double>* __restrict__ rowpart,
                                                                 const cx<double>* __restrict__ colpart,
                                                                 cx<double>* __restrict__ y, cx<double>* __restrict__ y2) {
    __shared__ double sr_s[RG][T128], si_s[RG][T128];
    const SymMat M = mats[find_by_row(mats, nmat, blockIdx.x)];
    const int n = M.n;
    const long long nt = (n + T128 - 1) / T128;
    const long long I = blockIdx.x - M.row0;
    const int r = threadIdx.x % T128, grp = threadIdx.x / T128;
    auto part = [&](long long J) -> cx<double> {
        return (J < I) ? colpart[(M.tile0 + tile_index(J, I, nt)) * T128 + r]
                       : rowpart[(M.tile0 + tile_index(I, J, nt)) * T128 + r];
    };
    double sr = 0.0, si = 0.0;
    long long J = grp;
    for (; J + 3 * RG < nt; J += 4 * RG) {
        const cx<double> v0 = part(J), v1 = part(J + RG), v2 = part(J + 2 * RG), v3 = part(J + 3 * RG);
        sr += v0.re;
        si += v0.im;
        sr += v1.re;
        si += v1.im;
        sr += v2.re;
        si += v2.im;
        sr += v3.re;
        si += v3.im;
    }
    for (; J < nt; J += RG) {
        const cx<double> v = part(J);
        sr += v.re;
        si += v.im;
    }
    sr_s[grp][r] = sr;
    si_s[grp][r] = si;
    __syncthreads();
    const long long gr = I * T128 + threadIdx.x;
    if (threadIdx.x < T128 && gr < n) {
        double tr = 0.0, ti = 0.0;
#pragma unroll
        for (int q = 0; q < RG; ++q) {
            tr += sr_s[q][threadIdx.x];
            ti += si_s[q][threadIdx.x];
        }
        const int idx = map[M.map0 + gr];
        y[idx] = {tr, ti};
        if (y2) y2[idx] = {tr, ti};
    }
}

// S[hs[j] * ld + hs[i]] -= C[j * hm + i] for i, j < h (one subdomain's share of
// the Schur complement; launched per subdomain in order: deterministic).
__global__ void schur_sub_kernel(int h, int hm, const double* __restrict__ C, const int* __restrict__ hs,
                                 double* __restrict__ S, long long ld) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i < h) S[(long long)hs[j] * ld + hs[i]] -= C[(long long)j * hm + i];
}

// Batched Gram blocks on the FP64 matrix cores: C_b = A_b^T B_b for every batch
// member b (A_b: K x M, B_b: K x N, C_b: M x N, all column-major, so the
// contraction index K is contiguous in both operands).  The Schur complement
// needs two such products per subdomain, W_d = (E_dd^-1)^T B_d and
// C_d = B_d^T W_d (E_dd^-1 symmetric: W_d = E_dd^-1 B_d to rounding).  A
// workgroup of four waves owns a 64 x 64 tile of C, each wave a 32 x 32 quarter
// as 2 x 2 fragments of v_mfma_f64_16x16x4f64 (operand lane l: row or column
// l mod 16 of the fragment, contraction index l / 16; result lane l: rows
// l / 16 + 4 r, column l mod 16).  K advances in slabs of 16: both operand
// tiles are staged in LDS (rows padded to 17 doubles), entries past M, N or K
// read as zero.
constexpr int GB_T = 64, GB_K = 16;
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void gram_tn_kernel(int M, int N, int K, const double* __restrict__ A, int lda,
                                                      long long sA, const double* __restrict__ B, int ldb,
                                                      long long sB, double* __restrict__ C, int ldc, long long sC) {
    __shared__ double As[GB_T][GB_K + 1];
    __shared__ double Bs[GB_T][GB_K + 1];
    A += (long long)blockIdx.z * sA;
    B += (long long)blockIdx.z * sB;
    C += (long long)blockIdx.z * sC;
    const int m0 = blockIdx.x * GB_T, n0 = blockIdx.y * GB_T;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    // staging: thread t loads 4 consecutive k of column t / 4 of each tile
    const int sc = t >> 2, sk = (t & 3) * 4;
    const bool am = m0 + sc < M, bn = n0 + sc < N;
    const double* Ap = A + (long long)(am ? m0 + sc : 0) * lda;
    const double* Bp = B + (long long)(bn ? n0 + sc : 0) * ldb;
    v4d acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += GB_K) {
        double av[4], bv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = k0 + sk + r;
            av[r] = (am && k < K) ? Ap[k] : 0.0;
            bv[r] = (bn && k < K) ? Bp[k] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            As[sc][sk + r] = av[r];
            Bs[sc][sk + r] = bv[r];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GB_K; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[wm + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[wn + j * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + j * 16 + (lane & 15);
            if (n >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
                if (m < M) C[(long long)n * ldc + m] = acc[i][j][r];
            }
        }
}

void launch_gram_tn(int M, int N, int K, const double* A, int lda, long long sA, const double* B, int ldb,
                    long long sB, double* C, int ldc, long long sC, int batch, hipStream_t s) {
    if (M <= 0 || N <= 0 || batch <= 0) return;
    HH_REQUIRE(batch <= 65535, "too many Gram blocks in one launch");
    const dim3 grid((M + GB_T - 1) / GB_T, (N + GB_T - 1) / GB_T, batch);
    hipLaunchKernelGGL(gram_tn_kernel, grid, dim3(256), 0, s, M, N, K, A, lda, sA, B, ldb, sB, C, ldc, sC);
    HH_HIP(hipGetLastError());
}

std::vector<int> split(int n, int B, int q) {
    const int tot = n - (B - 1) * q;
    if (B < 1 || tot < B) return {};
    std::vector<int> w((size_t)B, tot / B);
    for (int i = 0; i < tot % B; ++i) ++w[i];
    return w;
}

long long tiles_of(long long n) {
    const long long nt = (n + T128 - 1) / T128;
    return nt * (nt + 1) / 2;
}

// Bounds of the dense set-up work: the Schur complement and the padded blocks.
constexpr long long kMaxSep = 24576;
constexpr int kMaxBlock = 4096;

struct RocHandle {
    rocblas_handle h = nullptr;
    explicit RocHandle(hipStream_t s) {
        if (rocblas_create_handle(&h) != rocblas_status_success) throw Err{HH_EHIP, "rocblas_create_handle failed"};
        rocblas_set_stream(h, s);
    }
    ~RocHandle() {
        if (h) rocblas_destroy_handle(h);
    }
};

void roc_check(rocblas_status st, const char* what) {
    if (st != rocblas_status_success) throw Err{HH_EHIP, std::string(what) + " failed (rocblas status " +
                                                             std::to_string((int)st) + ")"};
}

}  // namespace

double symv_batch_tile_bytes(long long tiles) {
    return 8.0 * TSTRIDE * tiles + 2.0 * 16.0 * T128 * tiles + 2.0 * 16.0 * T128 * tiles;
}

void launch_symv_batch_tiles(const SymMat* mats_dev, int nmat, long long tiles, int rows, const double* P,
                             const int* map, const cx<double>* x, cx<double>* rowpart, cx<double>* colpart,
                             hipStream_t s) {
    meter(symv_batch_tile_bytes(tiles), 8.0 * TSTRIDE * tiles);
    hipLaunchKernelGGL(symvb_tiles_kernel, dim3((unsigned)tiles), dim3(256), 0, s, mats_dev, nmat, P, map, x, rowpart,
                       colpart);
}

void launch_symv_batch_reduce(const SymMat* mats_dev, int nmat, int rows, const int* map,
                              const cx<double>* rowpart, const cx<double>* colpart, cx<double>* y, cx<double>* y2,
                              hipStream_t s) {
    // the partial sums of every tile row read back, the outputs written
    meter(2.0 * 16.0 * T128 * (double)rows * 8 + 16.0 * T128 * rows, 0.0);
    hipLaunchKernelGGL(symvb_reduce_kernel, dim3((unsigned)rows), dim3(T128 * RG), 0, s, mats_dev, nmat, map,
                       rowpart, colpart, y, y2);
}

double SubstructE::bytes_per_apply() const {
    const double tiles = (double)(2 * sub_tiles + S_tiles) * (1 + refine);
    // stored tiles once; partial sums written and read (row and column); the
    // mapped vector reads and writes of the three products
    return 8.0 * TSTRIDE * tiles + 4.0 * 16.0 * T128 * tiles + 16.0 * (4.0 * nI + 3.0 * nS) * (1 + refine) +
           16.0 * 5.0 * (double)(nI + nS) * refine;
}

std::vector<std::pair<int, int>> substruct_partitions(int n1, int n2, int px, int py, int max_count) {
    std::vector<std::pair<long long, std::pair<int, int>>> all;
    const int mx = px > 0 ? std::min(64, n1 / (px + 1)) : 1;
    const int my = py > 0 ? std::min(64, n2 / (py + 1)) : 1;
    for (int bx = 1; bx <= std::max(1, mx); ++bx)
        for (int by = 1; by <= std::max(1, my); ++by) {
            if (bx * by < 2) continue;
            const auto wx = split(n1, bx, px), wy = split(n2, by, py);
            if (wx.empty() || wy.empty()) continue;
            long long ix = 0, iy = 0;
            for (int v : wx) ix += v;
            for (int v : wy) iy += v;
            const long long nS = (long long)n1 * n2 - ix * iy;
            if (nS > kMaxSep || nS < 1) continue;
            long long cost = tiles_of(nS);
            bool ok = true;
            for (int a : wx)
                for (int b : wy) {
                    if ((long long)a * b > kMaxBlock) ok = false;
                    cost += 2 * tiles_of((long long)a * b);
                }
            if (ok) all.push_back({cost, {bx, by}});
        }
    std::stable_sort(all.begin(), all.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    std::vector<std::pair<int, int>> out;
    for (const auto& c : all) {
        if ((int)out.size() >= max_count) break;
        out.push_back(c.second);
    }
    return out;
}

void substruct_build(SubstructE& E, int n1, int n2, int px, int py, int bx, int by, const RowVisitor& row,
                     hipStream_t s) {
    E.n1 = n1;
    E.n2 = n2;
    E.px = px;
    E.py = py;
    E.bx = bx;
    E.by = by;
    const auto wx = split(n1, bx, px), wy = split(n2, by, py);
    HH_REQUIRE(!wx.empty() && !wy.empty() && bx * by >= 2, "invalid substructuring partition");
    // per direction: block of each index (-1 on a separator band) and block starts
    std::vector<int> cx_((size_t)n1, -1), cy_((size_t)n2, -1), sx(bx), sy(by);
    for (int b = 0, at = 0; b < bx; ++b) {
        sx[b] = at;
        for (int i = 0; i < wx[b]; ++i) cx_[at + i] = b;
        at += wx[b] + px;
    }
    for (int b = 0, at = 0; b < by; ++b) {
        sy[b] = at;
        for (int i = 0; i < wy[b]; ++i) cy_[at + i] = b;
        at += wy[b] + py;
    }
    const long long N = (long long)n1 * n2;
    E.nsub = bx * by;
    // separators in grid order
    std::vector<int> sepidx((size_t)N, -1);
    std::vector<int> map;
    long long nS = 0;
    for (long long I = 0; I < N; ++I) {
        const int i1 = (int)(I % n1), i2 = (int)(I / n1);
        if (cx_[i1] < 0 || cy_[i2] < 0) sepidx[I] = (int)nS++;
    }
    E.nS = nS;
    HH_REQUIRE(nS <= kMaxSep, "separator count above the substructuring bound");
    // interiors, subdomain-major, row-major within each
    std::vector<int> nd(E.nsub), map0(E.nsub);
    int nd_max = 0;
    for (int jy = 0; jy < by; ++jy)
        for (int jx = 0; jx < bx; ++jx) {
            const int d = jy * bx + jx;
            map0[d] = (int)map.size();
            nd[d] = wx[jx] * wy[jy];
            nd_max = std::max(nd_max, nd[d]);
            for (int ly = 0; ly < wy[jy]; ++ly)
                for (int lx = 0; lx < wx[jx]; ++lx) map.push_back((sy[jy] + ly) * n1 + sx[jx] + lx);
        }
    E.nI = (long long)map.size();
    for (long long I = 0; I < N; ++I)
        if (sepidx[I] >= 0) map.push_back((int)I);
    E.nd_max = nd_max;
    // halos: separator unknowns within (px, py) of a subdomain, grid order
    std::vector<std::vector<int>> halo(E.nsub);
    int h_max = 0;
    for (int jy = 0; jy < by; ++jy)
        for (int jx = 0; jx < bx; ++jx) {
            const int d = jy * bx + jx;
            const int x0 = std::max(0, sx[jx] - px), x1 = std::min(n1, sx[jx] + wx[jx] + px);
            const int y0 = std::max(0, sy[jy] - py), y1 = std::min(n2, sy[jy] + wy[jy] + py);
            for (int i2 = y0; i2 < y1; ++i2)
                for (int i1 = x0; i1 < x1; ++i1) {
                    const long long I = (long long)i2 * n1 + i1;
                    if (sepidx[I] >= 0) halo[d].push_back((int)I);
                }
            h_max = std::max(h_max, (int)halo[d].size());
        }
    E.h_max = h_max;
    const int ndm = nd_max, hm = std::max(h_max, 1);
    // host blocks: E_dd (column-major, identity padding) and E_{d,halo} (zero padding)
    std::vector<double> A((size_t)E.nsub * ndm * ndm, 0.0), B((size_t)E.nsub * ndm * hm, 0.0);
    std::vector<long long> sidx;
    std::vector<double> sval;
    std::vector<int> hpos;   // subdomain-local: grid index -> halo position
    for (int jy = 0; jy < by; ++jy)
        for (int jx = 0; jx < bx; ++jx) {
            const int d = jy * bx + jx;
            double* Ad = A.data() + (size_t)d * ndm * ndm;
            double* Bd = B.data() + (size_t)d * ndm * hm;
            for (int i = nd[d]; i < ndm; ++i) Ad[(size_t)i * ndm + i] = 1.0;
            const int x0 = std::max(0, sx[jx] - px), y0 = std::max(0, sy[jy] - py);
            const int ex = std::min(n1, sx[jx] + wx[jx] + px) - x0;
            const int ey = std::min(n2, sy[jy] + wy[jy] + py) - y0;
            hpos.assign((size_t)ex * ey, -1);
            for (int q = 0; q < (int)halo[d].size(); ++q) {
                const int I = halo[d][q];
                hpos[(size_t)(I / n1 - y0) * ex + (I % n1 - x0)] = q;
            }
            for (int li = 0; li < nd[d]; ++li) {
                const long long I = map[map0[d] + li];
                row(I, [&](long long J, double v) {
                    const int j1 = (int)(J % n1), j2 = (int)(J / n1);
                    if (cx_[j1] == jx && cy_[j2] == jy) {
                        const int lj = (j2 - sy[jy]) * wx[jx] + (j1 - sx[jx]);
                        Ad[(size_t)lj * ndm + li] += v;
                    } else {
                        const int q = hpos[(size_t)(j2 - y0) * ex + (j1 - x0)];
                        if (q < 0) throw Err{HH_EINVAL, "deflation matrix couples beyond the separator width"};
                        Bd[(size_t)q * ndm + li] += v;
                    }
                });
            }
        }
    const long long ldS = (nS + 1) & ~1LL;
    {
        std::map<long long, double> rowacc;
        for (long long I = 0; I < N; ++I) {
            if (sepidx[I] < 0) continue;
            rowacc.clear();
            row(I, [&](long long J, double v) {
                if (sepidx[J] >= 0) rowacc[J] += v;
            });
            for (const auto& e : rowacc) {
                sidx.push_back((long long)sepidx[e.first] * ldS + sepidx[I]);
                sval.push_back(e.second);
            }
        }
    }
    // device: inverses of the blocks, their Schur contributions, S^-1
    RocHandle rh(s);
    DevBuf dA, ipiv, info;
    upload(dA, A);
    std::vector<double>().swap(A);
    ipiv.alloc((size_t)E.nsub * ndm * sizeof(rocblas_int));
    info.alloc((size_t)std::max<long long>(E.nsub, 1) * sizeof(rocblas_int));
    roc_check(rocsolver_dgetrf_strided_batched(rh.h, ndm, ndm, dA.as<double>(), ndm, (rocblas_stride)ndm * ndm,
                                               ipiv.as<rocblas_int>(), ndm, info.as<rocblas_int>(), E.nsub),
              "rocsolver_dgetrf_strided_batched");
    std::vector<rocblas_int> hinfo((size_t)E.nsub);
    HH_HIP(hipMemcpyAsync(hinfo.data(), info.p, hinfo.size() * sizeof(rocblas_int), hipMemcpyDeviceToHost, s));
    HH_HIP(hipStreamSynchronize(s));
    for (rocblas_int v : hinfo)
        if (v != 0) throw Err{HH_ENUMERIC, "a subdomain block of the deflation matrix E is singular"};
    roc_check(rocsolver_dgetri_strided_batched(rh.h, ndm, dA.as<double>(), ndm, (rocblas_stride)ndm * ndm,
                                               ipiv.as<rocblas_int>(), ndm, info.as<rocblas_int>(), E.nsub),
              "rocsolver_dgetri_strided_batched");
    DevBuf dS;
    dS.alloc((size_t)ldS * nS * sizeof(double));
    HH_HIP(hipMemsetAsync(dS.p, 0, (size_t)ldS * nS * sizeof(double), s));
    {
        DevBuf di, dv;
        upload(di, sidx);
        upload(dv, sval);
        launch_scatter((long long)sidx.size(), di.as<long long>(), dv.as<double>(), dS.as<double>(), s);
        HH_HIP(hipStreamSynchronize(s));
    }
    {
        DevBuf dB, dW, dC, dH;
        upload(dB, B);
        std::vector<double>().swap(B);
        dW.alloc((size_t)E.nsub * ndm * hm * sizeof(double));
        dC.alloc((size_t)E.nsub * hm * hm * sizeof(double));
        // W_d = (E_dd^-1)^T B_d, then the Gram blocks C_d = B_d^T W_d (FP64 MFMA)
        launch_gram_tn(ndm, hm, ndm, dA.as<double>(), ndm, (long long)ndm * ndm, dB.as<double>(), ndm,
                       (long long)ndm * hm, dW.as<double>(), ndm, (long long)ndm * hm, E.nsub, s);
        launch_gram_tn(hm, hm, ndm, dB.as<double>(), ndm, (long long)ndm * hm, dW.as<double>(), ndm,
                       (long long)ndm * hm, dC.as<double>(), hm, (long long)hm * hm, E.nsub, s);
        std::vector<int> hs;
        std::vector<int> h0(E.nsub);
        for (int d = 0; d < E.nsub; ++d) {
            h0[d] = (int)hs.size();
            for (int I : halo[d]) hs.push_back(sepidx[I]);
        }
        upload(dH, hs);
        for (int d = 0; d < E.nsub; ++d) {
            const int h = (int)halo[d].size();
            if (h == 0) continue;
            hipLaunchKernelGGL(schur_sub_kernel, dim3((h + 255) / 256, h), dim3(256), 0, s, h, hm,
                               dC.as<double>() + (size_t)d * hm * hm, dH.as<int>() + h0[d], dS.as<double>(), ldS);
        }
        HH_HIP(hipGetLastError());
        HH_HIP(hipStreamSynchronize(s));
    }
    {
        DevBuf sipiv, sinfo;
        sipiv.alloc((size_t)nS * sizeof(rocblas_int));
        sinfo.alloc(sizeof(rocblas_int));
        roc_check(rocsolver_dgetrf(rh.h, (rocblas_int)nS, (rocblas_int)nS, dS.as<double>(), (rocblas_int)ldS,
                                   sipiv.as<rocblas_int>(), sinfo.as<rocblas_int>()),
                  "rocsolver_dgetrf (Schur complement)");
        rocblas_int hi = 0;
        HH_HIP(hipMemcpyAsync(&hi, sinfo.p, sizeof(hi), hipMemcpyDeviceToHost, s));
        HH_HIP(hipStreamSynchronize(s));
        if (hi != 0) throw Err{HH_ENUMERIC, "deflation matrix E is singular (Schur complement)"};
        roc_check(rocsolver_dgetri(rh.h, (rocblas_int)nS, dS.as<double>(), (rocblas_int)ldS,
                                   sipiv.as<rocblas_int>(), sinfo.as<rocblas_int>()),
                  "rocsolver_dgetri (Schur complement)");
        HH_HIP(hipStreamSynchronize(s));
    }
    // packed triangles and the batch descriptors
    std::vector<SymMat> sm((size_t)E.nsub);
    long long t0 = 0;
    int r0 = 0;
    for (int d = 0; d < E.nsub; ++d) {
        sm[d] = {nd[d], (int)t0, r0, map0[d]};
        t0 += tiles_of(nd[d]);
        r0 += (nd[d] + T128 - 1) / T128;
    }
    E.sub_tiles = t0;
    E.sub_rows = r0;
    E.subP.alloc((size_t)t0 * TSTRIDE * sizeof(double));
    for (int d = 0; d < E.nsub; ++d)
        launch_sym_pack(nd[d], ndm, dA.as<double>() + (size_t)d * ndm * ndm,
                        E.subP.as<double>() + (size_t)sm[d].tile0 * TSTRIDE, s);
    E.S_tiles = tiles_of(nS);
    E.S_rows = (int)((nS + T128 - 1) / T128);
    E.SP.alloc((size_t)E.S_tiles * TSTRIDE * sizeof(double));
    launch_sym_pack((int)nS, ldS, dS.as<double>(), E.SP.as<double>(), s);
    HH_HIP(hipGetLastError());
    upload(E.subMats, sm);
    std::vector<SymMat> ss{{(int)nS, 0, 0, (int)E.nI}};
    upload(E.SMats, ss);
    upload(E.map, map);
    const size_t pbytes = (size_t)std::max(E.sub_tiles, E.S_tiles) * T128 * sizeof(cx<double>);
    E.rowpart.alloc(pbytes);
    E.colpart.alloc(pbytes);
    for (DevBuf* b : {&E.xhat, &E.xt, &E.rvec, &E.rr, &E.dd}) {
        b->alloc((size_t)N * sizeof(cx<double>));
        HH_HIP(hipMemsetAsync(b->p, 0, (size_t)N * sizeof(cx<double>), s));
    }
    HH_HIP(hipStreamSynchronize(s));
}

}  // namespace hh
