// Learned fine-level smoother: a complex 3x3 CNN (channels 2 -> 16 -> 16 -> 16
// -> 1, CReLU) evaluated and trained on the GPU with BF16 MFMA (FP32
// accumulation).  Not part of the paper's method, which keeps damped Jacobi;
// Jacobi remains the fallback.
//
// Representation.  A complex channel is a pair of real channels (re, im); a
// complex weight a + ib acting on a complex input becomes the real 2x2 block
// [[a, -b], [b, a]], and CReLU becomes a ReLU on every real channel.
// Activations are channel-last BF16 [H][W][C] on the interior control-point
// grid (C = 8 for the input layer: r.re, r.im, c, 0..., 32 for hidden layers).
//
// Convolution = implicit GEMM on v_mfma_f32_16x16x32_bf16: M = pixels (16 per
// wave), N = output channels (16 per MFMA tile), K = (tap, input channel): one
// tap of 32 channels per MFMA for hidden layers, four taps of 8 channels for the
// 8-channel input layer.  Per layer (training): a workgroup (4 waves) owns a
// 64-pixel row segment; its three input rows are staged in LDS, the packed
// weights sit in registers.  The smoother step runs all layers in one kernel
// (cnn_fused_kernel).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "cnn.h"

namespace hh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// --------------------------------------------------------------------------
// Forward / data-gradient convolution
// --------------------------------------------------------------------------
enum ConvMode { CONV_RELU = 0, CONV_OUT = 1, CONV_MASK = 2 };

template <int CINP, int COUTP, int MODE>
__global__ __launch_bounds__(256) void conv3x3_kernel(int H, int Wd, const __bf16* __restrict__ X,
                                                      const __bf16* __restrict__ Wp, const float* __restrict__ bias,
                                                      const __bf16* __restrict__ Mk, void* __restrict__ Y) {
    constexpr int SEG = 64;
    constexpr int NT = COUTP / 16;
    constexpr int KSTEPS = (CINP == 32) ? 9 : 3;
    constexpr int CH = CINP / 8;
    __shared__ __attribute__((aligned(16))) __bf16 xs[3][SEG + 2][CINP];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int x0 = blockIdx.x * SEG, h = blockIdx.y;
    for (int idx = tid; idx < 3 * (SEG + 2) * CH; idx += 256) {
        const int r = idx / ((SEG + 2) * CH);
        const int rem = idx - r * (SEG + 2) * CH;
        const int px = rem / CH, ch = rem - px * CH;
        const int hh = h + r - 1, ww = x0 + px - 1;
        uint4 v = {0u, 0u, 0u, 0u};
        if (hh >= 0 && hh < H && ww >= 0 && ww < Wd) v = *(const uint4*)(X + ((size_t)hh * Wd + ww) * CINP + ch * 8);
        *(uint4*)&xs[r][px][ch * 8] = v;
    }
    const int g = lane >> 4, col = lane & 15;
    bf16x8 bw[KSTEPS][NT];
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
        const int tap = (CINP == 32) ? s : 4 * s + g;
        const int ci0 = (CINP == 32) ? 8 * g : 0;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if (tap < 9) {
                bw[s][nt] = *(const bf16x8*)(Wp + ((size_t)tap * COUTP + nt * 16 + col) * CINP + ci0);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) bw[s][nt][e] = (__bf16)0.0f;
            }
        }
    }
    __syncthreads();
    f32x4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int pxa = wave * 16 + col;   // A-operand row: this lane's pixel
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
        const int tap = (CINP == 32) ? s : 4 * s + g;
        const int ci0 = (CINP == 32) ? 8 * g : 0;
        bf16x8 a;
        if (tap < 9) {
            const int dy = tap / 3, dx = tap - 3 * dy;
            a = *(const bf16x8*)&xs[dy][pxa + dx][ci0];
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) a[e] = (__bf16)0.0f;
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[s][nt], acc[nt], 0, 0, 0);
    }
    // D: this lane holds output channel nt*16 + col for pixels 4g .. 4g+3 of the wave
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int co = nt * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int pxo = x0 + wave * 16 + 4 * g + i;
            if (pxo >= Wd) continue;
            const size_t p = (size_t)h * Wd + pxo;
            float v = acc[nt][i];
            if (MODE == CONV_RELU) {
                v = fmaxf(v + bias[co], 0.0f);
                ((__bf16*)Y)[p * COUTP + co] = (__bf16)v;
            } else if (MODE == CONV_OUT) {
                if (co < 2) ((float*)Y)[p * 2 + co] = v + bias[co];
            } else {
                const float m = (float)Mk[p * COUTP + co];
                ((__bf16*)Y)[p * COUTP + co] = (m > 0.0f) ? (__bf16)v : (__bf16)0.0f;
            }
        }
    }
}

template <int CINP, int COUTP, int MODE>
static void conv_launch(int H, int Wd, const __bf16* X, const __bf16* Wp, const float* bias, const __bf16* Mk, void* Y,
                        hipStream_t s) {
    dim3 grid((Wd + 63) / 64, H);
    hipLaunchKernelGGL((conv3x3_kernel<CINP, COUTP, MODE>), grid, dim3(256), 0, s, H, Wd, X, Wp, bias, Mk, Y);
}

// ||r||^2 from nparts <= 64 partial sums: lane l of every wave loads part l and
// a butterfly adds them; each step adds the same two values in every lane
// (in either order: the same bits), so every thread gets the same sum
__device__ __forceinline__ double sum_parts(const double* __restrict__ parts, int nparts) {
    const int lane = threadIdx.x & 63;
    double s = lane < nparts ? parts[lane] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// --------------------------------------------------------------------------
// Fused smoother step (inference): input packing, the four layers and the
// update of x in one kernel.  A workgroup owns an output
// tile of FT_H x FT_W pixels and computes every layer on the tile grown by the
// halo the later layers need (input: +4 pixels on each side, layer 0: +3,
// layer 1: +2, layer 2: +1), the activations of each stage staying in LDS,
// with all four layers' packed weights copied into LDS at the start together
// with the input tile (one round trip to memory).  Every output pixel of every
// layer is formed by the same MFMA sequence as conv3x3_kernel (same operand
// fragments, taps in the same order), so the result is bit-identical to the
// four separate launches; stage pixels outside the grid are stored as zero, the
// padding the separate launches read.
// --------------------------------------------------------------------------
constexpr int FT_H = 16, FT_W = 32, FUSED_TB = 512;
// LDS (BF16 elements): packed weights of layers 0..3, then two activation
// regions used alternately (input tile / layer-1 output, layer-0 / layer-2 output)
constexpr int FW0 = 9 * 32 * 8, FW1 = 9 * 32 * 32, FW3 = 9 * 16 * 32;
constexpr int FIN = (FT_H + 8) * (FT_W + 8) * 8, FA0 = (FT_H + 6) * (FT_W + 6) * 32;
constexpr int FA1 = (FT_H + 4) * (FT_W + 4) * 32, FA2 = (FT_H + 2) * (FT_W + 2) * 32;
constexpr int FRA = FIN > FA1 ? FIN : FA1, FRB = FA0 > FA2 ? FA0 : FA2;
constexpr int FUSED_LDS = 2 * (FW0 + 2 * FW1 + FW3 + FRA + FRB);   // bytes

extern __shared__ __attribute__((aligned(16))) __bf16 cnn_smem[];

// n16 16-byte chunks from global src to LDS dst: clamped addresses (n16 >= 1)
// and unconditional stores (the last chunk may be written twice with its own
// value), so all of a thread's loads are issued before its first store
template <int PER>
__device__ __forceinline__ void stage_chunks(uint4* dst, const uint4* __restrict__ src, int n16) {
    uint4 v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) v[q] = src[min((int)threadIdx.x + q * FUSED_TB, n16 - 1)];
#pragma unroll
    for (int q = 0; q < PER; ++q) dst[min((int)threadIdx.x + q * FUSED_TB, n16 - 1)] = v[q];
}

// One stage: out[px][COUTP] = act(conv3x3(in)) over a (R x C) pixel region whose
// source region is (R + 2) x (C + 2), pixels linearised row-major; M-tiles of
// 16 pixels go to the waves in turn.  (gr0, gc0): grid position of the region's
// first pixel.  LAST: the network output (2 real channels, FP32, bias, no ReLU)
// written to Y[pixel][2] (LDS, the region's pixels) for pixels of the grid.  Ws:
// the layer's packed weights in LDS.
template <int CINP, int COUTP, bool LAST>
__device__ __forceinline__ void fused_stage(const __bf16* in, __bf16* outs, int R, int C, int gr0, int gc0, int H,
                                            int Wd, const __bf16* Ws, const float* __restrict__ bias,
                                            float* __restrict__ Y) {
    constexpr int NT = COUTP / 16;
    constexpr int KSTEPS = (CINP == 32) ? 9 : 3;
    constexpr int NW = FUSED_TB / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g = lane >> 4, col = lane & 15;
    const int Cs = C + 2;   // source region width
    bf16x8 bw[KSTEPS][NT];
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
        const int tap = (CINP == 32) ? s : 4 * s + g;
        const int ci0 = (CINP == 32) ? 8 * g : 0;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            if (tap < 9) {
                bw[s][nt] = *(const bf16x8*)(Ws + (tap * COUTP + nt * 16 + col) * CINP + ci0);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) bw[s][nt][e] = (__bf16)0.0f;
            }
        }
    }
    const int npx = R * C, ntiles = (npx + 15) / 16;
    for (int mt = wave; mt < ntiles; mt += NW) {
        // A-operand row of this lane: pixel mt*16 + col (clamped into the region)
        const int pa = min(mt * 16 + col, npx - 1);
        const int ra = pa / C, ca = pa - ra * C;
        f32x4 acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s) {
            const int tap = (CINP == 32) ? s : 4 * s + g;
            const int ci0 = (CINP == 32) ? 8 * g : 0;
            bf16x8 a;
            if (tap < 9) {
                const int dy = tap / 3, dx = tap - 3 * dy;
                a = *(const bf16x8*)(in + ((ra + dy) * Cs + (ca + dx)) * CINP + ci0);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) a[e] = (__bf16)0.0f;
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[s][nt], acc[nt], 0, 0, 0);
        }
        // D: output channel nt*16 + col for pixels mt*16 + 4g .. + 3 (their region
        // rows and columns from one division: C >= 4, so at most one row break)
        const int pb = mt * 16 + 4 * g;
        const int rb = pb / C, cb = pb - rb * C;
        bool ing[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int wrap = (cb + i >= C) ? 1 : 0;
            const int gr = gr0 + rb + wrap, gc = gc0 + cb + i - wrap * C;
            ing[i] = gr >= 0 && gr < H && gc >= 0 && gc < Wd;
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int co = nt * 16 + col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int po = pb + i;
                if (po >= npx) continue;
                const float v = acc[nt][i];
                if (LAST) {
                    if (co < 2 && ing[i]) Y[po * 2 + co] = v + bias[co];
                } else {
                    outs[po * COUTP + co] = ing[i] ? (__bf16)fmaxf(v + bias[co], 0.0f) : (__bf16)0.0f;
                }
            }
        }
    }
    __syncthreads();
}

// The whole smoother step: rms = ||r|| / sqrt(N) from the norm partials, the
// packed input (r / rms, c) of the tile, the four layers, and
// x (+)= omega D^-1 r + rms C(r / rms, c) on the tile's pixels, with the same
// formulas as pack_input_kernel and apply_step_kernel.
template <class TV>
__global__ __launch_bounds__(FUSED_TB) void cnn_fused_kernel(
    int H, int Wd, const cx<TV>* __restrict__ r, const double* __restrict__ nr2, int nparts,
    const float* __restrict__ feat, const __bf16* __restrict__ W0, const float* __restrict__ b0,
    const __bf16* __restrict__ W1, const float* __restrict__ b1, const __bf16* __restrict__ W2,
    const float* __restrict__ b2, const __bf16* __restrict__ W3, const float* __restrict__ b3,
    const cx<TV>* __restrict__ dinv, TV omega, cx<TV>* __restrict__ x, int accumulate) {
    __bf16* sW0 = cnn_smem;
    __bf16* sW1 = sW0 + FW0;
    __bf16* sW2 = sW1 + FW1;
    __bf16* sW3 = sW2 + FW1;
    __bf16* rA = sW3 + FW3;
    __bf16* rB = rA + FRA;
    const int r0 = blockIdx.y * FT_H, c0 = blockIdx.x * FT_W;
    const long long N = (long long)H * Wd;
    const double nrs = sum_parts(nr2, nparts);   // every lane takes part (butterfly)
    stage_chunks<1>((uint4*)sW0, (const uint4*)W0, FW0 / 8);
    stage_chunks<3>((uint4*)sW1, (const uint4*)W1, FW1 / 8);
    stage_chunks<3>((uint4*)sW2, (const uint4*)W2, FW1 / 8);
    stage_chunks<2>((uint4*)sW3, (const uint4*)W3, FW3 / 8);
    {
        // packed input tile (r / rms, c, 0...), zero outside the grid (values
        // read at a clamped valid pixel)
        constexpr int RI = FT_H + 8, CI = FT_W + 8;
        for (int e = threadIdx.x; e < RI * CI; e += FUSED_TB) {
            const int rr = e / CI, cc = e - rr * CI;
            const int gr = r0 - 4 + rr, gc = c0 - 4 + cc;
            const bool ok = gr >= 0 && gr < H && gc >= 0 && gc < Wd;
            const long long p = (long long)min(max(gr, 0), H - 1) * Wd + min(max(gc, 0), Wd - 1);
            const double nr = sqrt(nrs);
            const double inv = nr > 0.0 ? sqrt((double)N) / nr : 0.0;
            const cx<TV> v = r[p];
            const float fv = feat[p];
            bf16x8 o;
            o[0] = (__bf16)(float)(v.re * inv);
            o[1] = (__bf16)(float)(v.im * inv);
            o[2] = (__bf16)fv;
#pragma unroll
            for (int k = 3; k < 8; ++k) o[k] = (__bf16)0.0f;
            if (!ok) {
#pragma unroll
                for (int k = 0; k < 8; ++k) o[k] = (__bf16)0.0f;
            }
            *(bf16x8*)(rA + e * 8) = o;
        }
    }
    __syncthreads();
    fused_stage<8, 32, false>(rA, rB, FT_H + 6, FT_W + 6, r0 - 3, c0 - 3, H, Wd, sW0, b0, nullptr);
    fused_stage<32, 32, false>(rB, rA, FT_H + 4, FT_W + 4, r0 - 2, c0 - 2, H, Wd, sW1, b1, nullptr);
    fused_stage<32, 32, false>(rA, rB, FT_H + 2, FT_W + 2, r0 - 1, c0 - 1, H, Wd, sW2, b2, nullptr);
    float* outs = (float*)rA;   // the network output of the tile, [pixel][2]
    fused_stage<32, 16, true>(rB, nullptr, FT_H, FT_W, r0, c0, H, Wd, sW3, b3, outs);
    // x (+)= omega D^-1 r + rms out on the tile's pixels of the grid
    if (threadIdx.x < FT_H * FT_W) {
        const int e = threadIdx.x, gr = r0 + e / FT_W, gc = c0 + e % FT_W;
        if (gr < H && gc < Wd) {
            const long long p = (long long)gr * Wd + gc;
            const double rms = sqrt(nrs / (double)N);
            const cx<TV> d = dinv[p], v = r[p];
            const TV sr = omega * (d.re * v.re - d.im * v.im) + (TV)(rms * outs[e * 2]);
            const TV si = omega * (d.re * v.im + d.im * v.re) + (TV)(rms * outs[e * 2 + 1]);
            if (accumulate) {
                const cx<TV> o = x[p];
                x[p] = {o.re + sr, o.im + si};
            } else {
                x[p] = {sr, si};
            }
        }
    }
}

// --------------------------------------------------------------------------
// Weight gradient: G[tap][co][ci] = sum_p gY[p][co] X[p + off(tap)][ci] and
// Gb[co] = sum_p gY[p][co].  A GEMM with a small output (M = output channels,
// N = input channels, per tap) and K = all pixels, on v_mfma_f32_16x16x32_bf16:
// A[co][k] = gY[pixel k][co], B[k][ci] = X[pixel k + off][ci], 32 pixels per
// MFMA.  A workgroup walks 4 x 64-pixel tiles (grid-stride) with its
// accumulators in registers; a tile is staged transposed in LDS, channel-major,
// with one copy of X per horizontal tap offset, so that a lane's 8 consecutive
// pixels are one aligned 16-byte read.  The bias sums use a B operand of ones.
// Per-workgroup partial sums are then added in workgroup order (deterministic).
// --------------------------------------------------------------------------
constexpr int WG_TH = 4, WG_TW = 64;
constexpr int WG_MAXBLK = 1024;   // workgroups (and partial sums per output)

template <int CINP, int COUTP>
__global__ __launch_bounds__(256) void wgrad_kernel(int H, int Wd, int ci_n, int co_n, const __bf16* __restrict__ X,
                                                    const __bf16* __restrict__ gY, float* __restrict__ part) {
    constexpr int NCI = CINP >= 16 ? CINP : 16;     // input channels padded to MFMA tiles
    constexpr int NCO = COUTP >= 16 ? COUTP : 16;   // output channels padded
    constexpr int TCI = NCI / 16, TCO = NCO / 16;
    constexpr int NT = 9 * TCO * TCI;               // output tiles (tap, co tile, ci tile)
    constexpr int PER_WAVE = (NT + 3) / 4;
    __shared__ __attribute__((aligned(16))) __bf16 xsT[3][NCI][WG_TH + 2][WG_TW];
    __shared__ __attribute__((aligned(16))) __bf16 gsT[NCO][WG_TH][WG_TW];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int g = lane >> 4, col = lane & 15;
    const int tiles_x = (Wd + WG_TW - 1) / WG_TW, tiles = tiles_x * ((H + WG_TH - 1) / WG_TH);
    f32x4 acc[PER_WAVE], accb[TCO];
#pragma unroll
    for (int q = 0; q < PER_WAVE; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < TCO; ++q) accb[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 ones;
#pragma unroll
    for (int e = 0; e < 8; ++e) ones[e] = (__bf16)1.0f;
    for (int t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int x0 = (t % tiles_x) * WG_TW, h0 = (t / tiles_x) * WG_TH;
        // X over the tile grown by one pixel, into the three tap-shifted copies
        for (int idx = tid; idx < (WG_TH + 2) * (WG_TW + 2) * NCI; idx += 256) {
            const int c = idx % NCI, rest = idx / NCI;
            const int px = rest % (WG_TW + 2), r = rest / (WG_TW + 2);
            const int hh = h0 + r - 1, ww = x0 + px - 1;
            __bf16 v = (__bf16)0.0f;
            if (c < ci_n && hh >= 0 && hh < H && ww >= 0 && ww < Wd) v = X[((size_t)hh * Wd + ww) * CINP + c];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int q = px - dx;
                if (q >= 0 && q < WG_TW) xsT[dx][c][r][q] = v;
            }
        }
        for (int idx = tid; idx < WG_TH * WG_TW * NCO; idx += 256) {
            const int c = idx % NCO, rest = idx / NCO;
            const int px = rest % WG_TW, r = rest / WG_TW;
            const int hh = h0 + r, ww = x0 + px;
            __bf16 v = (__bf16)0.0f;
            if (c < co_n && hh < H && ww < Wd) v = gY[((size_t)hh * Wd + ww) * COUTP + c];
            gsT[c][r][px] = v;
        }
        __syncthreads();
#pragma unroll
        for (int ch = 0; ch < WG_TH * WG_TW / 32; ++ch) {
            const int r = ch >> 1, px = (ch & 1) * 32 + 8 * g;
            bf16x8 a[TCO];
#pragma unroll
            for (int ct = 0; ct < TCO; ++ct) a[ct] = *(const bf16x8*)&gsT[ct * 16 + col][r][px];
            if (wave == 0) {
#pragma unroll
                for (int ct = 0; ct < TCO; ++ct)
                    accb[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ct], ones, accb[ct], 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < PER_WAVE; ++q) {
                const int ot = wave + 4 * q;
                if (ot >= NT) break;
                const int tap = ot / (TCO * TCI), ct = (ot / TCI) % TCO, it = ot % TCI;
                const int dy = tap / 3, dx = tap - 3 * dy;
                const bf16x8 b = *(const bf16x8*)&xsT[dx][it * 16 + col][r + dy][px];
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ct], b, acc[q], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D layout: lane holds n = col (input channel), m = 4 g + i (output channel)
    const int nw = 9 * co_n * ci_n;
    float* out = part + (size_t)blockIdx.x * (nw + co_n);
#pragma unroll
    for (int q = 0; q < PER_WAVE; ++q) {
        const int ot = wave + 4 * q;
        if (ot >= NT) break;
        const int tap = ot / (TCO * TCI), ct = (ot / TCI) % TCO, it = ot % TCI;
        const int ci = it * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co = ct * 16 + 4 * g + i;
            if (co < co_n && ci < ci_n) out[((size_t)tap * co_n + co) * ci_n + ci] = acc[q][i];
        }
    }
    if (wave == 0 && col == 0) {
#pragma unroll
        for (int ct = 0; ct < TCO; ++ct)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = ct * 16 + 4 * g + i;
                if (co < co_n) out[nw + co] = accb[ct][i];
            }
    }
}

// out[o] = sum over the nblk workgroup partials of o.  A workgroup of RP_WAVES
// waves owns 64 outputs (lane = output, coalesced rows): wave w adds partials
// w, w + RP_WAVES, ... in that order, four loads in flight, and wave 0 adds
// the waves' sums in wave order (a fixed order: the same bits every run).
constexpr int RP_WAVES = 16;
__global__ __launch_bounds__(64 * RP_WAVES) void reduce_parts_kernel(int nblk, int nout, const float* __restrict__ part,
                                                                     float* __restrict__ out) {
    __shared__ float sh[RP_WAVES][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (o < nout) {
        int b = w;
        for (; b + 3 * RP_WAVES < nblk; b += 4 * RP_WAVES) {
            const float v0 = part[(size_t)b * nout + o];
            const float v1 = part[(size_t)(b + RP_WAVES) * nout + o];
            const float v2 = part[(size_t)(b + 2 * RP_WAVES) * nout + o];
            const float v3 = part[(size_t)(b + 3 * RP_WAVES) * nout + o];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; b < nblk; b += RP_WAVES) s += part[(size_t)b * nout + o];
    }
    sh[w][lane] = s;
    __syncthreads();
    if (w == 0 && o < nout) {
        float t = sh[0][lane];
        for (int q = 1; q < RP_WAVES; ++q) t += sh[q][lane];
        out[o] = t;
    }
}

// --------------------------------------------------------------------------
// Input packing, output application, loss gradient
// --------------------------------------------------------------------------
// X0[p] = (r.re / rms, r.im / rms, c[p], 0, 0, 0, 0, 0) with rms = ||r|| / sqrt(N),
// ||r||^2 = *nr2 (entries of order one whatever the grid size)

template <class TV>
__global__ void pack_input_kernel(long long N, const cx<TV>* __restrict__ r, const double* __restrict__ nr2,
                                  int nparts, const float* __restrict__ feat, __bf16* __restrict__ X0) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const double nr = sqrt(sum_parts(nr2, nparts));   // every lane takes part (butterfly)
    if (p >= N) return;
    const double inv = nr > 0.0 ? sqrt((double)N) / nr : 0.0;
    const cx<TV> v = r[p];
    bf16x8 o;
    o[0] = (__bf16)(float)(v.re * inv);
    o[1] = (__bf16)(float)(v.im * inv);
    o[2] = (__bf16)feat[p];
#pragma unroll
    for (int e = 3; e < 8; ++e) o[e] = (__bf16)0.0f;
    *(bf16x8*)(X0 + p * 8) = o;
}

// x (+)= omega D^-1 r + rms * out  (smoother step), out: complex FP32 network output
template <class TV>
__global__ void apply_step_kernel(long long N, const float* __restrict__ out, const double* __restrict__ nr2,
                                  int nparts, const cx<TV>* __restrict__ r, const cx<TV>* __restrict__ dinv,
                                  TV omega, cx<TV>* __restrict__ x, int accumulate) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const double rms = sqrt(sum_parts(nr2, nparts) / (double)N);   // every lane takes part (butterfly)
    if (p >= N) return;
    const cx<TV> d = dinv[p], v = r[p];
    const TV sr = omega * (d.re * v.re - d.im * v.im) + (TV)(rms * out[2 * p]);
    const TV si = omega * (d.re * v.im + d.im * v.re) + (TV)(rms * out[2 * p + 1]);
    if (accumulate) {
        const cx<TV> o = x[p];
        x[p] = {o.re + sr, o.im + si};
    } else {
        x[p] = {sr, si};
    }
}

// gOut[p] = -(2 rms / nr^2) * y[p] (real channels re, im; padded to 8), y = conj(M_beta) r'
__global__ void loss_grad_pack_kernel(long long N, const cx<double>* __restrict__ y, const double* nr2,
                                      __bf16* __restrict__ g) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const double nr = sqrt(*nr2);
    const double f = nr > 0.0 ? -2.0 / (nr * sqrt((double)N)) : 0.0;
    bf16x8 o;
    o[0] = (__bf16)(float)(f * y[p].re);
    o[1] = (__bf16)(float)(f * y[p].im);
#pragma unroll
    for (int e = 2; e < 8; ++e) o[e] = (__bf16)0.0f;
    *(bf16x8*)(g + p * 8) = o;
}

// s = omega D^-1 r + rms * out (complex FP64) for the loss
__global__ void scale_out_kernel(long long N, const float* __restrict__ out, const double* nr2,
                                 const cx<double>* __restrict__ r, const cx<double>* __restrict__ dinv, double omega,
                                 cx<double>* __restrict__ s) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const double rms = sqrt(*nr2 / (double)N);
    const cx<double> d = dinv[p], v = r[p];
    s[p] = {omega * (d.re * v.re - d.im * v.im) + rms * (double)out[2 * p],
            omega * (d.re * v.im + d.im * v.re) + rms * (double)out[2 * p + 1]};
}

// --------------------------------------------------------------------------
// Parameter handling: complex master parameters (float pairs), real-expanded
// BF16 packing, gradient folding and Adam.
// --------------------------------------------------------------------------
// Layer l parameter block: W[co][ci][dy][dx] (complex) then b[co] (complex).
struct LayerDims {
    int cin, cout;      // complex channels
    int cinp, coutp;    // padded real channels of the packed forward weights
    int off;            // offset of W (in complex entries) in the parameter vector
};

// dn: output channels of the data-gradient conv (the layer's input channels),
// dk: its input channels (the layer's output channels, padded)
__global__ void pack_weights_kernel(LayerDims d, const float* __restrict__ theta, __bf16* __restrict__ Wf,
                                    __bf16* __restrict__ Wd, int dn, int dk, float* __restrict__ bias) {
    // forward: Wf[tap][co_r][ci_r]; data-gradient: Wd[8 - tap][ci_r][co_r] ([tap'][dn][dk])
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = 9 * d.coutp * d.cinp;
    if (idx < nf) {
        const int ci_r = idx % d.cinp, rest = idx / d.cinp;
        const int co_r = rest % d.coutp, tap = rest / d.coutp;
        float v = 0.0f;
        if (ci_r < 2 * d.cin && co_r < 2 * d.cout) {
            const int o = co_r >> 1, s = co_r & 1, i = ci_r >> 1, t = ci_r & 1;
            const int dy = tap / 3, dx = tap % 3;
            const size_t w = (size_t)d.off + (((size_t)o * d.cin + i) * 3 + dy) * 3 + dx;
            const float a = theta[2 * w], b = theta[2 * w + 1];
            v = (s == 0) ? (t == 0 ? a : -b) : (t == 0 ? b : a);
        }
        Wf[idx] = (__bf16)v;
        if (Wd && co_r < dk && ci_r < dn) Wd[((size_t)(8 - tap) * dn + ci_r) * dk + co_r] = (__bf16)v;
    }
    if (idx < d.coutp) {
        float v = 0.0f;
        if (idx < 2 * d.cout) {
            const size_t bo = (size_t)d.off + (size_t)d.cout * d.cin * 9 + (idx >> 1);
            v = theta[2 * bo + (idx & 1)];
        }
        bias[idx] = v;
    }
}

// Complex gradient of layer d from the real-expanded G[tap][co_r][ci_r] (ci_n, co_n
// real channels) and Gb[co_r]: g_a = G[2o][2i] + G[2o+1][2i+1], g_b = G[2o+1][2i] - G[2o][2i+1].
__global__ void fold_grad_kernel(LayerDims d, int ci_n, int co_n, const float* __restrict__ G, float* __restrict__ grad) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = d.cout * d.cin * 9;
    if (idx < nw) {
        const int tapflat = idx % 9, rest = idx / 9;
        const int i = rest % d.cin, o = rest / d.cin;
        auto g = [&](int co_r, int ci_r) { return G[((size_t)tapflat * co_n + co_r) * ci_n + ci_r]; };
        const float ga = g(2 * o, 2 * i) + g(2 * o + 1, 2 * i + 1);
        const float gb = g(2 * o + 1, 2 * i) - g(2 * o, 2 * i + 1);
        const size_t w = (size_t)d.off + idx;
        grad[2 * w] = ga;
        grad[2 * w + 1] = gb;
    } else if (idx < nw + d.cout) {
        const int o = idx - nw;
        const float* Gb = G + (size_t)9 * co_n * ci_n;
        const size_t w = (size_t)d.off + nw + o;
        grad[2 * w] = Gb[2 * o];
        grad[2 * w + 1] = Gb[2 * o + 1];
    }
}

__global__ void adam_kernel(int n, float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    m[i] = b1 * m[i] + (1.0f - b1) * gi;
    v[i] = b2 * v[i] + (1.0f - b2) * gi * gi;
    theta[i] -= lr * (m[i] / c1) / (sqrtf(v[i] / c2) + eps);
}

// ||x||^2 as per-workgroup partial sums (FP64, tree in LDS): parts[blockIdx.x]
constexpr int kNormParts = 64;
template <class TV>
__global__ __launch_bounds__(256) void norm2_parts_kernel(long long N, const cx<TV>* __restrict__ x,
                                                          double* __restrict__ parts) {
    __shared__ double sh[256];
    double s = 0.0;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < N; t += (long long)gridDim.x * 256) {
        const cx<TV> v = x[t];
        s += (double)v.re * v.re + (double)v.im * v.im;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[blockIdx.x] = sh[0];
}

// The total of norm2_parts_kernel's partial sums (one wave, fixed order)
__global__ __launch_bounds__(64) void norm2_total_kernel(const double* __restrict__ parts, int nparts, double* out) {
    const double s = sum_parts(parts, nparts);
    if (threadIdx.x == 0) *out = s;
}

static inline unsigned g1(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------
CnnImpl::CnnImpl(unsigned long long seed) {
    int off = 0;
    for (int l = 0; l < 4; ++l) {
        LayerInfo& L = layers[l];
        L.cin = kChannels[l];
        L.cout = kChannels[l + 1];
        L.cinp = (l == 0) ? 8 : 32;
        L.coutp = (l == 3) ? 16 : 32;
        L.off = off;
        off += L.cout * L.cin * 9 + L.cout;
    }
    nparam = off;
    // seeded initial parameters (SplitMix64 -> Box-Muller), scale 0.5/sqrt(9 cin)
    std::vector<float> th(2 * (size_t)nparam, 0.0f);
    unsigned long long st = seed;
    auto next = [&]() {
        st += 0x9E3779B97F4A7C15ULL;
        unsigned long long z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    };
    auto unif = [&]() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
    auto normal = [&]() { return std::sqrt(-2.0 * std::log(unif())) * std::cos(2.0 * M_PI * unif()); };
    for (int l = 0; l < 4; ++l) {
        const LayerInfo& L = layers[l];
        const double sc = 0.5 / std::sqrt(9.0 * L.cin);
        for (int i = 0; i < L.cout * L.cin * 9; ++i) {
            th[2 * (L.off + i)] = (float)(sc * normal());
            th[2 * (L.off + i) + 1] = (float)(sc * normal());
        }
    }
    upload(theta, th);
    std::vector<float> z(2 * (size_t)nparam, 0.0f);
    upload(adam_m, z);
    upload(adam_v, z);
    upload(grad, z);
    for (int l = 0; l < 4; ++l) {
        LayerInfo& L = layers[l];
        L.wf.alloc((size_t)9 * L.coutp * L.cinp * 2);
        L.bias.alloc((size_t)L.coutp * 4);
        // data-gradient weights map the layer's output channels (padded to 8 or
        // 32) back to its input channels (32); the input layer needs none
        if (l > 0) {
            L.dinp = (l == 3) ? 8 : 32;
            L.doutp = 32;
            L.wd.alloc((size_t)9 * L.dinp * L.doutp * 2);
            HH_HIP(hipMemset(L.wd.p, 0, L.wd.bytes));
        }
    }
    repack(nullptr);
    HH_HIP(hipDeviceSynchronize());
}

void CnnImpl::repack(hipStream_t s) {
    for (int l = 0; l < 4; ++l) {
        LayerInfo& L = layers[l];
        LayerDims d{L.cin, L.cout, L.cinp, L.coutp, L.off};
        const int n = 9 * L.coutp * L.cinp;
        hipLaunchKernelGGL(pack_weights_kernel, dim3(g1(n, 256)), dim3(256), 0, s, d, theta.as<float>(),
                           L.wf.as<__bf16>(), l > 0 ? L.wd.as<__bf16>() : nullptr, L.doutp, L.dinp,
                           L.bias.as<float>());
    }
}

void CnnImpl::set_params(const float* host, int n) {
    HH_REQUIRE(n == 2 * nparam, "parameter count mismatch");
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) throw Err{HH_ENUMERIC, "non-finite network parameter"};
    HH_HIP(hipMemcpy(theta.p, host, (size_t)n * 4, hipMemcpyHostToDevice));
    HH_HIP(hipMemset(adam_m.p, 0, adam_m.bytes));
    HH_HIP(hipMemset(adam_v.p, 0, adam_v.bytes));
    adam_t = 0;
    repack(nullptr);
    HH_HIP(hipDeviceSynchronize());
}

void CnnImpl::ensure(int H, int Wd) {
    if (H == gH && Wd == gW) return;
    gH = H;
    gW = Wd;
    const size_t P = (size_t)H * Wd;
    x0.alloc(P * 8 * 2);
    for (int l = 0; l < 3; ++l) act[l].alloc(P * 32 * 2);
    out.alloc(P * 2 * 4);
    gA.alloc(P * 32 * 2);
    gB.alloc(P * 32 * 2);
    gOut.alloc(P * 8 * 2);
    sbuf.alloc(P * 16);
    rbuf.alloc(P * 16);
    ybuf.alloc(P * 16);
    scal.alloc(8 * (8 + kNormParts));   // [0] ||r||^2, [1] ||r'||^2 (loss); [8..] partial sums
    const int nblk = std::min(((Wd + WG_TW - 1) / WG_TW) * ((H + WG_TH - 1) / WG_TH), WG_MAXBLK);
    part.alloc((size_t)nblk * (9 * 32 * 32 + 32) * 4);
    gfull.alloc((size_t)(9 * 32 * 32 + 32) * 4);
}

// Network forward on the packed input x0 (activations kept in act[]); output in `out`.
void CnnImpl::forward(int H, int Wd, hipStream_t s) {
    conv_launch<8, 32, CONV_RELU>(H, Wd, x0.as<__bf16>(), layers[0].wf.as<__bf16>(), layers[0].bias.as<float>(),
                                  nullptr, act[0].p, s);
    conv_launch<32, 32, CONV_RELU>(H, Wd, act[0].as<__bf16>(), layers[1].wf.as<__bf16>(), layers[1].bias.as<float>(),
                                   nullptr, act[1].p, s);
    conv_launch<32, 32, CONV_RELU>(H, Wd, act[1].as<__bf16>(), layers[2].wf.as<__bf16>(), layers[2].bias.as<float>(),
                                   nullptr, act[2].p, s);
    conv_launch<32, 16, CONV_OUT>(H, Wd, act[2].as<__bf16>(), layers[3].wf.as<__bf16>(), layers[3].bias.as<float>(),
                                  nullptr, out.p, s);
}

template <class TV>
void CnnImpl::step(int H, int Wd, const cx<TV>* r, const float* feat, const cx<TV>* dinv, TV omega, cx<TV>* x,
                   int accumulate, hipStream_t s) {
    ensure(H, Wd);
    const long long N = (long long)H * Wd;
    // r read twice (norm, network input), D^-1 and the feature once, x read
    // (accumulate) and written; the network: 9 taps of complex channels
    // 2 -> 16 -> 16 -> 16 -> 1 (a complex MAC counts 8) per pixel
    meter((double)N * (3.0 * sizeof(cx<TV>) + 4.0 + (accumulate ? 2.0 : 1.0) * sizeof(cx<TV>)),
          8.0 * 9.0 * (2 * 16 + 16 * 16 + 16 * 16 + 16 * 1) * (double)N + 16.0 * N);
    double* parts = scal.as<double>() + 8;   // kNormParts partial sums of ||r||^2
    const int np = (int)std::min<long long>(kNormParts, (N + 255) / 256);
    hipLaunchKernelGGL(norm2_parts_kernel<TV>, dim3(np), dim3(256), 0, s, N, r, parts);
    if (fused) {
        // the rest of the step in one kernel
        HH_HIP(hipFuncSetAttribute((const void*)cnn_fused_kernel<TV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   FUSED_LDS));
        dim3 grid((Wd + FT_W - 1) / FT_W, (H + FT_H - 1) / FT_H);
        hipLaunchKernelGGL(cnn_fused_kernel<TV>, grid, dim3(FUSED_TB), FUSED_LDS, s, H, Wd, r, parts, np, feat,
                           layers[0].wf.as<__bf16>(), layers[0].bias.as<float>(), layers[1].wf.as<__bf16>(),
                           layers[1].bias.as<float>(), layers[2].wf.as<__bf16>(), layers[2].bias.as<float>(),
                           layers[3].wf.as<__bf16>(), layers[3].bias.as<float>(), dinv, omega, x, accumulate);
        return;
    }
    hipLaunchKernelGGL(pack_input_kernel<TV>, dim3(g1(N, 256)), dim3(256), 0, s, N, r, parts, np, feat,
                       x0.as<__bf16>());
    forward(H, Wd, s);
    hipLaunchKernelGGL(apply_step_kernel<TV>, dim3(g1(N, 256)), dim3(256), 0, s, N, out.as<float>(), parts, np, r,
                       dinv, omega, x, accumulate);
}
template void CnnImpl::step<float>(int, int, const cx<float>*, const float*, const cx<float>*, float, cx<float>*, int,
                                   hipStream_t);
template void CnnImpl::step<double>(int, int, const cx<double>*, const float*, const cx<double>*, double, cx<double>*,
                                    int, hipStream_t);

void CnnImpl::wgrad(int l, int H, int Wd, const __bf16* X, int cinp, const __bf16* gY, int coutp, int ci_n, int co_n,
                    hipStream_t s) {
    const int tiles = ((Wd + WG_TW - 1) / WG_TW) * ((H + WG_TH - 1) / WG_TH);
    const int nblk = std::min(tiles, WG_MAXBLK);
    const dim3 grid(nblk);
    const int nout = 9 * ci_n * co_n + co_n;
    if (cinp == 8 && coutp == 32)
        hipLaunchKernelGGL((wgrad_kernel<8, 32>), grid, dim3(256), 0, s, H, Wd, ci_n, co_n, X, gY, part.as<float>());
    else if (cinp == 32 && coutp == 32)
        hipLaunchKernelGGL((wgrad_kernel<32, 32>), grid, dim3(256), 0, s, H, Wd, ci_n, co_n, X, gY, part.as<float>());
    else
        hipLaunchKernelGGL((wgrad_kernel<32, 8>), grid, dim3(256), 0, s, H, Wd, ci_n, co_n, X, gY, part.as<float>());
    hipLaunchKernelGGL(reduce_parts_kernel, dim3(g1(nout, 64)), dim3(64 * RP_WAVES), 0, s, nblk, nout,
                       part.as<float>(), gfull.as<float>());
    const LayerInfo& L = layers[l];
    LayerDims d{L.cin, L.cout, L.cinp, L.coutp, L.off};
    const int nf = L.cout * L.cin * 9 + L.cout;
    hipLaunchKernelGGL(fold_grad_kernel, dim3(g1(nf, 256)), dim3(256), 0, s, d, ci_n, co_n, gfull.as<float>(),
                       grad.as<float>());
}

// Loss and parameter gradient for one residual sample r on the grid (H, Wd):
// s = omega D^-1 r + rms(r) C(r/rms(r), c), rms(r) = ||r||/sqrt(N), r' = r - M_beta s,
// L = ||r'||^2 / ||r||^2.
// `mbeta(x, b, y, conj)` computes y = b - M_beta x (conj = 0) or y = conj(M_beta) x
// (conj = 1) on the caller's stream.
double CnnImpl::loss_grad(int H, int Wd, const cx<double>* r, const float* feat, const cx<double>* dinv,
                          double omega, const MbetaFn& mbeta, hipStream_t s) {
    ensure(H, Wd);
    const long long N = (long long)H * Wd;
    double* nr2 = scal.as<double>();
    double* rn2 = nr2 + 1;
    // ||r||^2 and ||r'||^2: partial sums over up to 64 workgroups, then their total
    double* parts = nr2 + 8;
    const int np = (int)std::min<long long>(kNormParts, (N + 255) / 256);
    hipLaunchKernelGGL(norm2_parts_kernel<double>, dim3(np), dim3(256), 0, s, N, r, parts);
    hipLaunchKernelGGL(norm2_total_kernel, dim3(1), dim3(64), 0, s, parts, np, nr2);
    hipLaunchKernelGGL(pack_input_kernel<double>, dim3(g1(N, 256)), dim3(256), 0, s, N, r, nr2, 1, feat,
                       x0.as<__bf16>());
    forward(H, Wd, s);
    hipLaunchKernelGGL(scale_out_kernel, dim3(g1(N, 256)), dim3(256), 0, s, N, out.as<float>(), nr2, r, dinv, omega,
                       sbuf.as<cx<double>>());
    mbeta(sbuf.as<cx<double>>(), r, rbuf.as<cx<double>>(), 0);          // r' = r - M s
    hipLaunchKernelGGL(norm2_parts_kernel<double>, dim3(np), dim3(256), 0, s, N, rbuf.as<cx<double>>(), parts);
    hipLaunchKernelGGL(norm2_total_kernel, dim3(1), dim3(64), 0, s, parts, np, rn2);
    mbeta(rbuf.as<cx<double>>(), nullptr, ybuf.as<cx<double>>(), 1);   // y = conj(M) r'
    hipLaunchKernelGGL(loss_grad_pack_kernel, dim3(g1(N, 256)), dim3(256), 0, s, N, ybuf.as<cx<double>>(), nr2,
                       gOut.as<__bf16>());
    // layer 3 (16 complex -> 1): weights, then the data gradient into act[2]'s space
    wgrad(3, H, Wd, act[2].as<__bf16>(), 32, gOut.as<__bf16>(), 8, 32, 2, s);
    conv_launch<8, 32, CONV_MASK>(H, Wd, gOut.as<__bf16>(), layers[3].wd.as<__bf16>(), nullptr, act[2].as<__bf16>(),
                                  gA.p, s);
    wgrad(2, H, Wd, act[1].as<__bf16>(), 32, gA.as<__bf16>(), 32, 32, 32, s);
    conv_launch<32, 32, CONV_MASK>(H, Wd, gA.as<__bf16>(), layers[2].wd.as<__bf16>(), nullptr, act[1].as<__bf16>(),
                                   gB.p, s);
    wgrad(1, H, Wd, act[0].as<__bf16>(), 32, gB.as<__bf16>(), 32, 32, 32, s);
    conv_launch<32, 32, CONV_MASK>(H, Wd, gB.as<__bf16>(), layers[1].wd.as<__bf16>(), nullptr, act[0].as<__bf16>(),
                                   gA.p, s);
    wgrad(0, H, Wd, x0.as<__bf16>(), 8, gA.as<__bf16>(), 32, 4, 32, s);
    double h[2];
    HH_HIP(hipMemcpyAsync(h, nr2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HH_HIP(hipStreamSynchronize(s));
    return h[0] > 0.0 ? h[1] / h[0] : 0.0;
}

void CnnImpl::adam_step(double lr, hipStream_t s) {
    ++adam_t;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)adam_t), c2 = 1.0f - std::pow(b2, (float)adam_t);
    const int n = 2 * nparam;
    hipLaunchKernelGGL(adam_kernel, dim3(g1(n, 256)), dim3(256), 0, s, n, theta.as<float>(), adam_m.as<float>(),
                       adam_v.as<float>(), grad.as<float>(), (float)lr, b1, b2, 1e-8f, c1, c2);
    repack(s);
}

}  // namespace hh
