// Learned fine-level smoother (complex 3x3 CNN on BF16 MFMA): host-side object.
#pragma once

#include <functional>

#include "hh_internal.h"

namespace hh {

constexpr int kChannels[5] = {2, 16, 16, 16, 1};   // complex channels per layer boundary

struct LayerInfo {
    int cin = 0, cout = 0;      // complex channels
    int cinp = 0, coutp = 0;    // padded real channels of the packed forward weights
    int dinp = 0, doutp = 0;    // data-gradient conv: input / output real channels
    int off = 0;                // offset of W in the parameter vector (complex entries)
    DevBuf wf, wd, bias;        // BF16 [9][coutp][cinp], BF16 [9][doutp][dinp], FP32 [coutp]
};

// y = b - M_beta x (conj = 0) or y = conj(M_beta) x (conj = 1), on the finest level
using MbetaFn = std::function<void(const cx<double>* x, const cx<double>* b, cx<double>* y, int conj)>;

struct CnnImpl {
    LayerInfo layers[4];
    int nparam = 0;             // complex parameters
    DevBuf theta, adam_m, adam_v, grad;   // FP32 (re, im) pairs
    int adam_t = 0;
    bool fused = true;          // smoother step: one fused kernel (else packing, one kernel per layer, update)
    int gH = -1, gW = -1;       // grid of the work buffers
    DevBuf x0, act[3], out, gA, gB, gOut, sbuf, rbuf, ybuf, scal, part, gfull;

    explicit CnnImpl(unsigned long long seed);
    void repack(hipStream_t s);
    void set_params(const float* host, int n);
    void ensure(int H, int W);
    void forward(int H, int W, hipStream_t s);   // per layer, activations kept (training)
    // smoother step on the grid: x (+)= omega D^-1 r + rms C(r/rms, c), rms = ||r|| / sqrt(N)
    template <class TV>
    void step(int H, int W, const cx<TV>* r, const float* feat, const cx<TV>* dinv, TV omega, cx<TV>* x,
              int accumulate, hipStream_t s);
    void wgrad(int l, int H, int W, const __bf16* X, int cinp, const __bf16* gY, int coutp, int ci_n, int co_n,
               hipStream_t s);
    double loss_grad(int H, int W, const cx<double>* r, const float* feat, const cx<double>* dinv, double omega,
                     const MbetaFn& mbeta, hipStream_t s);
    void adam_step(double lr, hipStream_t s);
};

}  // namespace hh
