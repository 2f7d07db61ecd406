// Control-variate network: device state and the launchers the walk pipeline
// uses (the kernels live in mlp.hip).
//
// Network: Fourier features gamma(x) = [sin 2 pi B x, cos 2 pi B x, x, 0...]
// (64 inputs), four tanh layers of width 64, a linear scalar output.  The
// FP32 master parameters theta use the flat layout W_1, b_1, ..., W_4, b_4,
// w_5, b_5 with W_l row-major (row = output unit).
//
// The 64x64 products run on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16) with every FP32 operand split into a BF16 high
// part and a BF16 remainder; hi*hi + hi*lo + lo*hi keeps about 16 mantissa
// bits, so the value, gradient and Laplacian channels of the network agree
// with each other to ~1e-5 relative.  That agreement is what keeps the
// control variate unbiased.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "host_common.hpp"

namespace dwos_mlp_k {
constexpr int kWidth = 64;
constexpr int kLayers = 4;
constexpr int kLayerSize = kWidth * kWidth + kWidth;
constexpr int kThetaSize = kLayers * kLayerSize + kWidth + 1;
constexpr int kFrags = 8;                 // 4 row tiles x 2 K chunks of a 64x64 layer
// packed weights: [direction (forward W, backward W^T)][layer][frag][lane][hi, lo]
constexpr int kPackLayerU4 = kFrags * 64 * 2;
constexpr int kPackDirU4 = kLayers * kPackLayerU4;
constexpr int kPackU4 = 2 * kPackDirU4;
}  // namespace dwos_mlp_k

struct dwos_mlp {
    int dim = 0, F = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    dwos_host::DevBuf theta, m, v, grad, B, packed, loss;
    int64_t step = 0;
    // training workspace: per layer delta and input activations, hi/lo BF16,
    // unit-major with the batch padded to a multiple of 32
    dwos_host::DevBuf ws;
    int64_t ws_pad = 0;
    dwos_host::DevBuf zs;   // pre-activations of every layer and channel (vjp)
};

namespace dwos_host {

// N (and, if G or L is non-NULL, grad N [n x dim] and Lap N) at n points.
// A point p is evaluated only if mask is NULL or mask[p / mask_div] >=
// mask_min; other outputs are left untouched.
template <class TX>
hipError_t mlp_eval_launch(const dwos_mlp* m, hipStream_t s, const TX* X, int64_t n,
                           const int32_t* mask, int mask_div, int mask_min, float* N, float* G,
                           float* L);

// grad := d/dtheta sum_i 1/2 w_i (N(x_i) - t_i)^2 (w NULL: all 1), loss
// (device, may be NULL) := the loss.
hipError_t mlp_loss_grad_launch(dwos_mlp* m, hipStream_t s, const float* X, const float* T,
                                const float* w, int64_t n, float* loss);

// grad := d/dtheta sum_i (Nbar_i N(x_i) + Lbar_i Lap N(x_i)) (Lbar may be NULL).
hipError_t mlp_vjp_launch(dwos_mlp* m, hipStream_t s, const float* X, const float* Nbar,
                          const float* Lbar, int64_t n);

// One Adam step on theta with the current grad, then repack the BF16 weights.
hipError_t mlp_adam_launch(dwos_mlp* m, hipStream_t s, float lr, float beta1, float beta2,
                           float eps);

}  // namespace dwos_host
