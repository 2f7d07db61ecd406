// Control-variate network on the gfx950 matrix cores: packing of the FP32
// master weights into split-BF16 MFMA fragments, evaluation with value /
// gradient / Laplacian channels, the squared-loss gradient and Adam.
//
// Fragment layout (v_mfma_f32_16x16x32_bf16, 64 lanes, lane = 16 g + i):
//   A (16 x 32, weights):      lane holds row i, K slots (g, e), e = 0..7
//   B (32 x 16, activations):  lane holds column i, K slots (g, e)
//   D (16 x 16, FP32):         lane holds rows 4 g + r, column i, r = 0..3
// The K slot (kc, g, e) of K chunk kc is mapped to the hidden unit
//   16 (2 kc + e / 4) + 4 g + e % 4,
// which is exactly the set of units a lane holds in D after a layer (tile
// t = 2 kc + e / 4, row 4 g + e % 4).  With the weights packed in that order,
// a layer's output fragments become the next layer's B operands in the same
// lane: no cross-lane exchange and no LDS round trip between layers.  Points
// are the 16 columns of a tile; each wave streams 16-point tiles.
#include "mlp.hpp"

#include <cmath>
#include <cstring>
#include <new>
#include <string>

namespace dwos_mlp_k {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int slot_unit(int kc, int g, int e) {
    return 16 * (2 * kc + (e >> 2)) + 4 * g + (e & 3);
}

__device__ inline f32x4 mma3(const bf16x8& ah, const bf16x8& al, const bf16x8& bh, const bf16x8& bl,
                             f32x4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    return acc;
}

// x = hi + lo with hi = bf16(x) (round to nearest even) and lo = bf16(x - hi)
__device__ inline void split(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
}

// ---------------------------------------------------------------------------
// packing: one thread per (direction, layer, fragment, lane)
//   direction 0: A = W_l      (rows = output units, K = input slots)
//   direction 1: A = W_l^T    (rows = input units,  K = output-unit slots)
// ---------------------------------------------------------------------------
__global__ void pack_kernel(const float* __restrict__ theta, u32x4* __restrict__ packed) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * kLayers * kFrags * 64) return;
    const int lane = idx & 63, f = (idx >> 6) & 7, l = (idx >> 9) & 3, dir = idx >> 11;
    const int mt = f >> 1, kc = f & 1, i = lane & 15, g = lane >> 4;
    const float* W = theta + (size_t)l * kLayerSize;
    bf16x8 hi, lo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = slot_unit(kc, g, e);
        const float w = dir == 0 ? W[(16 * mt + i) * kWidth + k] : W[k * kWidth + 16 * mt + i];
        __bf16 h, o;
        split(w, h, o);
        hi[e] = h;
        lo[e] = o;
    }
    const size_t at = ((((size_t)dir * kLayers + l) * kFrags + f) * 64 + lane) * 2;
    packed[at] = __builtin_bit_cast(u32x4, hi);
    packed[at + 1] = __builtin_bit_cast(u32x4, lo);
}

// Input features of the lane's 16 slots: feature 16 t + 4 g + r for tile t,
// row r.  ch 0 = value, ch 1..D = d/dx_c, ch D+1 = Laplacian.
template <int D, int NC>
__device__ inline void features(const float* __restrict__ B, int F, const float x[D], int g,
                                float act[NC][4][4]) {
    constexpr float kTwoPi = 6.28318530717958647692f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int f = 16 * t + 4 * g + r;
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) act[ch][t][r] = 0.f;
            if (f < 2 * F) {
                const int j = f < F ? f : f - F;
                float th = 0.f, bb = 0.f, b[D];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    b[c] = B[j * D + c];
                    th += b[c] * x[c];
                    bb += b[c] * b[c];
                }
                float sn, cs;
                sincosf(kTwoPi * th, &sn, &cs);
                const float v = f < F ? sn : cs;     // value
                const float dv = f < F ? cs : -sn;   // derivative of the value in th
                act[0][t][r] = v;
                if constexpr (NC > 1) {
#pragma unroll
                    for (int c = 0; c < D; ++c) act[1 + c][t][r] = kTwoPi * b[c] * dv;
                    act[D + 1][t][r] = -(kTwoPi * kTwoPi) * bb * v;
                }
            } else if (f < 2 * F + D) {
                const int c0 = f - 2 * F;
                act[0][t][r] = x[c0];
                if constexpr (NC > 1) {
#pragma unroll
                    for (int c = 0; c < D; ++c) act[1 + c][t][r] = c == c0 ? 1.f : 0.f;
                }
            }
        }
    }
}

// B operands (hi, lo) of the two K chunks from a lane's 16 activations
template <int NC>
__device__ inline void to_operands(const float act[NC][4][4], bf16x8 bh[NC][2], bf16x8 bl[NC][2]) {
#pragma unroll
    for (int ch = 0; ch < NC; ++ch)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                __bf16 h, o;
                split(act[ch][t][r], h, o);
                bh[ch][t >> 1][((t & 1) << 2) | r] = h;
                bl[ch][t >> 1][((t & 1) << 2) | r] = o;
            }
}

// acc[ch][mt] = (W packed at w) x B for every channel
template <int NC>
__device__ inline void layer_product(const u32x4* w, int lane, const bf16x8 bh[NC][2],
                                     const bf16x8 bl[NC][2], f32x4 acc[NC][4]) {
#pragma unroll
    for (int ch = 0; ch < NC; ++ch)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[ch][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) {
            const int fr = (mt * 2 + kc) * 64 + lane;
            const bf16x8 ah = __builtin_bit_cast(bf16x8, w[2 * fr]);
            const bf16x8 al = __builtin_bit_cast(bf16x8, w[2 * fr + 1]);
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) acc[ch][mt] = mma3(ah, al, bh[ch][kc], bl[ch][kc], acc[ch][mt]);
        }
    }
}

template <class TX>
struct EvalArgs {
    const u32x4* packed;
    const float* theta;
    const float* B;
    int F;
    const TX* X;
    int64_t n;
    const int32_t* mask;
    int mask_div, mask_min;
    float* N;
    float* G;
    float* L;
};

// ---------------------------------------------------------------------------
// evaluation: N, and with LAP the gradient and Laplacian channels, carried
// through each layer by the chain rule (h = tanh z: h' = 1 - h^2,
// h'' = -2 h (1 - h^2)).  The forward weights (64 KB) are staged in LDS.
// ---------------------------------------------------------------------------
template <int D, bool LAP, class TX>
__global__ void __launch_bounds__(256) eval_kernel(EvalArgs<TX> a) {
    constexpr int NC = LAP ? D + 2 : 1;
    __shared__ u32x4 s_w[kPackDirU4];
    for (int i = threadIdx.x; i < kPackDirU4; i += blockDim.x) s_w[i] = a.packed[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int waves = blockDim.x >> 6;
    const float* w5 = a.theta + (size_t)kLayers * kLayerSize;
    for (int64_t tile = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); tile * 16 < a.n;
         tile += (int64_t)gridDim.x * waves) {
        const int64_t p = tile * 16 + col;
        bool valid = p < a.n;
        if (valid && a.mask) valid = a.mask[p / a.mask_div] >= a.mask_min;
        if (__ballot(valid) == 0ull) continue;   // wave-uniform
        float x[D];
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = valid ? (float)a.X[p * D + c] : 0.f;
        float act[NC][4][4];
        features<D, NC>(a.B, a.F, x, g, act);
        bf16x8 bh[NC][2], bl[NC][2];
        f32x4 acc[NC][4];
#pragma unroll 1
        for (int l = 0; l < kLayers; ++l) {
            to_operands<NC>(act, bh, bl);
            layer_product<NC>(s_w + (size_t)l * kPackLayerU4, lane, bh, bl, acc);
            const float* bias = a.theta + (size_t)l * kLayerSize + kWidth * kWidth;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float z = acc[0][mt][r] + bias[16 * mt + 4 * g + r];
                    const float h = tanhf(z), s = 1.f - h * h;
                    act[0][mt][r] = h;
                    if constexpr (LAP) {
                        float zz = 0.f;
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            const float zg = acc[1 + c][mt][r];
                            zz += zg * zg;
                            act[1 + c][mt][r] = s * zg;
                        }
                        act[D + 1][mt][r] = s * acc[D + 1][mt][r] - 2.f * h * s * zz;
                    }
                }
        }
        float o[NC];
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) o[ch] = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float w = w5[16 * t + 4 * g + r];
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) o[ch] += w * act[ch][t][r];
            }
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) {
            o[ch] += __shfl_xor(o[ch], 16);
            o[ch] += __shfl_xor(o[ch], 32);
        }
        if (g == 0 && valid) {
            a.N[p] = o[0] + w5[kWidth];
            if constexpr (LAP) {
                if (a.G)
#pragma unroll
                    for (int c = 0; c < D; ++c) a.G[p * D + c] = o[1 + c];
                if (a.L) a.L[p] = o[D + 1];
            }
        }
    }
}

// sum over the 16 columns (lanes with the same g)
__device__ inline float col_sum(float v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

struct TrainArgs {
    const u32x4* packed;
    const float* theta;
    const float* B;
    int F;
    const float* X;
    const float* T;
    const float* w;
    int64_t n;
    float* grad;
    float* loss;
    __bf16* ws;       // [layer][tile of 16 points][dh, dl, ah, al][64 units][16 points]
    int64_t pad;      // batch rounded up to 32 points
};

// ---------------------------------------------------------------------------
// squared-loss backward, part 1: forward, output-layer and bias gradients,
// back-propagated deltas; writes each layer's delta and input activation
// (hi/lo BF16, unit-major) for the weight-gradient products.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) loss_grad_kernel(TrainArgs a) {
    const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int waves = blockDim.x >> 6;
    const float* w5 = a.theta + (size_t)kLayers * kLayerSize;
    const u32x4* fwd = a.packed;
    const u32x4* bwd = a.packed + kPackDirU4;
    float loss_acc = 0.f;
    for (int64_t tile = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); tile * 16 < a.pad;
         tile += (int64_t)gridDim.x * waves) {
        const int64_t p = tile * 16 + col;
        const bool valid = p < a.n;
        float x[D];
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = valid ? a.X[p * D + c] : 0.f;
        const float om = valid ? (a.w ? a.w[p] : 1.f) : 0.f;
        const float tg = valid ? a.T[p] : 0.f;
        float cur[1][4][4];
        features<D, 1>(a.B, a.F, x, g, cur);
        bf16x8 bh[1][2], bl[1][2];
        f32x4 acc[1][4];
        // forward; each layer's input activation goes to the workspace (hi,
        // lo), where the weight-gradient product and the backward pass read it
        const int64_t ntiles = a.pad / 16;
        // this lane's slot in a tile block: unit 4 g (+ 16 t + r), point col
        const int lane_off = (4 * g) * 16 + col;
#pragma unroll 1
        for (int l = 0; l < kLayers; ++l) {
            __bf16* base = a.ws + ((size_t)l * ntiles + tile) * 4 * kWidth * 16 + lane_off;
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int uo = (16 * t + r) * 16;
                    __bf16 h, lo;
                    split(cur[0][t][r], h, lo);
                    base[2 * kWidth * 16 + uo] = h;
                    base[3 * kWidth * 16 + uo] = lo;
                }
            to_operands<1>(cur, bh, bl);
            layer_product<1>(fwd + (size_t)l * kPackLayerU4, lane, bh, bl, acc);
            const float* bias = a.theta + (size_t)l * kLayerSize + kWidth * kWidth;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) cur[0][mt][r] = tanhf(acc[0][mt][r] + bias[16 * mt + 4 * g + r]);
        }
        float o = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) o += w5[16 * t + 4 * g + r] * cur[0][t][r];
        o += __shfl_xor(o, 16);
        o += __shfl_xor(o, 32);
        const float N = o + w5[kWidth];
        const float res = om * (N - tg);
        if (g == 0) loss_acc += 0.5f * om * (N - tg) * (N - tg);
        // output layer
        float delta[1][4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int u = 16 * t + 4 * g + r;
                const float h = cur[0][t][r];
                const float gw = col_sum(res * h);
                if (col == 0) atomicAdd(&a.grad[(size_t)kLayers * kLayerSize + u], gw);
                delta[0][t][r] = res * w5[u] * (1.f - h * h);
            }
        {
            const float gb = col_sum(g == 0 ? res : 0.f);
            if (lane == 0) atomicAdd(&a.grad[(size_t)kLayers * kLayerSize + kWidth], gb);
        }
#pragma unroll 1
        for (int l = kLayers - 1; l >= 0; --l) {
            __bf16* base = a.ws + ((size_t)l * ntiles + tile) * 4 * kWidth * 16 + lane_off;
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int u = 16 * t + 4 * g + r;
                    const float gb = col_sum(delta[0][t][r]);
                    if (col == 0) atomicAdd(&a.grad[(size_t)l * kLayerSize + kWidth * kWidth + u], gb);
                    const int uo = (16 * t + r) * 16;
                    __bf16 h, lo;
                    split(delta[0][t][r], h, lo);
                    base[uo] = h;
                    base[kWidth * 16 + uo] = lo;
                }
            if (l == 0) break;
            // delta_{l-1} = (W_l^T delta_l) (1 - a_l^2), a_l read back (hi + lo)
            to_operands<1>(delta, bh, bl);
            layer_product<1>(bwd + (size_t)l * kPackLayerU4, lane, bh, bl, acc);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int uo = (16 * mt + r) * 16;
                    const float h = (float)base[2 * kWidth * 16 + uo] + (float)base[3 * kWidth * 16 + uo];
                    delta[0][mt][r] = acc[0][mt][r] * (1.f - h * h);
                }
        }
    }
    // loss: wave sum, one atomic per wave
    loss_acc += __shfl_xor(loss_acc, 1);
    loss_acc += __shfl_xor(loss_acc, 2);
    loss_acc += __shfl_xor(loss_acc, 4);
    loss_acc += __shfl_xor(loss_acc, 8);
    loss_acc += __shfl_xor(loss_acc, 16);
    loss_acc += __shfl_xor(loss_acc, 32);
    if (lane == 0 && a.loss) atomicAdd(a.loss, loss_acc);
}

// ---------------------------------------------------------------------------
// squared-loss backward, part 2: dW_l = delta_l a_l^T over the batch, one
// 16x16 output tile per wave and a slice of the batch per blockIdx.y
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) wgrad_kernel(const __bf16* __restrict__ ws, int64_t pad,
                                                   int64_t chunks_per_split, float* __restrict__ grad) {
    const int lane = threadIdx.x, i = lane & 15, g = lane >> 4;
    const int l = blockIdx.x >> 4, mo = (blockIdx.x >> 2) & 3, mi = blockIdx.x & 3;
    const int64_t ntiles = pad / 16, n_chunks = pad / 32;
    const int64_t c0 = (int64_t)blockIdx.y * chunks_per_split;
    const int64_t c1 = c0 + chunks_per_split < n_chunks ? c0 + chunks_per_split : n_chunks;
    if (c0 >= c1) return;
    // K slot (g, e) of chunk ck is point 32 ck + 8 g + e: tile 2 ck + g / 2,
    // column 8 (g & 1) + e
    const int a_off = (16 * mo + i) * 16 + 8 * (g & 1);
    const int b_off = (16 * mi + i) * 16 + 8 * (g & 1);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t ck = c0; ck < c1; ++ck) {
        const __bf16* blk = ws + ((size_t)l * ntiles + 2 * ck + (g >> 1)) * 4 * kWidth * 16;
        const bf16x8 Ah = *reinterpret_cast<const bf16x8*>(blk + a_off);
        const bf16x8 Al = *reinterpret_cast<const bf16x8*>(blk + kWidth * 16 + a_off);
        const bf16x8 Bh = *reinterpret_cast<const bf16x8*>(blk + 2 * kWidth * 16 + b_off);
        const bf16x8 Bl = *reinterpret_cast<const bf16x8*>(blk + 3 * kWidth * 16 + b_off);
        acc = mma3(Ah, Al, Bh, Bl, acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        atomicAdd(&grad[(size_t)l * kLayerSize + (16 * mo + 4 * g + r) * kWidth + 16 * mi + i], acc[r]);
}

struct VjpArgs {
    const u32x4* packed;
    const float* theta;
    const float* B;
    int F;
    const float* X;
    const float* Nbar;
    const float* Lbar;
    int64_t n;
    int64_t pad;
    float* grad;
    __bf16* ws;       // [layer][virtual tile = tile * NC + channel][zh, zl, ah, al][64][16]
    float* zs;        // [layer][tile][channel][64][16] pre-activations
};

// ---------------------------------------------------------------------------
// grad += d/dtheta sum_i (Nbar_i N(x_i) + Lbar_i Lap N(x_i)), part 1.  The
// forward pass carries the value, gradient and Laplacian channels (as in
// eval_kernel) and keeps each layer's pre-activations; the backward pass
// turns the output adjoints into pre-activation adjoints per layer
// (h = tanh z, s = 1 - h^2, Q = sum_c z_c^2):
//   zbar_L = s abar_L,  zbar_c = s abar_c - 4 h s z_c abar_L,
//   zbar = s abar - 2 h s sum_c z_c abar_c - (2 h s z_L + 2 s (s - 2 h^2) Q) abar_L
// and sends every channel back through W^T on the matrix cores.  Each
// layer's channel inputs and pre-activation adjoints go to the workspace for
// the weight-gradient products, which contract over points and channels.
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(256) vjp_kernel(VjpArgs a) {
    constexpr int NC = D + 2;
    const int lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int waves = blockDim.x >> 6;
    const float* w5 = a.theta + (size_t)kLayers * kLayerSize;
    const u32x4* fwd = a.packed;
    const u32x4* bwd = a.packed + kPackDirU4;
    const int64_t ntiles = a.pad / 16;
    const int lane_off = (4 * g) * 16 + col;
    for (int64_t tile = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); tile < ntiles;
         tile += (int64_t)gridDim.x * waves) {
        const int64_t p = tile * 16 + col;
        const bool valid = p < a.n;
        float x[D];
#pragma unroll
        for (int c = 0; c < D; ++c) x[c] = valid ? a.X[p * D + c] : 0.f;
        const float nb = valid ? a.Nbar[p] : 0.f;
        const float lb = (valid && a.Lbar) ? a.Lbar[p] : 0.f;
        float act[NC][4][4];
        features<D, NC>(a.B, a.F, x, g, act);
        bf16x8 bh[NC][2], bl[NC][2];
        f32x4 acc[NC][4];
#pragma unroll 1
        for (int l = 0; l < kLayers; ++l) {
            __bf16* wsl = a.ws + ((size_t)l * ntiles + tile) * NC * 4 * kWidth * 16 + lane_off;
            float* zsl = a.zs + (((size_t)l * ntiles + tile) * NC) * kWidth * 16 + lane_off;
#pragma unroll
            for (int ch = 0; ch < NC; ++ch)
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        __bf16 h, lo;
                        split(act[ch][t][r], h, lo);
                        const int uo = ch * 4 * kWidth * 16 + (16 * t + r) * 16;
                        wsl[2 * kWidth * 16 + uo] = h;
                        wsl[3 * kWidth * 16 + uo] = lo;
                    }
            to_operands<NC>(act, bh, bl);
            layer_product<NC>(fwd + (size_t)l * kPackLayerU4, lane, bh, bl, acc);
            const float* bias = a.theta + (size_t)l * kLayerSize + kWidth * kWidth;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float z = acc[0][mt][r] + bias[16 * mt + 4 * g + r];
                    const int uo = (16 * mt + r) * 16;
                    zsl[uo] = z;
#pragma unroll
                    for (int ch = 1; ch < NC; ++ch) zsl[ch * kWidth * 16 + uo] = acc[ch][mt][r];
                    const float h = tanhf(z), s = 1.f - h * h;
                    float zz = 0.f;
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        const float zg = acc[1 + c][mt][r];
                        zz += zg * zg;
                        act[1 + c][mt][r] = s * zg;
                    }
                    act[0][mt][r] = h;
                    act[D + 1][mt][r] = s * acc[D + 1][mt][r] - 2.f * h * s * zz;
                }
        }
        // output layer: N = w5 . a_v + b5, Lap N = w5 . a_L
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int u = 16 * t + 4 * g + r;
                const float gw = col_sum(nb * act[0][t][r] + lb * act[D + 1][t][r]);
                if (col == 0) atomicAdd(&a.grad[(size_t)kLayers * kLayerSize + u], gw);
#pragma unroll
                for (int ch = 0; ch < NC; ++ch) act[ch][t][r] = 0.f;   // becomes abar
                act[0][t][r] = nb * w5[u];
                act[D + 1][t][r] = lb * w5[u];
            }
        {
            const float gb = col_sum(g == 0 ? nb : 0.f);
            if (lane == 0) atomicAdd(&a.grad[(size_t)kLayers * kLayerSize + kWidth], gb);
        }
        // act now holds the adjoints abar of the current layer's outputs
#pragma unroll 1
        for (int l = kLayers - 1; l >= 0; --l) {
            __bf16* wsl = a.ws + ((size_t)l * ntiles + tile) * NC * 4 * kWidth * 16 + lane_off;
            const float* zsl = a.zs + (((size_t)l * ntiles + tile) * NC) * kWidth * 16 + lane_off;
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int uo = (16 * t + r) * 16;
                    const float z = zsl[uo];
                    const float zL = zsl[(D + 1) * kWidth * 16 + uo];
                    const float h = tanhf(z), s = 1.f - h * h;
                    const float aL = act[D + 1][t][r];
                    float Q = 0.f, za = 0.f;
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        const float zc = zsl[(1 + c) * kWidth * 16 + uo];
                        Q += zc * zc;
                        za += zc * act[1 + c][t][r];
                        act[1 + c][t][r] = s * act[1 + c][t][r] - 4.f * h * s * zc * aL;
                    }
                    act[0][t][r] = s * act[0][t][r] - 2.f * h * s * za -
                                   (2.f * h * s * zL + 2.f * s * (s - 2.f * h * h) * Q) * aL;
                    act[D + 1][t][r] = s * aL;
                    const int u = 16 * t + 4 * g + r;
                    const float gb = col_sum(act[0][t][r]);
                    if (col == 0) atomicAdd(&a.grad[(size_t)l * kLayerSize + kWidth * kWidth + u], gb);
#pragma unroll
                    for (int ch = 0; ch < NC; ++ch) {
                        __bf16 hh, lo;
                        split(act[ch][t][r], hh, lo);
                        const int o = ch * 4 * kWidth * 16 + uo;
                        wsl[o] = hh;
                        wsl[kWidth * 16 + o] = lo;
                    }
                }
            if (l == 0) break;
            to_operands<NC>(act, bh, bl);
            layer_product<NC>(bwd + (size_t)l * kPackLayerU4, lane, bh, bl, acc);
#pragma unroll
            for (int ch = 0; ch < NC; ++ch)
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) act[ch][mt][r] = acc[ch][mt][r];
        }
    }
}

__global__ void zero_kernel(float* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// Adam (Kingma and Ba, Algorithm 1) on the FP32 master parameters
__global__ void adam_kernel(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace dwos_mlp_k

namespace dwos_host {

using namespace dwos_mlp_k;

hipError_t pack(dwos_mlp* m, hipStream_t s) {
    hipLaunchKernelGGL(pack_kernel, dim3(blocks_for(2 * kLayers * kFrags * 64, 256)), dim3(256), 0, s,
                       m->theta.as<float>(), m->packed.as<u32x4>());
    return hipGetLastError();
}

hipError_t zero(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

unsigned grid_for_tiles(int64_t n, int max_blocks) {
    const int64_t tiles = (n + 15) / 16;
    int64_t b = (tiles + 3) / 4;
    if (b > max_blocks) b = max_blocks;
    return (unsigned)(b < 1 ? 1 : b);
}

template <class TX>
hipError_t mlp_eval_launch(const dwos_mlp* m, hipStream_t s, const TX* X, int64_t n,
                           const int32_t* mask, int mask_div, int mask_min, float* N, float* G,
                           float* L) {
    if (n <= 0) return hipSuccess;
    EvalArgs<TX> a{m->packed.as<u32x4>(), m->theta.as<float>(), m->B.as<float>(), m->F, X, n,
                   mask, mask_div < 1 ? 1 : mask_div, mask_min, N, G, L};
    const bool lap = G || L;
    const dim3 grid(grid_for_tiles(n, 2048)), block(256);
    if (m->dim == 2) {
        if (lap) hipLaunchKernelGGL((eval_kernel<2, true, TX>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((eval_kernel<2, false, TX>), grid, block, 0, s, a);
    } else {
        if (lap) hipLaunchKernelGGL((eval_kernel<3, true, TX>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((eval_kernel<3, false, TX>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

template hipError_t mlp_eval_launch<float>(const dwos_mlp*, hipStream_t, const float*, int64_t,
                                           const int32_t*, int, int, float*, float*, float*);
template hipError_t mlp_eval_launch<double>(const dwos_mlp*, hipStream_t, const double*, int64_t,
                                            const int32_t*, int, int, float*, float*, float*);

hipError_t mlp_loss_grad_launch(dwos_mlp* m, hipStream_t s, const float* X, const float* T,
                                const float* w, int64_t n, float* loss) {
    hipError_t e;
    if ((e = zero(m->grad.as<float>(), kThetaSize, s)) != hipSuccess) return e;
    if (loss && (e = zero(loss, 1, s)) != hipSuccess) return e;
    if (n <= 0) return hipSuccess;
    const int64_t pad = (n + 31) / 32 * 32;
    if ((e = m->ws.reserve((size_t)kLayers * 4 * kWidth * pad * sizeof(__bf16))) != hipSuccess) return e;
    m->ws_pad = pad;
    TrainArgs a{m->packed.as<u32x4>(), m->theta.as<float>(), m->B.as<float>(), m->F, X, T, w, n,
                m->grad.as<float>(), loss, m->ws.as<__bf16>(), pad};
    // the kernel walks every tile up to pad, so each workspace column is
    // written (padding points carry a zero delta)
    const dim3 grid(grid_for_tiles(pad, 1024)), block(256);
    if (m->dim == 2) hipLaunchKernelGGL(loss_grad_kernel<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(loss_grad_kernel<3>, grid, block, 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t chunks = pad / 32;
    int64_t splits = chunks < 128 ? chunks : 128;
    const int64_t per = (chunks + splits - 1) / splits;
    splits = (chunks + per - 1) / per;
    hipLaunchKernelGGL(wgrad_kernel, dim3(kLayers * 16, (unsigned)splits), dim3(64), 0, s,
                       m->ws.as<__bf16>(), pad, per, m->grad.as<float>());
    return hipGetLastError();
}

hipError_t mlp_vjp_launch(dwos_mlp* m, hipStream_t s, const float* X, const float* Nbar,
                          const float* Lbar, int64_t n) {
    hipError_t e;
    if ((e = zero(m->grad.as<float>(), kThetaSize, s)) != hipSuccess) return e;
    if (n <= 0) return hipSuccess;
    const int NC = m->dim + 2;
    const int64_t pad = (n + 31) / 32 * 32;
    if ((e = m->ws.reserve((size_t)kLayers * NC * 4 * kWidth * pad * sizeof(__bf16))) != hipSuccess) return e;
    if ((e = m->zs.reserve((size_t)kLayers * NC * kWidth * pad * sizeof(float))) != hipSuccess) return e;
    VjpArgs a{m->packed.as<u32x4>(), m->theta.as<float>(), m->B.as<float>(), m->F, X, Nbar, Lbar, n, pad,
              m->grad.as<float>(), m->ws.as<__bf16>(), m->zs.as<float>()};
    const dim3 grid(grid_for_tiles(pad, 1024)), block(256);
    if (m->dim == 2) hipLaunchKernelGGL(vjp_kernel<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(vjp_kernel<3>, grid, block, 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // weight gradients: contraction over the pad * NC (point, channel) pairs
    const int64_t padv = pad * NC;
    const int64_t chunks = padv / 32;
    int64_t splits = chunks < 128 ? chunks : 128;
    const int64_t per = (chunks + splits - 1) / splits;
    splits = (chunks + per - 1) / per;
    hipLaunchKernelGGL(wgrad_kernel, dim3(kLayers * 16, (unsigned)splits), dim3(64), 0, s,
                       m->ws.as<__bf16>(), padv, per, m->grad.as<float>());
    return hipGetLastError();
}

hipError_t mlp_adam_launch(dwos_mlp* m, hipStream_t s, float lr, float beta1, float beta2, float eps) {
    m->step += 1;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)m->step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)m->step));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(kThetaSize, 256)), dim3(256), 0, s,
                       m->theta.as<float>(), m->m.as<float>(), m->v.as<float>(), m->grad.as<float>(),
                       (int64_t)kThetaSize, lr, beta1, beta2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return pack(m, s);
}

}  // namespace dwos_host

// ===========================================================================
// C ABI (declared in include/dwos.h)
// ===========================================================================
using dwos_host::fail;

extern "C" {

int32_t dwos_mlp_theta_size(void) { return dwos_mlp_k::kThetaSize; }

dwos_status dwos_mlp_create(int32_t dim, int32_t F, const float* B, void* stream, dwos_mlp** out) {
    if (!out) return fail(DWOS_EINVAL, "mlp_create: NULL out");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(DWOS_EINVAL, "mlp_create: dim must be 2 or 3");
    if (F < 0 || 2 * F + dim > dwos_mlp_k::kWidth) return fail(DWOS_EINVAL, "mlp_create: need 0 <= 2F + dim <= 64");
    if (F > 0 && !B) return fail(DWOS_EINVAL, "mlp_create: NULL frequencies");
    for (int i = 0; i < F * dim; ++i)
        if (!std::isfinite(B[i])) return fail(DWOS_EINVAL, "mlp_create: non-finite frequency");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(DWOS_EDEVICE, "mlp_create: no GPU");
    auto m = new (std::nothrow) dwos_mlp();
    if (!m) return fail(DWOS_ENOMEM, "mlp_create: out of host memory");
    auto bail = [&](dwos_status st) { delete m; return st; };
    m->dim = dim;
    m->F = F;
    m->stream = static_cast<hipStream_t>(stream);
    if (hipGetDevice(&m->device) != hipSuccess) return bail(fail(DWOS_EDEVICE, "mlp_create: hipGetDevice"));
    using namespace dwos_mlp_k;
    const size_t tb = (size_t)kThetaSize * sizeof(float);
    if (m->theta.reserve(tb) || m->m.reserve(tb) || m->v.reserve(tb) || m->grad.reserve(tb) ||
        m->B.reserve(std::max<size_t>(1, (size_t)F * dim) * sizeof(float)) ||
        m->packed.reserve((size_t)kPackU4 * 16) || m->loss.reserve(sizeof(float)))
        return bail(fail(DWOS_ENOMEM, "mlp_create: device allocation failed"));
    hipStream_t s = m->stream;
    hipError_t e = hipSuccess;
    if (F > 0) e = hipMemcpyAsync(m->B.ptr, B, (size_t)F * dim * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = dwos_host::zero(m->theta.as<float>(), kThetaSize, s);
    if (e == hipSuccess) e = dwos_host::zero(m->m.as<float>(), kThetaSize, s);
    if (e == hipSuccess) e = dwos_host::zero(m->v.as<float>(), kThetaSize, s);
    if (e == hipSuccess) e = dwos_host::pack(m, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(fail(DWOS_EDEVICE, std::string("mlp_create: ") + hipGetErrorString(e)));
    *out = m;
    return DWOS_OK;
}

void dwos_mlp_destroy(dwos_mlp* m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipStreamSynchronize(m->stream);
    delete m;
}

dwos_status dwos_mlp_set_params(dwos_mlp* m, const float* theta) {
    if (!m || !theta) return fail(DWOS_EINVAL, "mlp_set_params: NULL argument");
    using namespace dwos_mlp_k;
    HIP_OK(hipSetDevice(m->device));
    hipStream_t s = m->stream;
    HIP_OK(hipMemcpyAsync(m->theta.ptr, theta, (size_t)kThetaSize * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIP_OK(dwos_host::zero(m->m.as<float>(), kThetaSize, s));
    HIP_OK(dwos_host::zero(m->v.as<float>(), kThetaSize, s));
    m->step = 0;
    HIP_OK(dwos_host::pack(m, s));
    return DWOS_OK;
}

dwos_status dwos_mlp_get_params(dwos_mlp* m, float* theta) {
    if (!m || !theta) return fail(DWOS_EINVAL, "mlp_get_params: NULL argument");
    HIP_OK(hipSetDevice(m->device));
    HIP_OK(hipMemcpyAsync(theta, m->theta.ptr, (size_t)dwos_mlp_k::kThetaSize * sizeof(float),
                          hipMemcpyDeviceToDevice, m->stream));
    return DWOS_OK;
}

dwos_status dwos_mlp_eval(dwos_mlp* m, const float* X, int64_t n, float* N, float* grad, float* lap) {
    if (!m) return fail(DWOS_EINVAL, "mlp_eval: NULL network");
    if (n < 0 || (n > 0 && (!X || !N))) return fail(DWOS_EINVAL, "mlp_eval: bad arguments");
    HIP_OK(hipSetDevice(m->device));
    HIP_OK(dwos_host::mlp_eval_launch<float>(m, m->stream, X, n, nullptr, 1, 0, N, grad, lap));
    return DWOS_OK;
}

dwos_status dwos_mlp_loss_grad(dwos_mlp* m, const float* X, const float* T, const float* w, int64_t n,
                               float* loss, float* grad) {
    if (!m) return fail(DWOS_EINVAL, "mlp_loss_grad: NULL network");
    if (n < 0 || (n > 0 && (!X || !T))) return fail(DWOS_EINVAL, "mlp_loss_grad: bad arguments");
    HIP_OK(hipSetDevice(m->device));
    HIP_OK(dwos_host::mlp_loss_grad_launch(m, m->stream, X, T, w, n, loss));
    if (grad)
        HIP_OK(hipMemcpyAsync(grad, m->grad.ptr, (size_t)dwos_mlp_k::kThetaSize * sizeof(float),
                              hipMemcpyDeviceToDevice, m->stream));
    return DWOS_OK;
}

dwos_status dwos_mlp_vjp(dwos_mlp* m, const float* X, const float* Nbar, const float* Lbar, int64_t n,
                         float* grad) {
    if (!m) return fail(DWOS_EINVAL, "mlp_vjp: NULL network");
    if (n < 0 || (n > 0 && (!X || !Nbar))) return fail(DWOS_EINVAL, "mlp_vjp: bad arguments");
    HIP_OK(hipSetDevice(m->device));
    HIP_OK(dwos_host::mlp_vjp_launch(m, m->stream, X, Nbar, Lbar, n));
    if (grad)
        HIP_OK(hipMemcpyAsync(grad, m->grad.ptr, (size_t)dwos_mlp_k::kThetaSize * sizeof(float),
                              hipMemcpyDeviceToDevice, m->stream));
    return DWOS_OK;
}

dwos_status dwos_mlp_adam_step(dwos_mlp* m, float lr, float beta1, float beta2, float eps) {
    if (!m) return fail(DWOS_EINVAL, "mlp_adam_step: NULL network");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(DWOS_EINVAL, "mlp_adam_step: bad hyperparameters");
    HIP_OK(hipSetDevice(m->device));
    HIP_OK(dwos_host::mlp_adam_launch(m, m->stream, lr, beta1, beta2, eps));
    return DWOS_OK;
}

}  // extern "C"
