// Control variate of the nested walks: combination of the walk traces with
// the network values, record export, and training-sample gathering.
//
// For any twice differentiable N, the ball's mean-value identity of the
// screened operator (Poisson-kernel mean of N on the sphere plus the
// Green's-function integral of -Lap N + sigma N over the ball, Sec. 3.3)
// applied at every step of a walk of Algorithm 1 makes
//   C = N(x_0) - sum_{source steps j} |B_j| G_j (-Lap N + sigma N)(y_j)
//       - [alive] N(x_stop)
// a zero-mean quantity under the walk's own stopping rules.  The sum over
// the L source steps is estimated by the reservoir-chosen step, weighted by
// L.  The nested estimate of u(xoff) becomes
//   N(xoff) + [run] (uhat - corr) / q,   corr = mean over the K nested walks
//   of L |B| G (-Lap N + sigma N)(y) + [alive] N(x_stop),
// which has the mean of uhat for any N and any q in (0, 1].
#pragma once
#include "aux_kernels.hpp"

namespace dwos {

template <class T>
struct CvCombineArgs {
    const int32_t* run;
    const int32_t* La;
    const T* rho;
    const T* d;
    const float* Noff;
    const float* Nstop;
    const float* Ny;
    const float* Ly;
    T* uoff;             // in: plain nested mean; out: control-variate estimate
    T* target;           // out: N(xoff) + uhat - corr (run == 1), NaN otherwise
    T* uoff_plain;       // optional copy of the plain nested mean
    int64_t nwalks;
    int32_t K;
    T kappa, sigma, inv_q;
};

template <class T, int D>
__global__ void cv_combine_kernel(CvCombineArgs<T> a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nwalks) return;
    const int run = a.run[i];
    const T uplain = a.uoff[i];
    if (a.uoff_plain) a.uoff_plain[i] = uplain;
    if (run < 0) {
        a.target[i] = T(NAN);
        return;
    }
    const T Noff = T(a.Noff[i]);
    if (run == 0) {
        a.uoff[i] = Noff;
        a.target[i] = T(NAN);
        return;
    }
    T corr = T(0);
    for (int j = 0; j < a.K; ++j) {
        const size_t q = (size_t)i * a.K + j;
        const int32_t La = a.La[q];
        const int32_t L = La >> 1;
        if (L > 0) {
            const T fN = -T(a.Ly[q]) + a.sigma * T(a.Ny[q]);
            corr += T(L) * green_ball_t<D, T>(a.kappa, a.rho[q], a.d[q]) * fN;
        }
        if (La & 1) corr += T(a.Nstop[q]);
    }
    corr /= T(a.K);
    a.target[i] = Noff + uplain - corr;
    a.uoff[i] = Noff + (uplain - corr) * a.inv_q;
}

// Export in the layout walk[9] = {run, xoff[3], uoff plain, uoff cv, target,
// u, primitive} and nested[10] = {L, alive, xstop[3], y[3], rho, d}.
template <class T, int D>
__global__ void cv_export_kernel(const int32_t* run, const T* xoff, const T* uplain, const T* ucv,
                                 const T* target, const T* u, const int32_t* prim, const int32_t* La,
                                 const T* stop, const T* y, const T* rho, const T* d, int64_t nwalks,
                                 int32_t K, int64_t off, double* walk, double* nested) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nwalks) return;
    double* w = walk + (size_t)(off + i) * 9;
    const int r = run[i];
    w[0] = r;
    for (int c = 0; c < 3; ++c) w[1 + c] = (r >= 0 && c < D) ? double(xoff[(size_t)i * D + c]) : 0.0;
    w[4] = r >= 0 ? double(uplain[i]) : 0.0;
    w[5] = r >= 0 ? double(ucv[i]) : 0.0;
    w[6] = r == 1 ? double(target[i]) : 0.0;
    w[7] = double(u[i]);
    w[8] = prim[i] >= 0 ? double(prim[i] >> 1) : -1.0;
    for (int j = 0; j < K; ++j) {
        const size_t q = (size_t)i * K + j;
        double* o = nested + (size_t)((off + i) * K + j) * 10;
        for (int c = 0; c < 10; ++c) o[c] = 0.0;
        if (r != 1) continue;
        o[0] = double(La[q] >> 1);
        o[1] = double(La[q] & 1);
        for (int c = 0; c < D; ++c) {
            o[2 + c] = double(stop[q * D + c]);
            o[5 + c] = double(y[q * D + c]);
        }
        o[8] = double(rho[q]);
        o[9] = double(d[q]);
    }
}

// Training batch from the last differential walks: sample j draws a walk i
// uniformly (Philox counter (j, step, 0, 0xC0000000), key seed) and yields
// two rows -- (xoff_i, target_i) at j if its nested walks ran, and
// (xbar_i, g_i) at batch + j if it reached the boundary -- each with weight
// 1 / batch (0 for a row that does not exist).
template <class T, int D>
__global__ void cv_gather_kernel(const int32_t* run, const T* xoff, const T* xbar, const T* g,
                                 const T* target, int64_t nwalks, int32_t batch, uint32_t step,
                                 uint32_t key0, uint32_t key1, float* X, float* tgt, float* w) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch) return;
    const u4 r = philox10(u4{(uint32_t)j, step, 0u, 0xC0000000u}, key0, key1);
    const int64_t i = (int64_t)(((unsigned long long)r.x * (unsigned long long)nwalks) >> 32);
    const int ri = run[i];
    const float wt = 1.0f / (float)batch;
    const bool off_ok = ri == 1 && isfinite(target[i]);
    for (int c = 0; c < D; ++c) {
        X[(size_t)j * D + c] = off_ok ? float(xoff[(size_t)i * D + c]) : 0.f;
        X[(size_t)(batch + j) * D + c] = ri >= 0 ? float(xbar[(size_t)i * D + c]) : 0.f;
    }
    tgt[j] = off_ok ? float(target[i]) : 0.f;
    w[j] = off_ok ? wt : 0.f;
    tgt[batch + j] = ri >= 0 ? float(g[i]) : 0.f;
    w[batch + j] = ri >= 0 ? wt : 0.f;
}

}  // namespace dwos
