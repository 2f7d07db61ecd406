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
// the source steps is estimated by one step J chosen with probability
// m_J / S (m_j = int_{B_j} G, the ball's Green's-function mass; S the walk's
// total) and one uniform point y of B_J.  The nested estimate of u(xoff) is
//   N(xoff) + [run] (uhat - corr) / q,   corr = mean over the K nested walks
//   of S |B| G(y) (-Lap N + sigma N)(y) / m_J + [alive] N(x_stop),
// which has the mean of uhat for any N and any q in (0, 1].  The control
// variate enters with a coefficient beta (uhat + beta C): any beta that does
// not depend on the current walks keeps the mean.  beta is the minimiser
// -E[uhat C] / E[C^2] estimated from the previous call's walks (E[C | xoff]
// = 0, so uncentred moments pooled over all offset points are unbiased
// estimates of the per-point ones), clamped to [0, 1]: a useless network
// falls back to the plain estimator.  The sums for beta run over the walks
// whose terminal primitive has a moving or parameterised vertex -- the only
// ones whose nested estimate enters a derivative.
#pragma once
#include "aux_kernels.hpp"

namespace dwos {

template <class T>
struct CvCombineArgs {
    const int32_t* run;
    const int32_t* prim;     // terminal code (orig * 2 + flip) of each walk
    const int32_t* pverts;   // primitive vertex indices (original order)
    const int32_t* vparam;   // per vertex: moves or carries a value parameter (NULL: all)
    const T* S;
    const int32_t* alive;
    const T* rho;
    const T* d;
    const float* Noff;
    const float* Nstop;
    const float* Ny;
    const float* Ly;
    T* uoff;             // in: plain nested mean; out: control-variate estimate
    T* target;           // out: N(xoff) + uhat - corr (run == 1), NaN otherwise
    T* uoff_plain;       // copy of the plain nested mean
    const double* beta;  // coefficient of the control variate
    double* stats;       // += {walks with run == 1, sum C^2, sum uhat C}
    int64_t nwalks;
    int32_t K;
    T kappa, sigma, inv_q;
};

__device__ inline double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <class T, int D>
__global__ void cv_combine_kernel(CvCombineArgs<T> a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s_n = 0.0, s_cc = 0.0, s_uc = 0.0;
    if (i < a.nwalks) {
        const int run = a.run[i];
        const T uplain = a.uoff[i];
        a.uoff_plain[i] = uplain;
        const T beta = T(*a.beta);
        if (run < 0) {
            a.target[i] = T(NAN);
        } else if (run == 0) {
            a.uoff[i] = beta * T(a.Noff[i]);
            a.target[i] = T(NAN);
        } else {
            const T Noff = T(a.Noff[i]);
            T corr = T(0);
            for (int j = 0; j < a.K; ++j) {
                const size_t q = (size_t)i * a.K + j;
                if (a.S[q] > T(0)) {
                    const T fN = -T(a.Ly[q]) + a.sigma * T(a.Ny[q]);
                    corr += a.S[q] * green_ball_t<D, T>(a.kappa, a.rho[q], a.d[q]) /
                            green_mass<D, T>(a.kappa, a.d[q]) * fN;
                }
                if (a.alive[q]) corr += T(a.Nstop[q]);
            }
            corr /= T(a.K);
            const T C = Noff - corr;
            a.target[i] = uplain + C;
            a.uoff[i] = beta * Noff + (uplain - beta * corr) * a.inv_q;
            bool moving = true;
            if (a.vparam) {
                const int32_t orig = a.prim[i] >> 1;
                moving = false;
                for (int k = 0; k < D; ++k) moving = moving || a.vparam[a.pverts[(size_t)orig * D + k]] != 0;
            }
            if (moving && isfinite(double(C)) && isfinite(double(uplain))) {
                s_n = 1.0;
                s_cc = double(C) * double(C);
                s_uc = double(uplain) * double(C);
            }
        }
    }
    s_n = wave_sum_f64(s_n);
    s_cc = wave_sum_f64(s_cc);
    s_uc = wave_sum_f64(s_uc);
    if ((threadIdx.x & 63) == 0 && s_n > 0.0) {
        atomicAdd(&a.stats[0], s_n);
        atomicAdd(&a.stats[1], s_cc);
        atomicAdd(&a.stats[2], s_uc);
    }
}

// beta for the next call from the last call's sums (kept when too few
// walks), then clear the sums; init != 0 sets beta = 1 instead.
__global__ void cv_beta_kernel(double* beta, double* stats, int init) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (init) {
        *beta = 1.0;
    } else if (stats[0] >= 64.0 && stats[1] > 0.0) {
        double b = -stats[2] / stats[1];
        *beta = b < 0.0 ? 0.0 : (b > 1.0 ? 1.0 : b);
    }
    stats[0] = stats[1] = stats[2] = 0.0;
}

// Export in the layout walk[9] = {run, xoff[3], uoff plain, uoff cv, target,
// u, primitive} and nested[10] = {S, alive, xstop[3], y[3], rho, d}.
template <class T, int D>
__global__ void cv_export_kernel(const int32_t* run, const T* xoff, const T* uplain, const T* ucv,
                                 const T* target, const T* u, const int32_t* prim, const T* S,
                                 const int32_t* alive, const T* stop, const T* y, const T* rho, const T* d, int64_t nwalks,
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
        o[0] = double(S[q]);
        o[1] = double(alive[q]);
        for (int c = 0; c < D; ++c) {
            o[2 + c] = double(stop[q * D + c]);
            o[5 + c] = double(y[q * D + c]);
        }
        o[8] = double(rho[q]);
        o[9] = double(d[q]);
    }
}

// Training of the network minimises the sample variance of the control-
// variate estimate: since E[C] = 0, E[(uhat + C)^2] = Var(uhat + C) + u^2, so
// the mean square of e = uhat + C over recorded walks is the variance up to
// a constant that does not depend on the network.  A boundary term
// lambda (N(xbar) - g)^2 anchors N to the data.  One step uses `batch` walks
// drawn uniformly from those of the last differential chunk whose nested
// walks ran at a terminal point on a primitive with a moving or
// parameterised vertex (only those enter the gradient): slot j tries up to
// kCvTries walks (Philox counter (j, step, try, 0xC0000000), key seed) and
// keeps the first that qualifies, else gets zero weight.  Rows of the
// network evaluations:
//   [0, b)            xoff           value
//   [b, 2b)           xbar           value
//   [2b, 2b + bK)     x_stop (j, k)  value
//   [2b + bK, 2b+2bK) y (j, k)       value and Laplacian
constexpr int kCvTries = 256;

template <class T, int D>
__global__ void cv_sample_kernel(const int32_t* run, const int32_t* prim, const int32_t* pverts,
                                 const int32_t* vparam, const T* xoff, const T* xbar, const T* g,
                                 const T* uplain, const T* S, const int32_t* alive, const T* stop, const T* y,
                                 const T* rho, const T* d, int64_t nwalks, int32_t batch, int32_t K,
                                 uint32_t step, uint32_t key0, uint32_t key1, T kappa, float* X,
                                 float* su, float* sg, float* sw, float* salive, int32_t* svalid) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= batch) return;
    int64_t i = 0;
    bool ok = false;
    for (uint32_t t = 0; t < (uint32_t)kCvTries && !ok; ++t) {
        const u4 r = philox10(u4{(uint32_t)j, step, t, 0xC0000000u}, key0, key1);
        i = (int64_t)(((unsigned long long)r.x * (unsigned long long)nwalks) >> 32);
        ok = run[i] == 1 && isfinite(double(uplain[i]));
        if (ok && vparam) {
            const int32_t orig = prim[i] >> 1;
            bool moving = false;
            for (int k = 0; k < D; ++k) moving = moving || vparam[pverts[(size_t)orig * D + k]] != 0;
            ok = moving;
        }
    }
    svalid[j] = ok ? 1 : 0;
    su[j] = ok ? float(uplain[i]) : 0.f;
    sg[j] = ok ? float(g[i]) : 0.f;
    const int64_t b = batch;
    for (int c = 0; c < D; ++c) {
        X[(size_t)j * D + c] = ok ? float(xoff[(size_t)i * D + c]) : 0.f;
        X[(size_t)(b + j) * D + c] = ok ? float(xbar[(size_t)i * D + c]) : 0.f;
    }
    for (int k = 0; k < K; ++k) {
        const size_t q = (size_t)i * K + k;
        const size_t rs = (size_t)(2 * b + (int64_t)j * K + k), ry = rs + (size_t)b * K;
        const bool src = ok && S[q] > T(0);
        for (int c = 0; c < D; ++c) {
            X[rs * D + c] = ok ? float(stop[q * D + c]) : 0.f;
            X[ry * D + c] = src ? float(y[q * D + c]) : 0.f;
        }
        salive[(size_t)j * K + k] = ok ? float(alive[q]) : 0.f;
        sw[(size_t)j * K + k] =
            src ? float(S[q] * green_ball_t<D, T>(kappa, rho[q], d[q]) / green_mass<D, T>(kappa, d[q])) : 0.f;
    }
}

// Output adjoints of the training objective
//   (1/b) sum_j [ 1/2 (uhat_j + C_j - m_j)^2 + lambda/2 (N(xbar_j) - g_j)^2 ],
//   C = N(xoff) - (1/K) sum_k (w_k (sigma N(y_k) - Lap N(y_k)) + alive_k N(x_stop_k))
// with w_k = S_k |B_k| G_k(y_k) / m_k.  The baseline m_j = N(xoff_j), held fixed in the
// differentiation, leaves the expected gradient unchanged (E[C | xoff] = 0
// for every network, so E[m dC/dtheta] = 0) and removes the u dC/dtheta noise:
// the residual is e = uhat - (1/K) sum_k (...).  loss (one float) += the
// objective.
__global__ void cv_adjoint_kernel(const float* N, const float* Ly, const float* su, const float* sg,
                                  const float* sw, const float* salive, const int32_t* svalid,
                                  int32_t batch, int32_t K, float sigma, float lambda, float* Nbar,
                                  float* Lbar, float* loss) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (j < batch) {
        const int64_t b = batch;
        const size_t rs = (size_t)(2 * b + (int64_t)j * K), ry = rs + (size_t)b * K;
        const float ib = 1.f / (float)batch, ik = 1.f / (float)K;
        if (svalid[j]) {
            float corr = 0.f;
            for (int k = 0; k < K; ++k) {
                const float w = sw[(size_t)j * K + k];
                corr += w * (sigma * N[ry + k] - Ly[(size_t)j * K + k]) + salive[(size_t)j * K + k] * N[rs + k];
            }
            const float e = su[j] - corr * ik;
            const float db = N[b + j] - sg[j];
            l = 0.5f * ib * (e * e + lambda * db * db);
            Nbar[j] = e * ib;
            Nbar[b + j] = lambda * db * ib;
            for (int k = 0; k < K; ++k) {
                const float w = sw[(size_t)j * K + k];
                Nbar[rs + k] = -e * salive[(size_t)j * K + k] * ik * ib;
                Nbar[ry + k] = -e * w * sigma * ik * ib;
                Lbar[ry + k] = e * w * ik * ib;
            }
        } else {
            Nbar[j] = 0.f;
            Nbar[b + j] = 0.f;
            for (int k = 0; k < K; ++k) {
                Nbar[rs + k] = 0.f;
                Nbar[ry + k] = 0.f;
                Lbar[ry + k] = 0.f;
            }
        }
        for (int k = 0; k < K; ++k) Lbar[rs + k] = 0.f;
        if (j < batch) { Lbar[j] = 0.f; Lbar[b + j] = 0.f; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o);
    if ((threadIdx.x & 63) == 0 && loss) atomicAdd(loss, l);
}

}  // namespace dwos
