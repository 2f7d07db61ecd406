// Walks on an implicit Dirichlet boundary (2D) on gfx950: the zero set of
// h(x) = c + sum_n a_n / |x - p_n| with the domain {h > 0} (the harmonic
// monopoles of the paper's curve-inflation example, Sec. 7.4), for
// Algorithm 1 and Algorithm 2.  No BVH: every step evaluates the monopole
// sum, so the kernel is bound by vector ALU.
//   * ball radius: the larger of two safe radii, the Harnack radius (1/r is
//     harmonic in 3D, so f = h - c > 0 obeys Harnack's inequality on the 3D
//     ball out to the nearest pole, whose planar section is a disk) and a
//     direct bound (each positive monopole term is at least
//     a_n / (|x - p_n| + d) on the disk; Newton on the concave 1/S(d) rises
//     to the root of S(d) = -c from below, eight iterations);
//   * shell: h <= |grad h| eps where h < -c (the gradient test would also
//     hold next to a pole), boundary point by one Newton projection
//     xbar = x - h grad h / |grad h|^2;
//   * differential terminal: outward normal n = -grad h / |grad h| at xbar,
//     nested walks from xbar - delta n, and for each parameter the normal
//     velocity (dh/dpi)/|grad h| in eq. (boundary_deriv_restricted):
//     udot_j = (dh/dpi_j)(xbar) s with s = (dg/dn - du/dn) / |grad h|.
// Per differential walk the kernel records xbar and s; imp_reduce_kernel
// turns them into forward-mode rows or the reverse-mode gradient.  The
// random numbers and step order are those of the walk-on-spheres kernel.
#pragma once
#include <type_traits>

#include "walk_kernels.hpp"

namespace dwos {

constexpr int kMaxMono = 1024;

constexpr int kImpRegs = 32;   // FP32: distances kept in registers per step

template <class T>
struct ImpArgs {
    const T* mono;     // n x 3: a, px, py
    int32_t n;
    T c;
    T* xbar;           // per differential walk: terminal boundary point (2)
    T* s;              // per differential walk: (dg/dn - du/dn) / |grad h|, 0 if none
};

// h and grad h at x.  The FP32 instantiation takes 1/r from the hardware
// reciprocal square root and the monopole terms as products with it; the
// FP64 one keeps the correctly rounded divisions of the plain formula.
template <class T>
__device__ __forceinline__ T imp_h(const T* mono, int n, T c, const T* x, T* gr) {
    T h = c;
    gr[0] = gr[1] = T(0);
    for (int i = 0; i < n; ++i) {
        const T dx = x[0] - mono[3 * i + 1], dy = x[1] - mono[3 * i + 2];
        if constexpr (std::is_same<T, float>::value) {
            const float rr = __builtin_amdgcn_rsqf(dx * dx + dy * dy);
            const float t = mono[3 * i] * rr;
            h += t;
            const float q = t * rr * rr;
            gr[0] -= q * dx;
            gr[1] -= q * dy;
        } else {
            const T r = sqrt(dx * dx + dy * dy);
            h += mono[3 * i] / r;
            const T q = mono[3 * i] / (r * r * r);
            gr[0] -= q * dx;
            gr[1] -= q * dy;
        }
    }
    return h;
}

// Safe radius: the larger of the direct bound (eight Newton steps on the
// concave 1/S(d) = 1/sum_n a_n / (r_n + d) towards -1/c from d = 0) and the
// Harnack radius of f = h - c out to the nearest pole.  FP32: r_n = |x - p_n|
// once per step, the Newton sums with the hardware reciprocal, and the
// iteration stops once converged to FP32 resolution.
template <class T>
__device__ __forceinline__ T imp_safe_radius(const T* mono, int n, T c, const T* x, T h) {
    const T A = -c;
    T d = T(0);
    T R = T(INFINITY);
    if constexpr (std::is_same<T, float>::value) {
        // r_n in registers for the first kImpRegs monopoles (the table is
        // padded with a = 0 up to kImpRegs entries, so the unrolled sums
        // need no branch), the rest recomputed in every Newton step
        float rreg[kImpRegs];
#pragma unroll
        for (int i = 0; i < kImpRegs; ++i) {
            const float dx = x[0] - mono[3 * i + 1], dy = x[1] - mono[3 * i + 2];
            const float r2 = dx * dx + dy * dy;
            const float r = r2 * __builtin_amdgcn_rsqf(r2);
            const bool live = i < n;
            rreg[i] = live ? r : 1.0f;
            R = live ? fminf(R, r) : R;
        }
        for (int i = kImpRegs; i < n; ++i) {
            const float dx = x[0] - mono[3 * i + 1], dy = x[1] - mono[3 * i + 2];
            const float r2 = dx * dx + dy * dy;
            R = fminf(R, r2 * __builtin_amdgcn_rsqf(r2));
        }
        for (int it = 0; it < 8; ++it) {
            float S = 0.0f, Tt = 0.0f;
#pragma unroll
            for (int i = 0; i < kImpRegs; ++i) {
                const float rq = __builtin_amdgcn_rcpf(rreg[i] + d);
                const float t = mono[3 * i] * rq;
                S += t;
                Tt = fmaf(t, rq, Tt);
            }
            for (int i = kImpRegs; i < n; ++i) {
                const float dx = x[0] - mono[3 * i + 1], dy = x[1] - mono[3 * i + 2];
                const float r2 = dx * dx + dy * dy;
                const float rq = __builtin_amdgcn_rcpf(r2 * __builtin_amdgcn_rsqf(r2) + d);
                const float t = mono[3 * i] * rq;
                S += t;
                Tt = fmaf(t, rq, Tt);
            }
            const float inc = (S * S / A - S) / Tt;
            d += inc;
            // the iterates rise monotonically to the root, quadratically
            // near it: once a step is below 1e-5 of the radius the rest are
            // below FP32 resolution (an earlier stop only shortens the step)
            if (inc <= 1e-5f * d) break;
        }
    } else {
        for (int it = 0; it < 8; ++it) {
            T S = T(0), Tt = T(0);
            for (int i = 0; i < n; ++i) {
                const T dx = x[0] - mono[3 * i + 1], dy = x[1] - mono[3 * i + 2];
                const T q = sqrt(dx * dx + dy * dy) + d;
                S += mono[3 * i] / q;
                Tt += mono[3 * i] / (q * q);
            }
            d += (S * S / A - S) / Tt;
        }
        for (int i = 0; i < n; ++i) {
            const T dx = x[0] - mono[3 * i + 1], dy = x[1] - mono[3 * i + 2];
            R = fmin(R, sqrt(dx * dx + dy * dy));
        }
    }
    const T f = h - c;
    const T t = T(2) * (f - A) / ((T(2) * A + f) + sqrt(f * f + T(8) * A * f));
    return fmax(d, t * R);
}

// restricted data of label 0 and its gradient
template <class T>
__device__ __forceinline__ T imp_g(const Params<T>& prm, const T* x, T* gr) {
    T v = prm.gc[0];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        v += prm.gb[0][i] * x[i];
#pragma unroll
        for (int j = 0; j < 2; ++j) v += x[i] * prm.gA[0][i * 3 + j] * x[j];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        gr[i] = prm.gb[0][i];
#pragma unroll
        for (int j = 0; j < 2; ++j) gr[i] += (prm.gA[0][i * 3 + j] + prm.gA[0][j * 3 + i]) * x[j];
    }
    return v;
}

// The monopole table sits in dynamic LDS (3 max(n, kImpRegs) scalars of T
// per block, zero past n).
template <class T, int MODE>
__global__ void __launch_bounds__(kBlock) implicit_kernel(WalkArgs<T> a, ImpArgs<T> im) {
    constexpr int D = 2;
    T* smono = reinterpret_cast<T*>(g_stage);
    const int npad = im.n < kImpRegs ? kImpRegs : im.n;   // zero scales past n
    for (int i = threadIdx.x; i < 3 * npad; i += blockDim.x) smono[i] = i < 3 * im.n ? im.mono[i] : T(0);
    __syncthreads();
    const int n = im.n;
    const T c = im.c;
    const int lane = threadIdx.x & 63;
    uint32_t key0 = a.key0, key1 = a.key1;
    if (a.seed_ptr) {
        const unsigned long long sd = *a.seed_ptr + (((unsigned long long)a.key1 << 32) | a.key0);
        key0 = (uint32_t)sd;
        key1 = (uint32_t)(sd >> 32);
    }
    unsigned long long pool_next = 0, pool_end = 0;   // wave-uniform
    bool done = false;
    int64_t wid = -1;
    T x[D], xoff[D], xb_t[D];
    T acc = T(0), u_main = T(0), usum = T(0);
    T kappa = T(0), eps = T(1), delta = T(1);
    T t_g = T(0), t_dgdn = T(0), t_gn = T(1);
    uint32_t k = 0, m = 0, p = 0;
    int32_t phase = 0;
    int64_t wsteps = 0;
    unsigned long long c_walks = 0, c_nested = 0, c_steps = 0, c_term = 0, c_trunc = 0, c_invalid = 0;
#pragma unroll 1
    while (true) {
        // ---- hand new walks to idle lanes ------------------------------------
        const bool need = (wid < 0) && !done;
        const unsigned long long mask = __ballot(need);
        if (mask) {
            const int cnt = __popcll(mask);
            const int rank = __popcll(mask & ((1ull << lane) - 1ull));
            const unsigned long long avail = pool_end - pool_next;
            unsigned long long myid;
            if (avail >= (unsigned long long)cnt) {
                myid = pool_next + rank;
                pool_next += cnt;
            } else {
                const int leader = __ffsll((long long)mask) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)kQueueChunk);
                base = bcast64(base, leader);
                myid = (unsigned long long)rank < avail ? pool_next + rank : base + (rank - avail);
                pool_next = base + (cnt - avail);
                pool_end = base + kQueueChunk;
            }
            if (need) {
                if (myid >= (unsigned long long)a.total) {
                    done = true;
                } else {
                    wid = (int64_t)myid;
                    const Instance<T> in = a.inst[0];
                    const int64_t local = wid + a.wid_offset - in.walk_begin;
                    const int64_t pin = local / a.W;
                    m = (uint32_t)(local - pin * a.W);
                    p = (uint32_t)(pin + in.p_counter);
                    kappa = in.kappa; eps = in.eps; delta = in.delta;
                    const double* xp = a.X + (size_t)(in.point_begin + pin) * D;
#pragma unroll
                    for (int i = 0; i < D; ++i) x[i] = T(xp[i]);
                    acc = T(0); k = 0; phase = 0; usum = T(0); wsteps = 0;
                    c_walks++;
                }
            }
        }
        if (__ballot(!done) == 0ull) break;
        if (done) continue;

        T gr[2];
        const T h = imp_h<T>(smono, n, c, x, gr);
        c_steps++;
        wsteps++;
        if (!(h == h)) {   // non-finite position: end the walk with a NaN result
            c_invalid++;
            a.rec_u[wid] = T(NAN);
            if (MODE == 1) { a.rec_prim[wid] = -1; a.rec_uoff[wid] = T(NAN); im.s[wid] = T(0); }
            if (a.rec_steps) a.rec_steps[wid] = wsteps;
            wid = -1;
            continue;
        }
        const T gn = sqrt(gr[0] * gr[0] + gr[1] * gr[1]);
        const bool shell = h <= gn * eps && h < -c;
        const bool cap = (int)(k + 1) >= a.prm.kmax;
        const bool nested = MODE == 1 && phase > 0;
        bool finished = false;
        T result = T(0);
        if (shell || cap) {
            if (cap && !shell) c_trunc++;
            T xb[2] = {x[0] - h * gr[0] / (gn * gn), x[1] - h * gr[1] / (gn * gn)};
            T ggr[2];
            const T g = imp_g<T>(a.prm, xb, ggr);
            if (MODE == 1 && phase == 0) {
                T gb[2];
                imp_h<T>(smono, n, c, xb, gb);
                const T gbn = sqrt(gb[0] * gb[0] + gb[1] * gb[1]);
                const T nx = -gb[0] / gbn, ny = -gb[1] / gbn;
                u_main = acc + g;
                t_g = g;
                t_dgdn = ggr[0] * nx + ggr[1] * ny;
                t_gn = gbn;
                xb_t[0] = xb[0]; xb_t[1] = xb[1];
                xoff[0] = xb[0] - delta * nx;
                xoff[1] = xb[1] - delta * ny;
                c_term++;
                phase = 1;
                x[0] = xoff[0]; x[1] = xoff[1];
                acc = T(0); k = 0;
                c_nested++;
                continue;
            }
            finished = true;
            result = acc + g;
        } else {
            const T d = imp_safe_radius<T>(smono, n, c, x, h);
            const uint32_t tag = nested ? (1u | ((uint32_t)(phase - 1) << 8)) : 0u;
            const u4 r = philox10(u4{k, m, p, tag}, key0, key1);
            if (a.prm.has_source) {
                T dir[3];
                unit_dir<T, D>(r.y, 0u, dir);
                const T rho = sqrt(unif_pos<T>(r.w));
                T y[3];
#pragma unroll
                for (int cc = 0; cc < D; ++cc) y[cc] = x[cc] + rho * d * dir[cc];
                acc += green_ball_t<D, T>(kappa, rho, d) * source_f<T, D>(a.prm, y);
            }
            const T alpha = poisson_scale<T, D>(kappa, d);
            if (a.prm.rr && alpha < unif<T>(r.z)) {
                finished = true;
                result = acc;
            } else {
                T dir[3];
                unit_dir<T, D>(r.x, r.y, dir);
#pragma unroll
                for (int cc = 0; cc < D; ++cc) x[cc] += d * dir[cc];
                ++k;
            }
        }
        if (!finished) continue;

        if (MODE == 0) {
            a.rec_u[wid] = result;
            if (a.rec_steps) a.rec_steps[wid] = wsteps;
            wid = -1;
        } else if (phase == 0) {   // stopped by roulette: udot = 0, u = sources
            a.rec_u[wid] = result;
            a.rec_prim[wid] = -1;
            a.rec_uoff[wid] = T(0);
            im.s[wid] = T(0);
            if (a.rec_steps) a.rec_steps[wid] = wsteps;
            wid = -1;
        } else {
            usum += result;
            if (phase >= a.prm.K) {
                const T uoff = usum / T(a.prm.K);
                a.rec_u[wid] = u_main;
                a.rec_prim[wid] = 0;
                a.rec_uoff[wid] = uoff;
                im.xbar[(size_t)wid * 2] = xb_t[0];
                im.xbar[(size_t)wid * 2 + 1] = xb_t[1];
                im.s[wid] = (t_dgdn - (t_g - uoff) / delta) / t_gn;
                if (a.rec_steps) a.rec_steps[wid] = wsteps;
                wid = -1;
            } else {
                ++phase;
                x[0] = xoff[0]; x[1] = xoff[1];
                acc = T(0); k = 0;
                c_nested++;
            }
        }
    }
    c_walks = wave_sum_u64(c_walks);
    c_nested = wave_sum_u64(c_nested);
    c_steps = wave_sum_u64(c_steps);
    c_term = wave_sum_u64(c_term);
    c_trunc = wave_sum_u64(c_trunc);
    c_invalid = wave_sum_u64(c_invalid);
    if (lane == 0) {
        Counters* dst[2] = {a.cnt, a.tot};
        for (int q = 0; q < 2; ++q) {
            Counters* cc = dst[q];
            atomicAdd(&cc->walks, c_walks);
            atomicAdd(&cc->nested, c_nested);
            atomicAdd(&cc->steps, c_steps);
            atomicAdd(&cc->terminal, c_term);
            if (c_trunc) atomicAdd(&cc->truncated, c_trunc);
            if (c_invalid) atomicAdd(&cc->invalid, c_invalid);
        }
    }
}

// One walk's row of udot for monopole (a, px, py): the terminal point xbar,
// s = (dg/dn - du/dn) / |grad h| and dh/da = 1/r, dh/dp = a (x - p) / r^3
// (r = |xbar - p|).  Both reductions take it from here, so that forward and
// reverse mode agree to the FP64 summation order.
template <class T>
__device__ __forceinline__ void imp_udot(T xb0, T xb1, T sw, T a, T px, T py, T* v) {
    const T dx = xb0 - px, dy = xb1 - py;
    const T r = sqrt(dx * dx + dy * dy);
    const T q = sw * a / (r * r * r);
    v[0] = sw / r;
    v[1] = q * dx;
    v[2] = q * dy;
}

// Forward mode.  One block per point, one thread per monopole (strided):
// the walk mean of udot_j = (dh/dpi_j)(xbar) s over the point's W walks and
// the variance of that mean, with dh/da_n = 1/r_n and
// dh/dp_n = a_n (x - p_n) / r_n^3 (r_n = |xbar - p_n|).  udot and udot_var
// (rows p_offset.. of P x 3n) are written if non-null; walk_udot
// (walks x 3n, walk-major) receives every walk's row if non-null.
template <class T>
__global__ void imp_jvp_kernel(const int32_t* prim, const T* xbar, const T* s, const T* mono, int32_t n,
                               int64_t P, int32_t W, int64_t p_offset, double* udot, double* udot_var,
                               double* walk_udot) {
    const int64_t pl = blockIdx.x;
    if (pl >= P) return;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const T a = mono[3 * i], px = mono[3 * i + 1], py = mono[3 * i + 2];
        double s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0};
        for (int32_t mm = 0; mm < W; ++mm) {
            const int64_t wd = pl * W + mm;
            double v[3] = {0, 0, 0};
            if (prim[wd] >= 0) {
                T vt[3];
                imp_udot<T>(xbar[2 * wd], xbar[2 * wd + 1], s[wd], a, px, py, vt);
#pragma unroll
                for (int j = 0; j < 3; ++j) v[j] = double(vt[j]);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) { s1[j] += v[j]; s2[j] += v[j] * v[j]; }
            if (walk_udot) {
#pragma unroll
                for (int j = 0; j < 3; ++j) walk_udot[wd * 3 * n + 3 * i + j] = v[j];
            }
        }
        const int64_t pg = pl + p_offset;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double mean = s1[j] / W;
            if (udot) udot[pg * 3 * n + 3 * i + j] = mean;
            if (udot_var)
                udot_var[pg * 3 * n + 3 * i + j] = W > 1 ? (s2[j] - W * mean * mean) / (double(W - 1) * W) : 0.0;
        }
    }
}

// Reverse-mode walk weights omega (FP64), one per differential walk:
// mode 0, omega = w_p / W; mode 1 (squared loss, U-statistic over batches
// of B walks), omega = [(S_b - u_m)/(B(B-1)) - uref_p/B]/(W/B) with S_b the
// sum of u over the walk's batch.  Walks stopped by roulette get 0.
template <class T>
__global__ void imp_coef_kernel(const T* rec_u, const int32_t* prim, int64_t walks, int32_t W,
                                int32_t B, int32_t mode, int64_t p_offset, const double* w, const double* uref,
                                double* coef) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= walks) return;
    if (prim[i] < 0) { coef[i] = 0.0; return; }
    const int64_t pl = i / W;
    const int32_t m = (int32_t)(i - pl * W);
    const int64_t pg = pl + p_offset;
    double omega;
    if (mode == 0) {
        omega = w[pg] / W;
    } else {
        const int64_t b0 = pl * W + (m / B) * B;
        double S = 0.0;
        for (int q = 0; q < B; ++q) S += double(rec_u[b0 + q]);
        omega = ((S - double(rec_u[i])) / (double(B) * (B - 1)) - uref[pg] / B) / double(W / B);
    }
    coef[i] = omega;
}

// grad_j += sum over walks of omega * udot_j (imp_udot).  Each block stages
// a tile of kImpTile walks (xbar, s, omega) in LDS; its threads form
// G = 256 / n groups (1 when n >= 256) that take monopole t % n over every
// G-th walk of the tile; the groups' FP64 partial sums meet in LDS and each
// parameter gets one atomic add per block.
constexpr int kImpTile = 1024;
template <class T>
__global__ void __launch_bounds__(256) imp_grad_kernel(const T* xbar, const T* s, const double* omega,
                                                       int64_t walks, const T* mono, int32_t n, double* grad) {
    __shared__ T sx[kImpTile], sy[kImpTile], ss[kImpTile];
    __shared__ double so[kImpTile];
    __shared__ double red[256 * 3];
    const int64_t w0 = (int64_t)blockIdx.x * kImpTile;
    const int cnt = walks - w0 < kImpTile ? (int)(walks - w0) : kImpTile;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
        const double om = omega[w0 + t];
        const bool on = om != 0.0;
        so[t] = om;
        sx[t] = on ? xbar[2 * (w0 + t)] : T(0);
        sy[t] = on ? xbar[2 * (w0 + t) + 1] : T(0);
        ss[t] = on ? s[w0 + t] : T(0);
    }
    __syncthreads();
    const int G = n >= (int)blockDim.x ? 1 : (int)blockDim.x / n;
    for (int i0 = 0; i0 < n; i0 += (int)blockDim.x) {
        const int t = threadIdx.x;
        const int i = i0 + (G > 1 ? t % n : t);
        const int g = G > 1 ? t / n : 0;
        double acc[3] = {0, 0, 0};
        if (i < n && g < G) {
            const T a = mono[3 * i], px = mono[3 * i + 1], py = mono[3 * i + 2];
            for (int q = g; q < cnt; q += G) {
                const double om = so[q];
                if (om == 0.0) continue;
                T v[3];
                imp_udot<T>(sx[q], sy[q], ss[q], a, px, py, v);
#pragma unroll
                for (int j = 0; j < 3; ++j) acc[j] += om * double(v[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) red[3 * t + j] = acc[j];
        __syncthreads();
        if (G > 1) {
            if (t < n) {
                double s3[3] = {0, 0, 0};
                for (int gg = 0; gg < G; ++gg)
#pragma unroll
                    for (int j = 0; j < 3; ++j) s3[j] += red[3 * (gg * n + t) + j];
#pragma unroll
                for (int j = 0; j < 3; ++j) atomicAdd(&grad[3 * t + j], s3[j]);
            }
        } else if (i < n) {
#pragma unroll
            for (int j = 0; j < 3; ++j) atomicAdd(&grad[3 * i + j], red[3 * t + j]);
        }
        __syncthreads();
    }
}

// Band points of the shape-functional derivative: per point, h and grad h
// in the working precision; a point in the band (h > 0, h < eps_band
// |grad h|, h < -c) gets the weight coef_p, s = 1/|grad h| and its
// coordinates for imp_grad_kernel (so that imp_udot gives V_n), every other
// point the weight 0.  region: 1 in the band, 2 elsewhere in the domain
// (h > 0), 0 outside.
template <class T>
__global__ void imp_band_kernel(const double* X, int64_t P, const double* coef, const T* mono, int32_t n, T c,
                                T eps_band, T* xb, T* sb, double* wout, int32_t* region) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const T x[2] = {T(X[2 * p]), T(X[2 * p + 1])};
    T gr[2];
    const T h = imp_h<T>(mono, n, c, x, gr);
    const T gn = sqrt(gr[0] * gr[0] + gr[1] * gr[1]);
    const bool band = h > T(0) && h < eps_band * gn && h < -c;
    xb[2 * p] = x[0];
    xb[2 * p + 1] = x[1];
    sb[p] = T(1) / gn;
    wout[p] = band ? coef[p] : 0.0;
    if (region) region[p] = band ? 1 : (h > T(0) ? 2 : 0);
}

}  // namespace dwos
