// Device math for the walk kernels: Philox4x32-10, uniform/direction sampling,
// the ball's Green's function and Poisson-kernel scale, and the source term.
//
// Philox4x32-10 follows Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
// as easy as 1, 2, 3" (SC'11): ten rounds, each multiplying counter words 0
// and 2 by fixed 32-bit constants, xoring the high halves into the other words
// with the key, and advancing the key by two Weyl constants.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace dwos {

struct u4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u4 philox10(u4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = u4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 24-bit uniforms: [0, 1 - 2^-24] and (0, 1]; exact in FP32 and FP64.
template <class T> __device__ __forceinline__ T unif(uint32_t w) {
    return T(w >> 8) * T(5.9604644775390625e-08);
}
template <class T> __device__ __forceinline__ T unif_pos(uint32_t w) {
    return T((w >> 8) + 1u) * T(5.9604644775390625e-08);
}

__device__ __forceinline__ void sincos2pi(float u, float* s, float* c) { sincospif(2.0f * u, s, c); }
__device__ __forceinline__ void sincos2pi(double u, double* s, double* c) { sincospi(2.0 * u, s, c); }

// Direction uniform on the unit circle (2D: angle from w0) or sphere (3D:
// z = 1 - 2 U(w0), azimuth from w1).
template <class T, int D>
__device__ __forceinline__ void unit_dir(uint32_t w0, uint32_t w1, T* s) {
    if constexpr (D == 2) {
        sincos2pi(unif<T>(w0), &s[1], &s[0]);
    } else {
        const T z = T(1) - T(2) * unif<T>(w0);
        T sp, cp;
        sincos2pi(unif<T>(w1), &sp, &cp);
        const T rho = sqrt(fmax(T(0), T(1) - z * z));
        s[0] = rho * cp;
        s[1] = rho * sp;
        s[2] = z;
    }
}

// ---------------------------------------------------------------------------
// Modified Bessel functions for the 2D kernels.
//   I0(z) = sum_k t_k,  t_k = (z^2/4)^k / (k!)^2
//   F(z)  = K0(z) + (ln(z/2) + gamma) I0(z) = sum_{k>=1} H_k t_k
// (H_k harmonic numbers).  Both series have positive terms.  For z > 2 the
// kernels use exponentially scaled forms I0s(z) = e^-z I0(z) and
// K0s(z) = e^z K0(z) so that nothing overflows:
//   I0s: the series times e^-z for z <= 20, else the asymptotic series
//        (2 pi z)^-1/2 sum_k ((2k-1)!!)^2 / (k! (8z)^k)
//   K0s: the trapezoidal rule on e^z K0(z) = int_0^inf exp(-z (cosh t - 1)) dt
//        for z <= 20 (integrand analytic in |Im t| < pi/2, so the error
//        falls geometrically in 1/h), else the asymptotic series
//        (pi/(2z))^1/2 sum_k (-1)^k ((2k-1)!!)^2 / (k! (8z)^k).
// ---------------------------------------------------------------------------
template <class T> struct BesselCfg;
template <> struct BesselCfg<float> {
    static constexpr float tol = 3e-8f;
    static constexpr float h = 0.25f;   // trapezoid step: error ~e^{0.46 z - 25}
};
template <> struct BesselCfg<double> {
    static constexpr double tol = 1e-17;
    static constexpr double h = 0.125;  // error ~e^{z - 79}
};

// 1/k^2 and H_k for k = 0..63 (index 0 unused)
struct SeriesTables {
    double inv_k2[64];
    double harm[64];
    constexpr SeriesTables() : inv_k2(), harm() {
        double h = 0.0;
        for (int k = 1; k < 64; ++k) {
            inv_k2[k] = 1.0 / (double(k) * double(k));
            h += 1.0 / double(k);
            harm[k] = h;
        }
    }
};
__constant__ constexpr SeriesTables kSeries{};

// I0 by its series (z up to ~20)
template <class T>
__device__ inline T i0_series(T z) {
    const T q = T(0.25) * z * z;
    T t = T(1), s = T(1);
    for (int k = 1; k < 64; ++k) {
        t *= q * T(kSeries.inv_k2[k]);
        s += t;
        if (t < BesselCfg<T>::tol * s) break;
    }
    return s;
}

// I0 and F by their series, fixed 13 terms: exact to double rounding for z <= 2
__device__ __forceinline__ void i0_f_small(double z, double& i0, double& f) {
    const double q = 0.25 * z * z;
    double t = 1.0, s = 1.0, sf = 0.0;
#pragma unroll
    for (int k = 1; k <= 13; ++k) {
        t *= q * kSeries.inv_k2[k];
        s += t;
        sf += kSeries.harm[k] * t;
    }
    i0 = s;
    f = sf;
}

template <class T>
__device__ inline T i0_scaled(T z) {   // e^-z I0(z), z >= 0
    if (z <= T(20)) return i0_series<T>(z) * exp(-z);
    T a = T(1), s = T(1);
    for (int k = 1; k < 30; ++k) {
        a *= T((2 * k - 1) * (2 * k - 1)) / (T(8) * T(k) * z);
        s += a;
        if (a < BesselCfg<T>::tol * s) break;
    }
    return s / sqrt(T(6.283185307179586) * z);
}

template <class T>
__device__ inline T k0_scaled(T z) {   // e^z K0(z), z > 2
    if (z > T(20)) {
        T a = T(1), s = T(1);
        for (int k = 1; k < 30; ++k) {
            a *= -T((2 * k - 1) * (2 * k - 1)) / (T(8) * T(k) * z);
            s += a;
            if (fabs(a) < BesselCfg<T>::tol * s) break;
        }
        return sqrt(T(1.5707963267948966) / z) * s;
    }
    const T h = BesselCfg<T>::h;
    T s = T(0.5);
    for (int j = 1; j < 128; ++j) {
        const T e = exp(-z * (cosh(T(j) * h) - T(1)));
        s += e;
        if (e < BesselCfg<T>::tol * s) break;
    }
    return h * s;
}

template <class T>
__device__ inline T k0_small(T z) {    // K0(z) for 0 < z <= 2 from F - (ln(z/2) + gamma) I0
    const T q = T(0.25) * z * z;
    T t = T(1), s = T(1), sf = T(0);
    for (int k = 1; k < 64; ++k) {
        t *= q * T(kSeries.inv_k2[k]);
        s += t;
        sf += T(kSeries.harm[k]) * t;
        if (t < BesselCfg<T>::tol * s) break;
    }
    return sf - (log(T(0.5) * z) + T(0.57721566490153286061)) * s;
}

// I1 and K1 for the reflecting-boundary step weight:
//   I1(z) = (z/2) sum_k t_k,  t_k = (z^2/4)^k / (k! (k+1)!)
//   z K1(z) = 1 + z (ln(z/2) + gamma) I1(z) - (z^2/4) sum_k (H_k + H_{k+1}) t_k
// (Abramowitz-Stegun 9.6.11 with n = 1; the second line is the series times
// z, free of the 1/z pole).  Scaled forms for z > 2: e^z K1(z) by the
// trapezoidal rule on int_0^inf cosh(t) exp(-z (cosh t - 1)) dt (z <= 20) or
// its asymptotic series sqrt(pi/(2z)) sum_k c_k z^-k, c_k = c_{k-1}
// (4 - (2k-1)^2)/(8k); e^-z I1(z) by the series (z <= 20) or
// (2 pi z)^-1/2 sum_k (-1)^k c_k z^-k.
template <class T>
__device__ inline T i1_series(T z) {
    const T q = T(0.25) * z * z;
    T t = T(1), s = T(1);
    for (int k = 1; k < 64; ++k) {
        t *= q / (T(k) * T(k + 1));
        s += t;
        if (t < BesselCfg<T>::tol * s) break;
    }
    return T(0.5) * z * s;
}

template <class T>
__device__ inline T i1_scaled(T z) {   // e^-z I1(z), z >= 0
    if (z <= T(20)) return i1_series<T>(z) * exp(-z);
    T a = T(1), s = T(1);
    for (int k = 1; k < 30; ++k) {
        a *= -(T(4) - T((2 * k - 1) * (2 * k - 1))) / (T(8) * T(k) * z);
        s += a;
        if (fabs(a) < BesselCfg<T>::tol * s) break;
    }
    return s / sqrt(T(6.283185307179586) * z);
}

template <class T>
__device__ inline T zk1_small(T z) {   // z K1(z), 0 < z <= 2
    const T q = T(0.25) * z * z;
    T t = T(1), si = T(1), sh = T(1);   // t_0 = 1, H_0 + H_1 = 1
    for (int k = 1; k < 63; ++k) {      // harm[] has entries up to index 63
        t *= q / (T(k) * T(k + 1));
        si += t;
        sh += T(kSeries.harm[k] + kSeries.harm[k + 1]) * t;
        if (t < BesselCfg<T>::tol * si) break;
    }
    const T i1 = T(0.5) * z * si;
    return T(1) + z * (log(T(0.5) * z) + T(0.57721566490153286061)) * i1 - q * sh;
}

template <class T>
__device__ inline T k1_scaled(T z) {   // e^z K1(z), z > 2
    if (z > T(20)) {
        T a = T(1), s = T(1);
        for (int k = 1; k < 30; ++k) {
            a *= (T(4) - T((2 * k - 1) * (2 * k - 1))) / (T(8) * T(k) * z);
            s += a;
            if (fabs(a) < BesselCfg<T>::tol * s) break;
        }
        return sqrt(T(1.5707963267948966) / z) * s;
    }
    const T h = BesselCfg<T>::h;
    T s = T(0.5);
    for (int j = 1; j < 128; ++j) {
        const T c = cosh(T(j) * h);
        const T e = c * exp(-z * (c - T(1)));
        s += e;
        if (e < BesselCfg<T>::tol * s) break;
    }
    return h * s;
}

// ---------------------------------------------------------------------------
// Ball kernels for Algorithm 1 (Sec. 3.3.1), k = sqrt(sigma):
//   alpha(R) = P(R)/p^dB = 1/I0(kR) (2D),  kR/sinh(kR) (3D),  1 (sigma = 0)
//   G(r;R)|B_R| with r = rho R, rho in (0, 1]:
//     2D: pi R^2 [K0(kr) - K0(kR) I0(kr)/I0(kR)] / (2 pi)
//     3D: (4/3) pi R^3 sinh(k(R-r)) / (4 pi r sinh(kR))
// 2D at small radius (kR <= 2) is evaluated in FP64 with the log-factored form
//   2 pi G = I0(kr) ln(R/r) + [F(kr) I0(kR) - F(kR) I0(kr)] / I0(kR),
// which removes the cancellation between the logarithmic singular parts of
// K0(kr) and K0(kR); at kR > 2 the direct form is evaluated with scaled
// functions in the working precision.  3D uses expm1 so that the sinh ratio
// e^{-kr} (1 - e^{-2k(R-r)}) / (1 - e^{-2kR}) has no cancellation.
// ---------------------------------------------------------------------------
template <class T, int D>
__device__ __forceinline__ T poisson_scale(T kappa, T R) {
    if (kappa == T(0)) return T(1);
    const T a = kappa * R;
    if constexpr (D == 2) {
        if constexpr (sizeof(T) == 4) {
            if (a <= T(2)) {   // eight terms of the I0 series reach FP32 resolution
                const float q = 0.25f * a * a;
                float t = 1.0f, sum = 1.0f;
#pragma unroll
                for (int k = 1; k <= 8; ++k) {
                    t *= q * (1.0f / float(k * k));
                    sum += t;
                }
                return T(1) / sum;
            }
        }
        if (a <= T(20)) return T(1) / i0_series<T>(a);
        return exp(-a) / i0_scaled<T>(a);
    } else {
        return T(2) * a * exp(-a) / (-expm1(T(-2) * a));
    }
}

// Green's-function mass of the ball, int_B G dy = (1 - alpha(R))/sigma
// (R^2/(2D) at sigma = 0), with 1 - alpha from its power series where alpha
// is close to 1: 2D (I0(x) - 1)/I0(x), 3D (sinh x - x)/sinh x, x = kR.
template <int D, class T>
__device__ inline T green_mass(T kappa, T R) {
    if (kappa == T(0)) return R * R / T(2 * D);
    const T x = kappa * R, k2 = kappa * kappa;
    if constexpr (D == 2) {
        if (x < T(2)) {
            const T q = T(0.25) * x * x;
            T t = T(1), s = T(0);
            for (int k = 1; k < 40; ++k) {
                t *= q * T(kSeries.inv_k2[k]);
                s += t;
                if (t < BesselCfg<T>::tol * s) break;
            }
            return s / ((T(1) + s) * k2);
        }
        return (T(1) - poisson_scale<T, 2>(kappa, R)) / k2;
    } else {
        if (x < T(1)) {
            const T x2 = x * x;
            T t = x, s = T(0);
            for (int k = 1; k < 20; ++k) {
                t *= x2 / (T(2 * k) * T(2 * k + 1));
                s += t;
                if (t < BesselCfg<T>::tol * s) break;
            }
            return s / (sinh(x) * k2);
        }
        return (T(1) - poisson_scale<T, 3>(kappa, R)) / k2;
    }
}

// FP32 2D ball Green's function for b = kappa R <= 2 (returns 2 pi G for
// a = rho b, given L = -ln rho).  With A = a^2/4, B = b^2/4, c_k = 1/(k!)^2,
// the series I0 = sum c_k Z^k and F = sum H_k c_k Z^k (H_k the harmonic
// numbers) of 2 pi G = I0(a) L + (F(a) I0(b) - F(b) I0(a)) / I0(b), and the
// divided differences P_k = (B^k - A^k) / (B - A) = B P_{k-1} + A^(k-1):
//   F(a) - F(b)   = -(B - A) sum H_k c_k P_k,
//   I0(b) - I0(a) =  (B - A) sum c_k P_k,
// so the second term is (B - A) [F(b)/I0(b) sum c_k P_k - sum H_k c_k P_k],
// whose summands all have one sign (F(b)/I0(b) < 1 <= H_k for B <= 1):
// no cancellation as a -> b, where the term vanishes.  Eight terms reach
// FP32 resolution for B <= 1.
__device__ __forceinline__ float green2_small_f32(float rho, float b, float L) {
    const float a = rho * b;
    const float A = 0.25f * a * a, B = 0.25f * b * b;
    float ck = 1.0f, Ak = 1.0f, Bk = 1.0f, hk = 0.0f;
    float i0a = 1.0f, i0b = 1.0f, fb = 0.0f, P = 1.0f, sc = 0.0f, sh = 0.0f;
#pragma unroll
    for (int k = 1; k <= 8; ++k) {
        ck *= 1.0f / float(k * k);
        hk += 1.0f / float(k);
        if (k > 1) P = B * P + Ak;   // Ak still holds A^(k-1)
        Ak *= A;
        Bk *= B;
        i0a += ck * Ak;
        i0b += ck * Bk;
        fb += hk * ck * Bk;
        sc += ck * P;
        sh += hk * ck * P;
    }
    const float ba = B * ((1.0f - rho) * (1.0f + rho));
    return i0a * L + ba * (fb / i0b * sc - sh);
}

template <int D, class T>
__device__ inline T green_ball_t(T kappa, T rho, T R) {
    if constexpr (D == 2) {
        const T lnR_r = -log(rho);
        if (kappa == T(0)) return T(0.5) * R * R * lnR_r;
        const T b = kappa * R, a = rho * b;
        if (b <= T(2)) {
            if constexpr (sizeof(T) == 4) return T(0.5) * R * R * green2_small_f32(rho, b, lnR_r);
            double i0a, fa, i0b, fb;
            i0_f_small(double(a), i0a, fa);
            i0_f_small(double(b), i0b, fb);
            const double g2pi = i0a * double(lnR_r) + (fa * i0b - fb * i0a) / i0b;
            return T(0.5 * double(R) * double(R) * g2pi);
        }
        // 2 pi G = K0(a) - K0(b) I0(a)/I0(b)
        //        = K0(a) - K0s(b) I0s(a)/I0s(b) e^{a - 2b}
        const T ka = a <= T(2) ? k0_small<T>(a) : k0_scaled<T>(a) * exp(-a);
        const T g2pi = ka - k0_scaled<T>(b) * (i0_scaled<T>(a) / i0_scaled<T>(b)) * exp(a - T(2) * b);
        return T(0.5) * R * R * g2pi;
    } else {
        const T r = rho * R;
        if (kappa == T(0)) return R * R * (R - r) / (T(3) * r);
        const T ratio = exp(-kappa * r) * (expm1(T(-2) * kappa * (R - r)) / expm1(T(-2) * kappa * R));
        return R * R * R * ratio / (T(3) * r);
    }
}

// Weight of a walk-on-stars step that ends on the reflecting boundary at
// distance r < R: the ball's Poisson kernel there (-dG/dn, the normal
// derivative of G from green_ball_t's Green's function) over the density of
// that point under uniform direction sampling, |dS_1| r^(D-1) |dG/dr|:
//   2D: a [K1(a) + K0(b) I1(a) / I0(b)],  a = k r, b = k R
//   3D: [a cosh(b - a) + sinh(b - a)] / sinh(b)
//       = e^-a [a (2 + E) - E] / (1 - e^-2b),  E = e^{-2(b - a)} - 1
// It is 1 at sigma = 0, tends to 1 as r -> 0 and equals poisson_scale at
// r = R.  2D with b > 2 uses the scaled functions:
//   K0(b) I1(a) / I0(b) = K0s(b) I1s(a) / I0s(b) e^{a - 2b}.
template <int D, class T>
__device__ inline T reflect_weight(T kappa, T r, T R) {
    if (kappa == T(0)) return T(1);
    const T a = kappa * r, b = kappa * R;
    if constexpr (D == 2) {
        const T t1 = a <= T(2) ? zk1_small<T>(a) : a * k1_scaled<T>(a) * exp(-a);
        T t2;
        if (b <= T(2)) t2 = a * k0_small<T>(b) * i1_series<T>(a) / i0_series<T>(b);
        else t2 = a * k0_scaled<T>(b) * (i1_scaled<T>(a) / i0_scaled<T>(b)) * exp(a - T(2) * b);
        return t1 + t2;
    } else {
        const T E = expm1(T(-2) * (b - a));
        return exp(-a) * (a * (T(2) + E) - E) / (-expm1(T(-2) * b));
    }
}

}  // namespace dwos
