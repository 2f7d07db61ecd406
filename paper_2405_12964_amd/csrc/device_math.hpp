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
// Both series have positive terms (no cancellation).  K0 for 2 < z <= 20
// uses the trapezoidal rule on K0(z) = int_0^inf exp(-z cosh t) dt, whose
// integrand is analytic in the strip |Im t| < pi/2 (geometric convergence in
// 1/h); for z > 20 its asymptotic expansion.
// ---------------------------------------------------------------------------
template <class T> struct SeriesTol;
template <> struct SeriesTol<float> { static constexpr float v = 3e-8f; };
template <> struct SeriesTol<double> { static constexpr double v = 1e-17; };

template <class T>
__device__ inline T bessel_i0(T z) {
    const T q = T(0.25) * z * z;
    T t = T(1), s = T(1);
    for (int k = 1; k < 200; ++k) {
        t *= q / T(k * k);
        s += t;
        if (t < SeriesTol<T>::v * s) break;
    }
    return s;
}

// I0(z) and F(z) together.
__device__ inline void bessel_i0_f(double z, double* i0, double* f) {
    const double q = 0.25 * z * z;
    double t = 1.0, s = 1.0, sf = 0.0, H = 0.0;
    for (int k = 1; k < 200; ++k) {
        t *= q / double(k * k);
        H += 1.0 / double(k);
        s += t;
        sf += H * t;
        if (t * H < 1e-17 * sf && t < 1e-17 * s) break;
    }
    *i0 = s;
    *f = sf;
}

__device__ inline double bessel_k0(double z) {
    const double euler_gamma = 0.57721566490153286061;
    if (z <= 2.0) {
        double i0, f;
        bessel_i0_f(z, &i0, &f);
        return f - (log(0.5 * z) + euler_gamma) * i0;
    }
    if (z > 20.0) {
        // asymptotic series sqrt(pi/(2z)) e^-z sum_k a_k, a_k = -a_{k-1} (2k-1)^2/(8kz);
        // its smallest term is ~e^{-2z}, below 1e-17 here
        double a = 1.0, s = 1.0;
        for (int k = 1; k < 40; ++k) {
            a *= -double((2 * k - 1) * (2 * k - 1)) / (8.0 * k * z);
            s += a;
            if (fabs(a) < 1e-18 * s) break;
        }
        return sqrt(1.5707963267948966 / z) * exp(-z) * s;
    }
    // trapezoid on e^z K0(z) = int_0^inf exp(-z (cosh t - 1)) dt; the error of
    // step h behaves like exp(z - pi^2/h), so h = 1/8 keeps it below 1e-25
    // for z <= 20
    const double h = 0.125;
    double s = 0.5;
    for (int j = 1; j < 128; ++j) {
        const double e = exp(-z * (cosh(j * h) - 1.0));
        s += e;
        if (e < 1e-18 * s) break;
    }
    return h * s * exp(-z);
}

// ---------------------------------------------------------------------------
// Ball kernels for Algorithm 1 (Sec. 3.3.1), k = sqrt(sigma):
//   alpha(R) = P(R)/p^dB = 1/I0(kR) (2D),  kR/sinh(kR) (3D),  1 (sigma = 0)
//   G(r;R)|B_R| with r = rho R, rho in (0, 1]:
//     2D: pi R^2 [K0(kr) - K0(kR) I0(kr)/I0(kR)] / (2 pi)
//     3D: (4/3) pi R^3 sinh(k(R-r)) / (4 pi r sinh(kR))
// 2D is evaluated in FP64.  For kR <= 2 it uses the log-factored form
//   2 pi G = I0(kr) ln(R/r) + [F(kr) I0(kR) - F(kR) I0(kr)] / I0(kR),
// which removes the cancellation of the two logarithmic singular parts of
// K0(kr) - K0(kR) at small radius.  3D uses expm1 so that the sinh ratio
// e^{-kr} (1 - e^{-2k(R-r)}) / (1 - e^{-2kR}) has no cancellation.
// ---------------------------------------------------------------------------
template <class T, int D>
__device__ __forceinline__ T poisson_scale(T kappa, T R) {
    if (kappa == T(0)) return T(1);
    const T a = kappa * R;
    if constexpr (D == 2) {
        return T(1) / bessel_i0<T>(a);
    } else {
        return T(2) * a * exp(-a) / (-expm1(T(-2) * a));
    }
}

template <int D>
__device__ inline double green_ball(double kappa, double rho, double R) {
    if constexpr (D == 2) {
        const double area = 3.14159265358979323846 * R * R;
        const double lnR_r = -log(rho);
        if (kappa == 0.0) return area * lnR_r / (2.0 * 3.14159265358979323846);
        const double b = kappa * R, a = rho * b;
        double g2pi;
        if (b <= 2.0) {
            double i0a, fa, i0b, fb;
            bessel_i0_f(a, &i0a, &fa);
            bessel_i0_f(b, &i0b, &fb);
            g2pi = i0a * lnR_r + (fa * i0b - fb * i0a) / i0b;
        } else {
            const double i0a = bessel_i0<double>(a), i0b = bessel_i0<double>(b);
            g2pi = bessel_k0(a) - bessel_k0(b) * (i0a / i0b);
        }
        return area * g2pi / (2.0 * 3.14159265358979323846);
    } else {
        const double r = rho * R;
        if (kappa == 0.0) return R * R * (R - r) / (3.0 * r);
        const double ratio = exp(-kappa * r) * (expm1(-2.0 * kappa * (R - r)) / expm1(-2.0 * kappa * R));
        return R * R * R * ratio / (3.0 * r);
    }
}

template <int D, class T>
__device__ __forceinline__ T green_ball_t(T kappa, T rho, T R) {
    if constexpr (D == 2) {
        return T(green_ball<2>(double(kappa), double(rho), double(R)));
    } else {
        if constexpr (sizeof(T) == 8) {
            return green_ball<3>(kappa, rho, R);
        } else {
            const T r = rho * R;
            if (kappa == T(0)) return R * R * (R - r) / (T(3) * r);
            const T ratio = exp(-kappa * r) * (expm1(T(-2) * kappa * (R - r)) / expm1(T(-2) * kappa * R));
            return R * R * R * ratio / (T(3) * r);
        }
    }
}

}  // namespace dwos
