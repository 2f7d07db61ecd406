// The adjoint formulation of the shape derivative (Appendix B, eq.
// (functional_deriv_adjoint)) on gfx950: the alternative to Algorithm 2 that
// the paper rejects for its quadratic nesting, as an ablation.
//
// For the squared loss J = int_Omega l(u), l(u) = 1/2 (u - uref)^2 with a
// quadratic reference uref(x) = c + b.x + x^T A x, the adjoint lambda solves
//   -Lap lambda + sigma lambda = u - uref in Omega,  lambda = 0 on the boundary
// (eq. (bvp_adjoint) with the operator's sign flipped together with lambda),
// and
//   dJ/dpi_j = int_boundary [ -dlambda/dn udot_j + l(g) V_n,j ] dsigma
// where udot_j is the boundary value of the differential problem (the same
// terminal term as Algorithm 2's) and l(g) V_n,j the boundary term of
// eq. (functional_deriv).  At a boundary sample y with outward normal n:
//   * lambda(y - delta n) by walk on spheres with zero boundary data and the
//     source u - uref, whose u at each step's ball point comes from a whole
//     forward walk started there (the quadratic nesting);
//   * -dlambda/dn = lambda(y - delta n) / delta (backward difference);
//   * du/dn from the mean of K forward walks from y - delta n, as at a
//     differential terminal.
// One lane per (sample, walk); each query is a whole BVH traversal (no
// resumable queries or persistent queue: the walks of one lane are nested,
// not a flat sequence).  The lane writes the record (side code,
// barycentrics, offset mean) that the reverse-mode scatter turns into
// udot_j, the per-walk weight wq/W lambda/delta of that udot, and the
// coefficient wq/W l(g) of V_n.
//
// Random numbers: Philox4x32-10 keyed by the seed, counter (k, m, s,
// purpose): 0x10 the adjoint walk's step k (0x12 the second draw of a 3D
// step), 0x20 | k' << 8 the forward walk at the ball point of adjoint step
// k' (its steps k), 0x30 | i << 8 the i-th forward walk from the offset
// point (bit 1 of the purpose again marks a 3D step's second draw).
#pragma once
#include "walk_kernels.hpp"

namespace dwos {

constexpr uint32_t kAdjStep = 0x10u, kAdjSource = 0x20u, kAdjOffset = 0x30u;

template <class T>
struct AdjArgs {
    Scene<T> s;
    Params<T> prm;
    T kappa, eps, delta;
    const int32_t* code;     // S: primitive * 2 + flip (outward normal = -geometric normal)
    const double* bary;      // S x (D - 1)
    const double* wq;        // S quadrature weights
    int64_t S;
    int32_t W;
    double ref[13];          // uref: c, b[3], A[3][3] row-major (D x D used)
    uint32_t key0, key1;
    const int32_t* prim_dep; // per primitive: 1 if it moves with a parameter
    int32_t* rec_prim;       // S*W records for the reverse-mode scatter
    T* rec_b;
    T* rec_uoff;
    double* rec_w;           // per-walk weight of udot
    double* rec_e;           // per-walk coefficient of V_n
    double* out_lam;         // optional S*W: lambda at the offset point
    double* out_uoff;        // optional S*W: offset mean
    Counters* cnt;
    Counters* tot;
};

struct AdjCount {
    unsigned long long steps = 0, nested = 0, terminal = 0, truncated = 0, nodes = 0, prims = 0, invalid = 0;
};

template <class T, int D>
__device__ __forceinline__ T adj_uref(const AdjArgs<T>& a, const T* x) {
    T v = T(a.ref[0]);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        v += T(a.ref[1 + i]) * x[i];
#pragma unroll
        for (int j = 0; j < D; ++j) v += x[i] * T(a.ref[4 + i * 3 + j]) * x[j];
    }
    return v;
}

// Closest primitive to x (whole traversal); leaf position or -1 for a
// non-finite point.
template <class T, int D>
__device__ __forceinline__ int32_t adj_query(const AdjArgs<T>& a, const T* x, int32_t warm, T& d2, AdjCount& c) {
    TravStack<T, false> st;
    QueryCount qc{0, 0, 0};
    const StageView sv{0, -1};
    const int32_t leaf = closest_leaf<T, D>(a.s, sv, 0, x, warm, d2, qc, st);
    c.nodes += qc.nodes;
    c.prims += qc.prims;
    c.steps++;
    return leaf;
}

// Boundary value at the closest point of leaf `leaf` to x.
template <class T, int D>
__device__ __forceinline__ T adj_boundary(const AdjArgs<T>& a, int32_t leaf, const T* x) {
    const StageView sv{0, -1};
    T P[9], bary[3];
    scene_prim<T, D>(a.s, sv, leaf, P);
    prim_closest<T, D>(P, x, bary);
    const int32_t orig = a.s.orig[leaf];
    T V[9];
    int32_t vid[3];
    prim_vertices<T, D>(a.s, orig, V, vid);
    T xbar[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < D; ++c) {
        T v = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) v += bary[k] * V[k * D + c];
        xbar[c] = v;
    }
    return boundary_value<T, D>(a.s, a.prm, orig, bary, xbar, vid);
}

// Ball point of step k (stream (m, p, tag)) at x, radius d: returns rho.
template <class T, int D>
__device__ __forceinline__ T adj_ball_point(const u4& r, uint32_t k, uint32_t m, uint32_t p, uint32_t tag,
                                            const AdjArgs<T>& a, const T* x, T d, T* y) {
    T dir[3];
    if constexpr (D == 2) {
        unit_dir<T, D>(r.y, 0u, dir);
    } else {
        const u4 r2 = philox10(u4{k, m, p, tag | 2u}, a.key0, a.key1);
        unit_dir<T, D>(r2.x, r2.y, dir);
    }
    T rho;
    if constexpr (D == 2) rho = sqrt(unif_pos<T>(r.w));
    else rho = cbrt(unif_pos<T>(r.w));
#pragma unroll
    for (int c = 0; c < D; ++c) y[c] = x[c] + rho * d * dir[c];
    return rho;
}

// Algorithm 1 from x0 with the problem's source and boundary data.
template <class T, int D>
__device__ T adj_forward(const AdjArgs<T>& a, const T* x0, uint32_t m, uint32_t p, uint32_t tag, AdjCount& c) {
    T x[D];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = x0[i];
    T acc = T(0);
    int32_t warm = -1;
    c.nested++;
#pragma unroll 1
    for (uint32_t k = 0;; ++k) {
        T d2;
        const int32_t leaf = adj_query<T, D>(a, x, warm, d2, c);
        if (leaf < 0 || !(d2 >= T(0))) { c.invalid++; return T(NAN); }
        const T d = sqrt(d2);
        const bool cap = (int)(k + 1) >= a.prm.kmax;
        if (d < a.eps || cap) {
            if (cap && !(d < a.eps)) c.truncated++;
            return acc + adj_boundary<T, D>(a, leaf, x);
        }
        const u4 r = philox10(u4{k, m, p, tag}, a.key0, a.key1);
        if (a.prm.has_source) {
            T y[3];
            const T rho = adj_ball_point<T, D>(r, k, m, p, tag, a, x, d, y);
            acc += green_ball_t<D, T>(a.kappa, rho, d) * source_f<T, D>(a.prm, y);
        }
        const T alpha = poisson_scale<T, D>(a.kappa, d);
        if (a.prm.rr && alpha < unif<T>(r.z)) return acc;
        T dir[3];
        unit_dir<T, D>(r.x, r.y, dir);
#pragma unroll
        for (int i = 0; i < D; ++i) x[i] += d * dir[i];
        warm = leaf;
    }
}

// The adjoint at x0: zero boundary data, source u - uref with u from a
// forward walk at each step's ball point.
template <class T, int D>
__device__ T adj_lambda(const AdjArgs<T>& a, const T* x0, uint32_t m, uint32_t p, AdjCount& c) {
    T x[D];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = x0[i];
    T acc = T(0);
    int32_t warm = -1;
#pragma unroll 1
    for (uint32_t k = 0;; ++k) {
        T d2;
        const int32_t leaf = adj_query<T, D>(a, x, warm, d2, c);
        if (leaf < 0 || !(d2 >= T(0))) { c.invalid++; return T(NAN); }
        const T d = sqrt(d2);
        const bool cap = (int)(k + 1) >= a.prm.kmax;
        if (d < a.eps || cap) {
            if (cap && !(d < a.eps)) c.truncated++;
            return acc;
        }
        const u4 r = philox10(u4{k, m, p, kAdjStep}, a.key0, a.key1);
        T y[3];
        const T rho = adj_ball_point<T, D>(r, k, m, p, kAdjStep, a, x, d, y);
        const T uy = adj_forward<T, D>(a, y, m, p, kAdjSource | (k << 8), c);
        acc += green_ball_t<D, T>(a.kappa, rho, d) * (uy - adj_uref<T, D>(a, y));
        const T alpha = poisson_scale<T, D>(a.kappa, d);
        if (a.prm.rr && alpha < unif<T>(r.z)) return acc;
        T dir[3];
        unit_dir<T, D>(r.x, r.y, dir);
#pragma unroll
        for (int i = 0; i < D; ++i) x[i] += d * dir[i];
        warm = leaf;
    }
}

template <class T, int D>
__global__ void __launch_bounds__(256) adjoint_kernel(AdjArgs<T> a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    AdjCount c;
    if (i < a.S * a.W) {
        const int64_t sidx = i / a.W;
        const uint32_t m = (uint32_t)(i - sidx * a.W);
        const uint32_t p = (uint32_t)sidx;
        const int32_t code = a.code[sidx];
        const int32_t orig = code >> 1;
        T bary[3];
        if constexpr (D == 2) {
            bary[1] = T(a.bary[sidx]);
            bary[0] = T(1) - bary[1];
            bary[2] = T(0);
        } else {
            bary[1] = T(a.bary[sidx * 2]);
            bary[2] = T(a.bary[sidx * 2 + 1]);
            bary[0] = T(1) - bary[1] - bary[2];
        }
        T V[9];
        int32_t vid[3];
        prim_vertices<T, D>(a.s, orig, V, vid);
        T xbar[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int cc = 0; cc < D; ++cc) {
            T v = T(0);
#pragma unroll
            for (int k = 0; k < D; ++k) v += bary[k] * V[k * D + cc];
            xbar[cc] = v;
        }
        T n[3] = {T(0), T(0), T(0)};
        geo_normal<T, D>(V, n);
        if (code & 1) {
#pragma unroll
            for (int cc = 0; cc < D; ++cc) n[cc] = -n[cc];
        }
        T xoff[3];
#pragma unroll
        for (int cc = 0; cc < D; ++cc) xoff[cc] = xbar[cc] - a.delta * n[cc];
        const T g = boundary_value<T, D>(a.s, a.prm, orig, bary, xbar, vid);
        const T e = g - adj_uref<T, D>(a, xbar);
        T lam = T(0), uoff = g;
        c.terminal++;
        if (!a.prim_dep || a.prim_dep[orig]) {
            lam = adj_lambda<T, D>(a, xoff, m, p, c);
            T usum = T(0);
#pragma unroll 1
            for (int q = 0; q < a.prm.K; ++q)
                usum += adj_forward<T, D>(a, xoff, m, p, kAdjOffset | ((uint32_t)q << 8), c);
            uoff = usum / T(a.prm.K);
        }
        a.rec_prim[i] = code;
        a.rec_b[(size_t)i * (D - 1)] = bary[1];
        if constexpr (D == 3) a.rec_b[(size_t)i * 2 + 1] = bary[2];
        a.rec_uoff[i] = uoff;
        const double wq = a.wq[sidx] / a.W;
        a.rec_w[i] = wq * double(lam) / double(a.delta);
        a.rec_e[i] = wq * 0.5 * double(e) * double(e);
        if (a.out_lam) a.out_lam[i] = double(lam);
        if (a.out_uoff) a.out_uoff[i] = double(uoff);
    }
    // statistics: wave sums, one atomic per counter per wave
    const unsigned long long walks = wave_sum_u64(i < a.S * a.W ? 1ull : 0ull);
    c.steps = wave_sum_u64(c.steps);
    c.nested = wave_sum_u64(c.nested);
    c.terminal = wave_sum_u64(c.terminal);
    c.truncated = wave_sum_u64(c.truncated);
    c.nodes = wave_sum_u64(c.nodes);
    c.prims = wave_sum_u64(c.prims);
    c.invalid = wave_sum_u64(c.invalid);
    if ((threadIdx.x & 63) == 0) {
        Counters* dst[2] = {a.cnt, a.tot};
        for (int q = 0; q < 2; ++q) {
            Counters* cn = dst[q];
            atomicAdd(&cn->walks, walks);
            atomicAdd(&cn->nested, c.nested);
            atomicAdd(&cn->steps, c.steps);
            atomicAdd(&cn->terminal, c.terminal);
            atomicAdd(&cn->nodes, c.nodes);
            atomicAdd(&cn->prims, c.prims);
            if (c.truncated) atomicAdd(&cn->truncated, c.truncated);
            if (c.invalid) atomicAdd(&cn->invalid, c.invalid);
        }
    }
}

}  // namespace dwos
