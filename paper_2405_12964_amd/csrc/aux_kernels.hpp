// Kernels around the walk kernel: per-point statistics, reverse-mode scatter
// of the differential terminal term, parameter-space SpMV, forward-mode
// derivatives, BVH refit, and debug queries.
#pragma once
#include "walk_kernels.hpp"

namespace dwos {

// ---------------------------------------------------------------------------
// wave reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---------------------------------------------------------------------------
// Differential boundary value at a recorded terminal (Sec. 4, eqs.
// (boundary_deriv_restricted) and (boundary_deriv_mapped); Sec. 5.1,
// eq. (wos_deriv) with du/dn from eq. (dudn_fd_estimate)).  For parameter j
//   udot_j = sum_k b_k (Tvec . dv_{i_k}/dpi_j) + [mapped] sum_k b_k [bc_pid(i_k) = j]
// with
//   restricted: Tvec = n (dg/dn - du/dn)
//   mapped:     Tvec = -grad_G g - n du/dn   (material derivative of the
//               carried values; the tangential gradient absorbs the
//               reparameterisation term of the mapped form)
// and du/dn = (g(xbar) - u(xbar - delta n)) / delta.
// ---------------------------------------------------------------------------
template <class T, int D>
struct Terminal {
    T bary[3];
    int32_t vid[3];
    T Tvec[3];
    T n[3];        // outward normal
    bool mapped;
};

template <class T, int D>
__device__ __forceinline__ void terminal_term(const Scene<T>& s, const Params<T>& prm, T delta,
                                              int32_t code, const T* rb, T uoff, Terminal<T, D>& t) {
    const int32_t orig = code >> 1;
    const bool flip = code & 1;
    if constexpr (D == 2) { t.bary[1] = rb[0]; t.bary[2] = T(0); t.bary[0] = T(1) - rb[0]; }
    else { t.bary[1] = rb[0]; t.bary[2] = rb[1]; t.bary[0] = T(1) - rb[0] - rb[1]; }
    T V[9];
    prim_vertices<T, D>(s, orig, V, t.vid);
    T xbar[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < D; ++c) {
        T v = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) v += t.bary[k] * V[k * D + c];
        xbar[c] = v;
    }
    const T g = boundary_value<T, D>(s, prm, orig, t.bary, xbar, t.vid);
    T n[3] = {T(0), T(0), T(0)};
    geo_normal<T, D>(V, n);
    if (flip) {
#pragma unroll
        for (int c = 0; c < D; ++c) n[c] = -n[c];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) t.n[c] = n[c];
    const T dudn = (g - uoff) / delta;
    const int L = s.label[orig];
    t.mapped = prm.kind[L] == 1;
    if (!t.mapped) {
        T dgdn = T(0);
#pragma unroll
        for (int i = 0; i < D; ++i) {
            T gi = prm.gb[L][i];
#pragma unroll
            for (int j = 0; j < D; ++j) gi += (prm.gA[L][i * 3 + j] + prm.gA[L][j * 3 + i]) * xbar[j];
            dgdn += gi * n[i];
        }
#pragma unroll
        for (int c = 0; c < D; ++c) t.Tvec[c] = n[c] * (dgdn - dudn);
    } else {
        T gr[3] = {T(0), T(0), T(0)};
        const T ga = s.gvert[t.vid[0]], gb = s.gvert[t.vid[1]];
        if constexpr (D == 2) {
            const T tx = V[2] - V[0], ty = V[3] - V[1];
            const T L2 = tx * tx + ty * ty;
            gr[0] = (gb - ga) * tx / L2;
            gr[1] = (gb - ga) * ty / L2;
        } else {
            const T gc = s.gvert[t.vid[2]];
            const T e1[3] = {V[3] - V[0], V[4] - V[1], V[5] - V[2]};
            const T e2[3] = {V[6] - V[0], V[7] - V[1], V[8] - V[2]};
            const T d11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
            const T d12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
            const T d22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
            const T det = d11 * d22 - d12 * d12;
            const T r1 = gb - ga, r2 = gc - ga;
            const T al = (d22 * r1 - d12 * r2) / det, be = (d11 * r2 - d12 * r1) / det;
#pragma unroll
            for (int c = 0; c < 3; ++c) gr[c] = al * e1[c] + be * e2[c];
        }
#pragma unroll
        for (int c = 0; c < D; ++c) t.Tvec[c] = -gr[c] - n[c] * dudn;
    }
}

struct ParamCSR {
    const int64_t* rowptr;   // by vertex
    const int32_t* pid;
    const double* vel;       // nnz x D
    const int32_t* bc_pid;   // nv or null
    const int64_t* colptr;   // by parameter (transpose)
    const int32_t* cvert;
    const double* cvel;      // nnz x D
    const int64_t* bcptr;    // by parameter: vertices whose mapped value is it
    const int32_t* bcvert;
    int64_t N;
};

// velocity dv_i/dpi_j (zero if absent): binary search in the sorted CSR row
template <int D>
__device__ __forceinline__ bool jac_entry(const ParamCSR& J, int32_t i, int32_t j, double* v) {
    int64_t lo = J.rowptr[i], hi = J.rowptr[i + 1] - 1;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t q = J.pid[mid];
        if (q == j) {
#pragma unroll
            for (int c = 0; c < D; ++c) v[c] = J.vel[mid * D + c];
            return true;
        }
        if (q < j) lo = mid + 1; else hi = mid - 1;
    }
    return false;
}

template <class T, int D>
__device__ __forceinline__ double udot_component(const ParamCSR& J, const Terminal<T, D>& t, int32_t j) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double v[3];
        if (jac_entry<D>(J, t.vid[k], j, v)) {
            double dotv = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) dotv += double(t.Tvec[c]) * v[c];
            s += double(t.bary[k]) * dotv;
        }
        if (t.mapped && J.bc_pid && J.bc_pid[t.vid[k]] == j) s += double(t.bary[k]);
    }
    return s;
}

// ---------------------------------------------------------------------------
// per-point mean and variance of the mean over W walk records (one wave/point)
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) point_stats_kernel(const T* rec_u, int64_t P, int32_t W,
                                                          double* mean, double* var) {
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= P) return;
    double s1 = 0.0, s2 = 0.0;
    const T* r = rec_u + p * W;
    for (int m = lane; m < W; m += 64) { const double v = double(r[m]); s1 += v; s2 += v * v; }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
        const double mu = s1 / W;
        mean[p] = mu;
        if (var) var[p] = W > 1 ? fmax(0.0, (s2 - W * mu * mu) / (W - 1)) / W : 0.0;
    }
}

__global__ void sqloss_kernel(const double* mean, const double* uref, int64_t P, double* loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t p = threadIdx.x; p < P; p += 256) {
        const double e = mean[p] - uref[p];
        s += 0.5 * e * e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0];
}

// ---------------------------------------------------------------------------
// reverse mode: scatter omega_m * b_k * Tvec into per-vertex FP64 accumulators
//   mode 0 (weights): omega = w_p / W
//   mode 1 (squared loss, U-statistics over batches of B walks):
//     omega = [(S_b - u_m)/(B(B-1)) - uref_p/B] / (W/B),  S_b = sum of the batch
//   mode 2 (per-walk weights, the adjoint formulation): omega = w[i], plus
//     e[i] b_k n for the term e V_n of each record
// ---------------------------------------------------------------------------
template <class T>
struct AccArgs {
    Scene<T> s;
    Params<T> prm;
    T delta;
    const T* rec_u;
    const int32_t* rec_prim;
    const T* rec_b;
    const T* rec_uoff;
    const T* rec_w;          // per-walk throughput multiplying udot (null: 1)
    int64_t nwalks;          // records in this chunk
    int64_t p_offset;        // first point of this chunk
    int32_t W, B, mode;
    const double* w;         // mode 0: per point; mode 2: per walk
    const double* uref;      // mode 1
    const double* e;         // mode 2: per-walk coefficient of V_n
    const int32_t* bc_pid;
    // skip lists (NULL: none): terminals on primitives that depend on no
    // parameter, and vertices without a Jacobian row or value parameter --
    // their accumulators are multiplied by zero in the SpMV
    const int32_t* prim_dep;
    const int32_t* vparam;
    double* A;               // nv x D
    double* Bacc;            // nv
};

template <class T, int D>
__global__ void __launch_bounds__(256) accumulate_kernel(AccArgs<T> a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nwalks) return;
    const int32_t code = a.rec_prim[i];
    if (code < 0) return;
    if (a.prim_dep && !a.prim_dep[code >> 1]) return;
    const int64_t pl = i / a.W;
    const int32_t m = (int32_t)(i - pl * a.W);
    const int64_t p = pl + a.p_offset;
    double omega, ev = 0.0;
    if (a.mode == 0) {
        omega = a.w[p] / a.W;
    } else if (a.mode == 2) {
        omega = a.w[i];
        ev = a.e[i];
    } else {
        const int32_t b0 = (m / a.B) * a.B;
        const T* ub = a.rec_u + pl * a.W + b0;
        double S = 0.0;
        for (int q = 0; q < a.B; ++q) S += double(ub[q]);
        const double nb = double(a.W / a.B);
        omega = ((S - double(a.rec_u[i])) / (double(a.B) * (a.B - 1)) - a.uref[p] / a.B) / nb;
    }
    if (a.rec_w) omega *= double(a.rec_w[i]);
    Terminal<T, D> t;
    terminal_term<T, D>(a.s, a.prm, a.delta, code, a.rec_b + i * (D - 1), a.rec_uoff[i], t);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (a.vparam && !a.vparam[t.vid[k]]) continue;
        const double wb = omega * double(t.bary[k]);
        const double eb = ev * double(t.bary[k]);
#pragma unroll
        for (int c = 0; c < D; ++c)
            unsafeAtomicAdd(&a.A[(size_t)t.vid[k] * D + c], wb * double(t.Tvec[c]) + eb * double(t.n[c]));
        if (t.mapped && a.bc_pid && a.bc_pid[t.vid[k]] >= 0) unsafeAtomicAdd(&a.Bacc[t.vid[k]], wb);
    }
}

// grad_j = sum_{i in col j} A_i . dv_i/dpi_j + sum_{i: bc_pid(i) = j} Bacc_i (one wave/column)
template <int D>
__global__ void __launch_bounds__(256) spmv_kernel(ParamCSR J, const double* A, const double* Bacc,
                                                   double* grad) {
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= J.N) return;
    double s = 0.0;
    for (int64_t e = J.colptr[j] + lane; e < J.colptr[j + 1]; e += 64) {
        const int32_t v = J.cvert[e];
#pragma unroll
        for (int c = 0; c < D; ++c) s += A[(size_t)v * D + c] * J.cvel[e * D + c];
    }
    if (J.bcptr)
        for (int64_t e = J.bcptr[j] + lane; e < J.bcptr[j + 1]; e += 64) s += Bacc[J.bcvert[e]];
    s = wave_sum(s);
    if (lane == 0) grad[j] = s;
}

// ---------------------------------------------------------------------------
// forward mode: per point p, parameters j (block of 64 per (p, j-group))
// ---------------------------------------------------------------------------
template <class T>
struct JvpArgs {
    Scene<T> s;
    Params<T> prm;
    T delta;
    ParamCSR J;
    const T* rec_prim_u;     // unused placeholder to keep layout simple
    const int32_t* rec_prim;
    const T* rec_b;
    const T* rec_uoff;
    const T* rec_w;          // per-walk throughput multiplying udot (null: 1)
    int64_t P;
    int64_t p_offset;
    int32_t W;
    double* udot;            // P x N
    double* udot_var;
    double* walk_udot;       // per-walk P*W*N (debug) or null
};

template <class T, int D>
__global__ void __launch_bounds__(64) jvp_kernel(JvpArgs<T> a) {
    const int64_t pl = blockIdx.x;
    const int64_t j = (int64_t)blockIdx.y * 64 + threadIdx.x;
    if (pl >= a.P || j >= a.J.N) return;
    double s1 = 0.0, s2 = 0.0;
    for (int m = 0; m < a.W; ++m) {
        const int64_t i = pl * a.W + m;
        const int32_t code = a.rec_prim[i];
        double v = 0.0;
        if (code >= 0) {
            Terminal<T, D> t;
            terminal_term<T, D>(a.s, a.prm, a.delta, code, a.rec_b + i * (D - 1), a.rec_uoff[i], t);
            v = udot_component<T, D>(a.J, t, (int32_t)j);
            if (a.rec_w) v *= double(a.rec_w[i]);
        }
        if (a.walk_udot) a.walk_udot[i * a.J.N + j] = v;
        s1 += v;
        s2 += v * v;
    }
    const int64_t p = pl + a.p_offset;
    if (a.udot) {
        const double mu = s1 / a.W;
        a.udot[p * a.J.N + j] = mu;
        if (a.udot_var)
            a.udot_var[p * a.J.N + j] = a.W > 1 ? fmax(0.0, (s2 - a.W * mu * mu) / (a.W - 1)) / a.W : 0.0;
    }
}

// ---------------------------------------------------------------------------
// debug queries
// ---------------------------------------------------------------------------
template <class T, int D>
__global__ void closest_kernel(Scene<T> s, int32_t root, const double* X, int64_t P, double* out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const StageView sv{0, -1};
    T x[D];
#pragma unroll
    for (int c = 0; c < D; ++c) x[c] = T(X[p * D + c]);
    T d2;
    QueryCount qc{0, 0, 0};
    TravStack<T, false> stack;
    const int32_t leaf = closest_leaf<T, D>(s, sv, root, x, -1, d2, qc, stack);
    double* o = out + p * 8;
    if (leaf < 0) {
        for (int k = 0; k < 8; ++k) o[k] = NAN;
        return;
    }
    T P9[9], bary[3];
    scene_prim<T, D>(s, sv, leaf, P9);
    prim_closest<T, D>(P9, x, bary);
    const int32_t orig = s.orig[leaf];
    T V[9];
    int32_t vid[3];
    prim_vertices<T, D>(s, orig, V, vid);
    o[0] = sqrt(double(d2));
    o[1] = double(orig);
    for (int k = 0; k < 3; ++k) o[2 + k] = k < D ? double(bary[k]) : 0.0;
    for (int c = 0; c < 3; ++c) {
        double v = 0.0;
        if (c < D)
            for (int k = 0; k < D; ++k) v += double(bary[k]) * double(V[k * D + c]);
        o[5 + c] = v;
    }
}

// closest primitive of each start point (shared first query of its walks);
// ---------------------------------------------------------------------------
// Spatial scheduling order of a chunk's points: the walk kernel hands out
// walks point by point in this order, so the walks in flight at any time
// start close together and gather from the same part of the BVH (the L2 of
// each XCD then holds that part).  A counting sort by cell of a 16^3 (3D) or
// 64^2 (2D) grid over the boundary's bounding box, cells in Morton order;
// the order within a cell is whatever the atomics give -- walks and their
// records are indexed by point, so no result depends on it.
// ---------------------------------------------------------------------------
constexpr int kOrderCells = 4096;

__device__ __forceinline__ uint32_t spread_bits(uint32_t v, int D) {
    uint32_t out = 0;
    const int nb = D == 3 ? 4 : 6;
    for (int b = 0; b < nb; ++b) out |= ((v >> b) & 1u) << (b * D);
    return out;
}

template <class T, int D>
__global__ void order_cell_kernel(const T* nodes, const double* X, int64_t P, int32_t* cell, uint32_t* hist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    NodeData<T, D> nd;
    load_node<T, D>(nodes, 0, nd);
    const int side = D == 3 ? 16 : 64;
    uint32_t code = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        T lo = T(INFINITY), hi = T(-INFINITY);
        if (!(nd.t0 < T(0))) { lo = fmin(lo, nd.lo0[c]); hi = fmax(hi, nd.hi0[c]); }
        if (!(nd.t1 < T(0))) { lo = fmin(lo, nd.lo1[c]); hi = fmax(hi, nd.hi1[c]); }
        const double ext = double(hi) - double(lo);
        double f = ext > 0.0 ? (X[i * D + c] - double(lo)) / ext : 0.0;
        f = f == f ? fmin(fmax(f, 0.0), 1.0) : 0.0;          // NaN -> cell 0
        const uint32_t q = (uint32_t)fmin(f * side, double(side - 1));
        code |= spread_bits(q, D) << c;
    }
    cell[i] = (int32_t)code;
    atomicAdd(&hist[code], 1u);
}

// exclusive scan of the kOrderCells counts, in place, by one 1024-thread block
__global__ void __launch_bounds__(1024) order_scan_kernel(uint32_t* hist) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) { v[k] = hist[t * 4 + k]; s += v[k]; }
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint32_t add = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
#pragma unroll
    for (int k = 0; k < 4; ++k) { hist[t * 4 + k] = run; run += v[k]; }
}

__global__ void order_scatter_kernel(const int32_t* cell, int64_t P, uint32_t* cursor, int32_t* perm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const uint32_t slot = atomicAdd(&cursor[cell[i]], 1u);
    perm[slot] = (int32_t)i;
}

// row r of X is global point x_base + r, which lies in the instance whose
// point range contains it.  warm_in (or null): per row a primitive (leaf
// position) to start the query from (it may be leaf_out itself), used only
// when it lies in the row's instance's leaf positions: prange[2 i] ..
// prange[2 i + 1] for instance i, or (prange null, a single-instance scene
// whose tree holds every primitive) 0 .. n_prims.
template <class T, int D>
__global__ void first_query_kernel(Scene<T> s, const Instance<T>* inst, int32_t n_inst, const double* X,
                                   int64_t x_base, int64_t P, const int32_t* prange, const int32_t* warm_in,
                                   int32_t* leaf_out, T* d2_out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P) return;
    const int64_t g = x_base + r;
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (inst[mid].point_begin <= g) lo = mid; else hi = mid - 1;
    }
    const StageView sv{0, -1};
    T x[D];
#pragma unroll
    for (int c = 0; c < D; ++c) x[c] = T(X[r * D + c]);
    T d2;
    QueryCount qc{0, 0, 0};
    TravStack<T, false> stack;
    int32_t warm = -1;
    if (warm_in) {
        const int32_t w = warm_in[r];
        const int64_t b = prange ? (int64_t)prange[2 * lo] : 0;
        const int64_t e = prange ? (int64_t)prange[2 * lo + 1] : s.n_prims;
        if ((int64_t)w >= b && (int64_t)w < e) warm = w;
    }
    leaf_out[r] = closest_leaf<T, D>(s, sv, inst[lo].root, x, warm, d2, qc, stack);
    d2_out[r] = d2;
}

template <class T, int D>
__global__ void ball_kernel_eval(const double* r, const double* R, int64_t n, T kappa, double* GB,
                                 double* alpha) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T RR = T(R[i]);
    const T rho = T(r[i] / R[i]);
    GB[i] = double(green_ball_t<D, T>(kappa, rho, RR));
    alpha[i] = double(poisson_scale<T, D>(kappa, RR));
}

// ---------------------------------------------------------------------------
// refit: repack primitive coordinates from new vertices, then recompute the
// child boxes of every pair node level by level, deepest first
// ---------------------------------------------------------------------------
template <class T, int D>
__global__ void pack_vertices_kernel(const double* V, int64_t nv, T* verts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv * D) return;
    verts[i] = T(V[i]);
}

template <class T, int D>
__global__ void pack_prims_kernel(const T* verts, const int32_t* pverts, const int32_t* order,
                                  int64_t np, T* prims) {
    const int64_t lp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lp >= np) return;
    const int32_t o = order[lp];
    T* dst = prims + lp * prim_scalars(D);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int32_t v = pverts[(size_t)o * D + k];
#pragma unroll
        for (int c = 0; c < D; ++c) dst[k * D + c] = verts[(size_t)v * D + c];
    }
}

// Refit one pair node per wavefront: recompute both children's boxes and
// slab offsets/thicknesses (normals kept) from the primitives in their
// leaf-order ranges.  Every node is independent, so one launch refits the tree.
template <class T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

template <class T, int D>
__global__ void __launch_bounds__(256) refit_nodes_kernel(T* nodes, const T* prims, const int32_t* ranges,
                                                          int64_t n_nodes) {
    const int64_t ni = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (ni >= n_nodes) return;
    T* p = nodes + ni * node_scalars(D);
    for (int c = 0; c < 2; ++c) {
        const int32_t b = ranges[ni * 4 + 2 * c], e = ranges[ni * 4 + 2 * c + 1];
        if (e <= b) continue;   // empty child keeps its sentinel bounds
        T* lo = p + 2 * c * D;
        T* hi = p + (2 * c + 1) * D;
        T* slab = p + slab_offset(D) + c * (D + 2);
        T n[D];
#pragma unroll
        for (int k = 0; k < D; ++k) n[k] = slab[k];
        T mn[D], mx[D], smin = T(INFINITY), smax = T(-INFINITY);
#pragma unroll
        for (int k = 0; k < D; ++k) { mn[k] = T(INFINITY); mx[k] = T(-INFINITY); }
        for (int32_t i = b + lane; i < e; i += 64) {
            const T* P = prims + (size_t)i * prim_scalars(D);
#pragma unroll
            for (int v = 0; v < D; ++v) {
                T pr = T(0);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const T x = P[v * D + k];
                    mn[k] = fmin(mn[k], x);
                    mx[k] = fmax(mx[k], x);
                    pr += n[k] * x;
                }
                smin = fmin(smin, pr);
                smax = fmax(smax, pr);
            }
        }
#pragma unroll
        for (int k = 0; k < D; ++k) { mn[k] = wave_min(mn[k]); mx[k] = wave_max(mx[k]); }
        smin = wave_min(smin);
        smax = wave_max(smax);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < D; ++k) { lo[k] = mn[k]; hi[k] = mx[k]; }
            T scale = fmax(fabs(smin), fabs(smax));
#pragma unroll
            for (int k = 0; k < D; ++k) scale += fmax(fabs(mn[k]), fabs(mx[k]));
            slab[D] = T(0.5) * (smin + smax);
            slab[D + 1] = T(0.5) * (smax - smin) + slab_pad<T>(scale);
        }
    }
}

// V_i = V_base_i + sum_{e in row i} vel_e pi_{pid_e}
template <int D>
__global__ void apply_params_kernel(const double* Vb, const int64_t* rowptr, const int32_t* pid,
                                    const double* vel, const double* pi, int64_t nv, double* V) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) v[c] = Vb[i * D + c];
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const double q = pi[pid[e]];
#pragma unroll
        for (int c = 0; c < D; ++c) v[c] += vel[e * D + c] * q;
    }
#pragma unroll
    for (int c = 0; c < D; ++c) V[i * D + c] = v[c];
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// per primitive: does any of its vertices move or carry a value parameter?
__global__ void prim_dep_kernel(const int32_t* pverts, const int32_t* vparam, int64_t np, int D,
                                int32_t* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    int dep = 0;
    for (int k = 0; k < D; ++k) dep |= vparam[pverts[i * D + k]] != 0;
    out[i] = dep;
}

__global__ void fill_f32_kernel(float* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__global__ void fill_f64_kernel(double* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace dwos
