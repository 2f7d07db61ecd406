// Shape-optimisation step for mesh vertices on gfx950: vector Adam on the
// Laplacian-preconditioned variable u = (I + lambda L) x with the step size
// set by the largest second moment over all vertices -- the optimiser the
// paper uses for vertex parameters (Sec. 6 "Implementation and evaluation",
// Sec. 7.2 "Gradient preconditioning": vector Adam of Ling et al. 2022, the
// Laplacian preconditioner and max-moment step of Nicolet et al. 2021).
//
// One step, with M = I + lambda L (L the combinatorial Laplacian over edges
// between movable vertices; a fixed vertex's row is the identity):
//   g_u = M^-1 g_x            (M is symmetric)
//   m = b1 m + (1 - b1) g_u;  v_i = b2 v_i + (1 - b2) |g_u,i|^2  (per vertex)
//   u -= lr m_hat / (sqrt(max_i v_hat_i) + eps)   (movable vertices only)
//   x = M^-1 u
// The solves are Jacobi-preconditioned conjugate gradients on the D
// coordinate systems at once (block-diagonal M (x) I_D), warm-started from
// the previous solution, with every scalar kept on the device; the host
// reads a convergence flag every kCheckEvery iterations.  An iteration is
// three launches (M p with p . q, the update with r . z, the new direction),
// each block adding the previous launch's per-block partials itself in one
// fixed order, so no launch waits on a separate reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dwos.h"
#include "host_common.hpp"

using dwos_host::DevBuf;
using dwos_host::blocks_for;
using dwos_host::fail;
using dwos_host::upload;

namespace {
constexpr int kThreads = 256;
constexpr int kRedBlocks = 512;      // partial sums of a reduction
constexpr int kCheckEvery = 16;      // CG iterations between convergence reads
// device scalars
// S_RZ, S_RZ1: r . z of the current iteration in alternating slots (iteration
// k reads slot k & 1 and leaves the next one in the other)
enum { S_RZ = 0, S_RZ1, S_RZ0, S_PQ, S_VMAX, S_DONE, S_COUNT };
}  // namespace

struct dwos_opt {
    int D = 0;
    int64_t nv = 0, nnz = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    DevBuf rowptr, col, val, diag, movable;
    DevBuf u, m, v, gu, r, z, p, q, red, scal;
    int64_t t = 0;
    bool ready = false;
};

namespace opt_k {

// y = M x for D interleaved columns: y[i D + c] = sum_k val[k] x[col[k] D + c]
__global__ void spmv(const int64_t* rowptr, const int32_t* col, const double* val, const double* x,
                     double* y, int64_t nv, int D) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const double a = val[k];
        const int64_t j = (int64_t)col[k] * D;
        for (int c = 0; c < D; ++c) acc[c] += a * x[j + c];
    }
    for (int c = 0; c < D; ++c) y[i * D + c] = acc[c];
}

// block partial sums of a . b (or of a . a / diag-weighted forms, see mode)
__device__ __forceinline__ double block_sum(double s) {
    __shared__ double sh[kThreads / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kThreads / 64; ++w) t += sh[w];
    return t;
}

__global__ void dot_partial(const double* a, const double* b, int64_t n, double* red, const double* scal) {
    if (scal[S_DONE] != 0.0) return;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += a[i] * b[i];
    s = block_sum(s);
    if (threadIdx.x == 0) red[blockIdx.x] = s;
}

__device__ __forceinline__ double final_sum(const double* red) {
    double s = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) s += red[i];
    return block_sum(s);
}

// r = b - M x, z = r / diag (per row and column)
__global__ void residual(const int64_t* rowptr, const int32_t* col, const double* val, const double* diag,
                         const double* b, const double* x, double* r, double* z, double* p, int64_t nv, int D) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const double a = val[k];
        const int64_t j = (int64_t)col[k] * D;
        for (int c = 0; c < D; ++c) acc[c] += a * x[j + c];
    }
    const double di = 1.0 / diag[i];
    for (int c = 0; c < D; ++c) {
        const double rr = b[i * D + c] - acc[c];
        r[i * D + c] = rr;
        z[i * D + c] = rr * di;
        p[i * D + c] = rr * di;
    }
}

// start: rz0 = rz = (r . z); done if r is already zero
__global__ void cg_start(const double* red, double* scal, double tol2) {
    const double s = final_sum(red);
    if (threadIdx.x == 0) {
        scal[S_RZ] = s;
        scal[S_RZ0] = s;
        scal[S_DONE] = (s <= 0.0) ? 1.0 : 0.0;
        (void)tol2;
    }
}

// The sum of red[0..n) for every thread of the block, added in the same
// order by every block.
__device__ __forceinline__ double block_total(const double* red, int64_t n) {
    __shared__ double sh[kThreads / 64];
    __shared__ double tot;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += red[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += sh[w];
        tot = t;
    }
    __syncthreads();
    return tot;
}

// The convergence flag as one value for the whole block (block 0 of a launch
// may set it while other blocks start).
__device__ __forceinline__ bool block_done(const double* scal) {
    __shared__ int d;
    if (threadIdx.x == 0) d = scal[S_DONE] != 0.0 ? 1 : 0;
    __syncthreads();
    return d != 0;
}

// One CG iteration takes three launches over blocks of kThreads rows, each
// block leaving its partial of the next dot product in red:
// q = M p with partials of p . q
__global__ void cg_spmv_dot(const int64_t* rowptr, const int32_t* col, const double* val, const double* p,
                            double* q, int64_t nv, int D, double* red_pq, const double* scal) {
    if (block_done(scal)) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (i < nv) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            const double a = val[k];
            const int64_t j = (int64_t)col[k] * D;
            for (int c = 0; c < D; ++c) acc[c] += a * p[j + c];
        }
        for (int c = 0; c < D; ++c) {
            q[i * D + c] = acc[c];
            s += p[i * D + c] * acc[c];
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) red_pq[blockIdx.x] = s;
}

// alpha = rz / (p . q); x += alpha p; r -= alpha q; z = r / diag, with
// partials of r . z (stops the solve if p . q is not positive)
__global__ void cg_update_dot(double* x, double* r, double* z, const double* p, const double* q, const double* diag,
                              int64_t nv, int D, const double* red_pq, int64_t nblk, double* red_rz, double* scal,
                              int par) {
    if (block_done(scal)) return;
    const double pq = block_total(red_pq, nblk);
    if (!(pq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_DONE] = 1.0;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_PQ] = pq;
    const double al = scal[S_RZ + par] / pq;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (i < nv) {
        const double di = 1.0 / diag[i];
        for (int c = 0; c < D; ++c) {
            const int64_t k = i * D + c;
            x[k] += al * p[k];
            const double rr = r[k] - al * q[k];
            r[k] = rr;
            const double zz = rr * di;
            z[k] = zz;
            s += rr * zz;
        }
    }
    s = block_sum(s);
    if (threadIdx.x == 0) red_rz[blockIdx.x] = s;
}

// beta = rz_new / rz; p = z + beta p; converged when rz_new <= tol^2 rz0
__global__ void cg_direction_beta(double* p, const double* z, int64_t nv, int D, const double* red_rz, int64_t nblk,
                                  double* scal, int par, double tol2) {
    if (block_done(scal)) return;
    const double rzn = block_total(red_rz, nblk);
    const double rz = scal[S_RZ + par];
    const double beta = rz > 0.0 ? rzn / rz : 0.0;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scal[S_RZ + (par ^ 1)] = rzn;
        if (rzn <= tol2 * scal[S_RZ0]) scal[S_DONE] = 1.0;
    }
    if (i >= nv) return;
    for (int c = 0; c < D; ++c) p[i * D + c] = z[i * D + c] + beta * p[i * D + c];
}

// moments of the vector Adam step; partial maxima of v_hat over movable vertices
__global__ void adam_moments(const double* g, double* m, double* v, const int32_t* movable, int64_t nv, int D,
                             double b1, double b2, double c2, double* red) {
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        if (!movable[i]) continue;
        double g2 = 0.0;
        for (int c = 0; c < D; ++c) {
            const double gc = g[i * D + c];
            m[i * D + c] = b1 * m[i * D + c] + (1.0 - b1) * gc;
            g2 += gc * gc;
        }
        const double vi = b2 * v[i] + (1.0 - b2) * g2;
        v[i] = vi;
        mx = fmax(mx, vi / c2);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    __shared__ double sh[kThreads / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t = fmax(t, sh[w]);
        red[blockIdx.x] = t;
    }
}

__global__ void max_final(const double* red, double* scal) {
    double mx = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) mx = fmax(mx, red[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    __shared__ double sh[kThreads / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t = fmax(t, sh[w]);
        scal[S_VMAX] = t;
    }
}

__global__ void adam_update(double* u, const double* m, const int32_t* movable, int64_t nv, int D, double lr,
                            double c1, double eps, const double* scal) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv || !movable[i]) return;
    const double s = lr / (c1 * (sqrt(scal[S_VMAX]) + eps));
    for (int c = 0; c < D; ++c) u[i * D + c] -= s * m[i * D + c];
}

__global__ void fill(double* a, int64_t n, double v) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) a[k] = v;
}

__global__ void copy(double* dst, const double* src, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[k];
}

}  // namespace opt_k

namespace {

// x := M^-1 b by preconditioned CG from the current x.  iters: used.
dwos_status cg_solve(dwos_opt* o, const double* b, double* x, int32_t max_iters, double tol, int32_t* iters) {
    hipStream_t s = o->stream;
    const int64_t nv = o->nv, n = nv * o->D;
    const int D = o->D;
    double* red = o->red.as<double>();
    const int64_t nblk = blocks_for(nv, kThreads);
    double* red_pq = red + kRedBlocks;   // per-block partials of the iteration's dot products
    double* red_rz = red_pq + nblk;
    double* sc = o->scal.as<double>();
    const int64_t* rp = o->rowptr.as<int64_t>();
    const int32_t* cl = o->col.as<int32_t>();
    const double* va = o->val.as<double>();
    const double* dg = o->diag.as<double>();
    double *r = o->r.as<double>(), *z = o->z.as<double>(), *p = o->p.as<double>(), *q = o->q.as<double>();
    const double tol2 = tol * tol;
    hipLaunchKernelGGL(opt_k::fill, dim3(1), dim3(64), 0, s, sc, (int64_t)S_COUNT, 0.0);
    hipLaunchKernelGGL(opt_k::residual, dim3(blocks_for(nv, kThreads)), dim3(kThreads), 0, s, rp, cl, va, dg, b, x,
                       r, z, p, nv, D);
    hipLaunchKernelGGL(opt_k::dot_partial, dim3(kRedBlocks), dim3(kThreads), 0, s, r, z, n, red, sc);
    hipLaunchKernelGGL(opt_k::cg_start, dim3(1), dim3(kThreads), 0, s, red, sc, tol2);
    int32_t it = 0;
    for (; it < max_iters; ++it) {
        if (it % kCheckEvery == 0) {
            double done = 0.0;
            HIP_OK(hipMemcpyAsync(&done, sc + S_DONE, sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
            if (done != 0.0) break;
        }
        const int par = it & 1;
        hipLaunchKernelGGL(opt_k::cg_spmv_dot, dim3(nblk), dim3(kThreads), 0, s, rp, cl, va, p, q, nv, D, red_pq, sc);
        hipLaunchKernelGGL(opt_k::cg_update_dot, dim3(nblk), dim3(kThreads), 0, s, x, r, z, p, q, dg, nv, D, red_pq,
                           nblk, red_rz, sc, par);
        hipLaunchKernelGGL(opt_k::cg_direction_beta, dim3(nblk), dim3(kThreads), 0, s, p, z, nv, D, red_rz, nblk, sc,
                           par, tol2);
    }
    HIP_OK(hipGetLastError());
    if (iters) *iters = it;
    return DWOS_OK;
}

dwos_status check_opt(dwos_opt* o) {
    if (!o) return fail(DWOS_EINVAL, "NULL optimiser");
    if (!o->ready) return fail(DWOS_ESTATE, "optimiser: call dwos_opt_reset first");
    return DWOS_OK;
}

}  // namespace

extern "C" {

dwos_status dwos_opt_create(int32_t dim, int64_t nv, const int32_t* prims, int64_t np, const int32_t* movable,
                            double lambda, void* stream, dwos_opt** out) {
    if (!out) return fail(DWOS_EINVAL, "opt_create: NULL output");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(DWOS_EINVAL, "opt_create: dim must be 2 or 3");
    if (nv <= 0 || nv > INT32_MAX || np < 0 || (np > 0 && !prims))
        return fail(DWOS_EINVAL, "opt_create: bad mesh sizes");
    if (!(lambda >= 0) || !std::isfinite(lambda)) return fail(DWOS_EINVAL, "opt_create: lambda must be >= 0");
    for (int64_t i = 0; i < np * dim; ++i)
        if (prims[i] < 0 || prims[i] >= nv) return fail(DWOS_EINVAL, "opt_create: vertex index out of range");
    std::vector<int32_t> mv(nv, 1);
    if (movable)
        for (int64_t i = 0; i < nv; ++i) mv[i] = movable[i] ? 1 : 0;
    // undirected edges between movable vertices
    std::vector<std::pair<int32_t, int32_t>> e;
    const int ne = dim == 2 ? 1 : 3;
    for (int64_t f = 0; f < np; ++f)
        for (int k = 0; k < ne; ++k) {
            int32_t a = prims[f * dim + k], b = prims[f * dim + (dim == 2 ? 1 : (k + 1) % 3)];
            if (a == b || !mv[a] || !mv[b]) continue;
            if (a > b) std::swap(a, b);
            e.emplace_back(a, b);
        }
    std::sort(e.begin(), e.end());
    e.erase(std::unique(e.begin(), e.end()), e.end());
    // M = I + lambda (Deg - Adj), CSR with the diagonal first in each row
    std::vector<std::vector<int32_t>> adj(nv);
    for (auto& pr : e) { adj[pr.first].push_back(pr.second); adj[pr.second].push_back(pr.first); }
    std::vector<int64_t> rowptr(nv + 1, 0);
    std::vector<int32_t> col;
    std::vector<double> val, diag(nv);
    for (int64_t i = 0; i < nv; ++i) {
        std::sort(adj[i].begin(), adj[i].end());
        diag[i] = 1.0 + lambda * (double)adj[i].size();
        col.push_back((int32_t)i);
        val.push_back(diag[i]);
        for (int32_t j : adj[i]) { col.push_back(j); val.push_back(-lambda); }
        rowptr[i + 1] = (int64_t)col.size();
    }
    auto* o = new dwos_opt();
    o->D = dim;
    o->nv = nv;
    o->nnz = (int64_t)col.size();
    o->stream = static_cast<hipStream_t>(stream);
    hipError_t he = hipGetDevice(&o->device);
    if (he != hipSuccess) { delete o; return fail(DWOS_EDEVICE, std::string("opt_create: ") + hipGetErrorString(he)); }
    auto up = [&]() -> dwos_status {
        hipStream_t s = o->stream;
        HIP_OK(upload(o->rowptr, rowptr.data(), rowptr.size(), s));
        HIP_OK(upload(o->col, col.data(), col.size(), s));
        HIP_OK(upload(o->val, val.data(), val.size(), s));
        HIP_OK(upload(o->diag, diag.data(), diag.size(), s));
        HIP_OK(upload(o->movable, mv.data(), mv.size(), s));
        const size_t vb = (size_t)nv * dim * sizeof(double);
        for (DevBuf* b : {&o->u, &o->m, &o->gu, &o->r, &o->z, &o->p, &o->q}) HIP_OK(b->reserve(vb));
        HIP_OK(o->v.reserve((size_t)nv * sizeof(double)));
        HIP_OK(o->red.reserve((kRedBlocks + 2 * blocks_for(nv, kThreads)) * sizeof(double)));
        HIP_OK(o->scal.reserve(S_COUNT * sizeof(double)));
        return DWOS_OK;
    };
    dwos_status st = up();
    if (st) { delete o; return st; }
    *out = o;
    return DWOS_OK;
}

void dwos_opt_destroy(dwos_opt* o) {
    if (!o) return;
    (void)hipStreamSynchronize(o->stream);
    delete o;
}

dwos_status dwos_opt_reset(dwos_opt* o, const double* x) {
    if (!o) return fail(DWOS_EINVAL, "NULL optimiser");
    if (!x) return fail(DWOS_EINVAL, "opt_reset: NULL vertices");
    HIP_OK(hipSetDevice(o->device));
    hipStream_t s = o->stream;
    const int64_t n = o->nv * o->D;
    hipLaunchKernelGGL(opt_k::spmv, dim3(blocks_for(o->nv, kThreads)), dim3(kThreads), 0, s, o->rowptr.as<int64_t>(),
                       o->col.as<int32_t>(), o->val.as<double>(), x, o->u.as<double>(), o->nv, o->D);
    hipLaunchKernelGGL(opt_k::fill, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, o->m.as<double>(), n, 0.0);
    hipLaunchKernelGGL(opt_k::fill, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, o->gu.as<double>(), n, 0.0);
    hipLaunchKernelGGL(opt_k::fill, dim3(blocks_for(o->nv, kThreads)), dim3(kThreads), 0, s, o->v.as<double>(),
                       o->nv, 0.0);
    HIP_OK(hipGetLastError());
    o->t = 0;
    o->ready = true;
    return DWOS_OK;
}

dwos_status dwos_opt_solve(dwos_opt* o, const double* b, double* x, int32_t max_iters, double tol, int32_t* iters) {
    if (!o) return fail(DWOS_EINVAL, "NULL optimiser");
    if (!b || !x || max_iters < 0 || !(tol >= 0)) return fail(DWOS_EINVAL, "opt_solve: bad arguments");
    HIP_OK(hipSetDevice(o->device));
    return cg_solve(o, b, x, max_iters, tol, iters);
}

dwos_status dwos_opt_step(dwos_opt* o, const double* gx, double* x, double lr, double beta1, double beta2,
                          double eps, int32_t max_iters, double tol, int32_t* iters) {
    dwos_status st = check_opt(o);
    if (st) return st;
    if (!gx || !x || max_iters < 0 || !(tol >= 0) || !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) ||
        !(beta2 >= 0 && beta2 < 1) || !(eps >= 0))
        return fail(DWOS_EINVAL, "opt_step: bad arguments");
    HIP_OK(hipSetDevice(o->device));
    hipStream_t s = o->stream;
    int32_t it[2] = {0, 0};
    // g_u = M^-1 g_x, warm-started from the previous g_u
    st = cg_solve(o, gx, o->gu.as<double>(), max_iters, tol, &it[0]);
    if (st) return st;
    o->t += 1;
    const double c1 = 1.0 - std::pow(beta1, (double)o->t), c2 = 1.0 - std::pow(beta2, (double)o->t);
    hipLaunchKernelGGL(opt_k::adam_moments, dim3(kRedBlocks), dim3(kThreads), 0, s, o->gu.as<double>(),
                       o->m.as<double>(), o->v.as<double>(), o->movable.as<int32_t>(), o->nv, o->D, beta1, beta2, c2,
                       o->red.as<double>());
    hipLaunchKernelGGL(opt_k::max_final, dim3(1), dim3(kThreads), 0, s, o->red.as<double>(), o->scal.as<double>());
    hipLaunchKernelGGL(opt_k::adam_update, dim3(blocks_for(o->nv, kThreads)), dim3(kThreads), 0, s, o->u.as<double>(),
                       o->m.as<double>(), o->movable.as<int32_t>(), o->nv, o->D, lr, c1, eps, o->scal.as<double>());
    HIP_OK(hipGetLastError());
    // x = M^-1 u, warm-started from the current x
    st = cg_solve(o, o->u.as<double>(), x, max_iters, tol, &it[1]);
    if (st) return st;
    if (iters) { iters[0] = it[0]; iters[1] = it[1]; }
    return DWOS_OK;
}

}  // extern "C"
