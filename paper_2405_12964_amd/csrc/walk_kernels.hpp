// Walk kernels for (differential) walk on spheres on gfx950.
//
// One walk per lane.  The walk kernel is persistent: each wavefront takes
// chunks of logical walk ids from a global atomic counter and hands a new
// walk to every lane whose walk has ended (ballot + prefix count), so lanes
// stay busy while walk lengths differ.  Each loop iteration performs exactly
// one closest-point query per active lane (one "walk step") followed by the
// step logic of Algorithm 1 (forward) or Algorithm 2 (differential, with K
// nested forward walks at the terminal point), written as a state machine.
//
// Outputs are per-walk records indexed by the logical walk id p*W + m; small
// follow-up kernels reduce them (per-point statistics, reverse-mode scatter,
// parameter-space SpMV), so results do not depend on scheduling.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <climits>

#include "bvh.hpp"
#include "device_math.hpp"

namespace dwos {

#ifndef DWOS_BLOCK
#define DWOS_BLOCK 256
#endif
// Default scheduling knobs of the walk kernels (a context may change them
// at run time, e.g. through the autotuner).
// park: a wavefront stops traversing once this many of its lanes have their
// query answered; they take their walk step while the others resume later.
#ifndef DWOS_PARK
#define DWOS_PARK 24
#endif
constexpr int kParkLanes = DWOS_PARK;

#ifndef DWOS_LDS_STACK
#define DWOS_LDS_STACK 0
#endif
constexpr int kBlock = DWOS_BLOCK;          // threads per walk-kernel block
#ifndef DWOS_BLOCK_STAGED
#define DWOS_BLOCK_STAGED 1024
#endif
constexpr int kBlockStaged = DWOS_BLOCK_STAGED;  // block of the LDS-staged walk kernel
constexpr bool kLdsStack = DWOS_LDS_STACK;  // traversal stack in LDS (else private memory)
constexpr int kMaxLabels = 16;
constexpr int kMaxGauss = 8;
constexpr uint32_t kQueueChunk = 128;   // default walk ids taken per wavefront refill

template <class T>
struct Params {
    int K, kmax, rr, n_gauss, n_labels, has_source;
    T src_c0;
    T gauss[kMaxGauss][5];
    int kind[kMaxLabels];
    T gc[kMaxLabels];
    T gb[kMaxLabels][3];
    T gA[kMaxLabels][9];
};

// Per-instance constants (a plain solve has one instance).
template <class T>
struct Instance {
    int64_t walk_begin;   // first logical walk id of the instance
    int64_t point_begin;  // first point (row of X) of the instance
    int64_t p_counter;    // added to the point index inside the instance to
                          // form the Philox point word (chunked solves)
    int32_t root;         // root pair node
    int32_t P;            // points of the instance
    T kappa, eps, delta;
};

template <class T>
struct Scene {
    const T* nodes;          // pair nodes
    const T* prims;          // leaf-order primitive coordinates
    const int32_t* orig;     // leaf position -> original primitive
    const T* verts;          // vertices (original order), nv x D
    const int32_t* pverts;   // original primitive -> vertex ids, np x D
    const int32_t* label;    // original primitive -> label
    const T* gvert;          // per-vertex values of mapped labels
    int32_t n_stage_nodes;   // nodes to stage in LDS (staged kernels)
    int32_t stage_prims;     // 1: stage every primitive as well
    int64_t n_prims;
    int32_t tail;            // descending lanes a query round leaves to the
                             // next round (0: none), see query_round
};

struct Counters {   // device-side statistics (int64 atomics)
    unsigned long long walks, nested, steps, terminal, truncated, nodes, prims, overflow, invalid;
};

template <class T>
struct WalkArgs {
    Scene<T> s;
    Params<T> prm;
    const Instance<T>* inst;
    int32_t n_inst;
    const double* X;         // points, rows point_begin.. of each instance
    int32_t W;
    int64_t total;           // walks in this launch
    int64_t wid_offset;      // logical id of walk 0 of this launch
    uint32_t key0, key1;
    const unsigned long long* seed_ptr;   // if set, the key is seed + *seed_ptr
    unsigned long long* queue;
    int32_t park;            // lanes answered before a wavefront takes its step (1..64)
    uint32_t chunk;          // walk ids taken per wavefront refill (multiple of 64)
    Counters* cnt;           // this call
    Counters* tot;           // cumulative for this walk kind
    // records (indexed by logical id - wid_offset)
    T* rec_u;
    int32_t* rec_prim;       // orig*2 + flip, -1 when stopped by roulette
    T* rec_b;                // barycentrics b1 (2D) or b1,b2 (3D)
    T* rec_uoff;             // mean of the nested walks
    int64_t* rec_steps;      // optional per-walk query count
    T* rec_w;                // walk-on-stars differential walks with a Robin
                             // condition: the throughput at the terminal (null: 1)
    // closest primitive of every start point (all walks of a point share
    // their first query), indexed by X row - x_base; null: query per walk
    const int32_t* first_leaf;
    const T* first_d2;
    int64_t x_base;
    // scheduling order of the points (slot -> point of the chunk), or null
    // for the identity; only for a single instance with wid_offset 0
    const int32_t* perm;
    // control variate of the nested walks (MODE 1; cv_run == nullptr: off).
    // Per walk: cv_run (-1 no terminal, 0 nested walks skipped, 1 run),
    // the offset point, the terminal point and g there.  Per nested walk
    // (walk-major, K per walk): the stop point, the reservoir-chosen ball
    // sample y = x_J + rho d_J dir, S and alive (alive:
    // ended in the shell or at the cap rather than by roulette).
    // S: the walk's total Green's-function mass over its source steps; the
    // ball sample is taken in the step chosen with probability m_j / S.
    int32_t* cv_run;
    // per original primitive: 1 if a vertex moves or carries a value
    // parameter; the nested walks of a terminal on any other primitive are
    // skipped (their mean enters every derivative times V_n = 0 and
    // gdot = 0) and reported as g.  NULL: run everywhere.
    const int32_t* prim_dep;
    T* cv_xoff;
    T* cv_xbar;
    T* cv_g;
    T* cv_stop;
    T* cv_y;
    T* cv_rho;
    T* cv_d;
    T* cv_S;
    int32_t* cv_alive;
    uint32_t cv_qthresh;     // nested walks run iff (u32 >> 8) < cv_qthresh; 1 << 24: always
};

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
template <class T> struct Slack;
template <> struct Slack<float> { static constexpr float v = 1.00001f; };
template <> struct Slack<double> { static constexpr double v = 1.000000000001; };
// Relative band within which two squared distances count as a tie (shared
// edges and vertices); ties keep the lowest original primitive index.
template <class T> struct TieBand;
template <> struct TieBand<float> { static constexpr float v = 0.0f; };
template <> struct TieBand<double> { static constexpr double v = 1e-12; };

template <class T, int D>
__device__ __forceinline__ T box_d2(const T* lo, const T* hi, const T* x) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const T e = fmax(fmax(lo[i] - x[i], x[i] - hi[i]), T(0));
        s += e * e;
    }
    return s;
}

// Closest point on a segment (2D) or triangle (3D) with its barycentrics.
// Triangle: classify the query against the vertex, edge and face Voronoi
// regions using the dot products of the query offset with the two edges
// (the classical region test, e.g. Ericson, Real-Time Collision Detection
// Sec. 5.1.5).
// a / b in the walk precision: FP32 uses the hardware reciprocal (1 ulp),
// FP64 (the walk-for-walk reference build) the correctly rounded division
template <class T>
__device__ __forceinline__ T quot(T a, T b) {
    if constexpr (sizeof(T) == 4) return a * __builtin_amdgcn_rcpf(b);
    else return a / b;
}

template <class T, int D>
__device__ __forceinline__ T prim_closest(const T* P, const T* x, T* bary) {
    if constexpr (D == 2) {
        const T ex = P[2] - P[0], ey = P[3] - P[1];
        const T ax = x[0] - P[0], ay = x[1] - P[1];
        const T L2 = ex * ex + ey * ey;
        T t = L2 > T(0) ? quot<T>(ax * ex + ay * ey, L2) : T(0);
        t = fmin(fmax(t, T(0)), T(1));
        const T dx = ax - t * ex, dy = ay - t * ey;
        bary[0] = T(1) - t; bary[1] = t; bary[2] = T(0);
        return dx * dx + dy * dy;
    } else {
        const T ab[3] = {P[3] - P[0], P[4] - P[1], P[5] - P[2]};
        const T ac[3] = {P[6] - P[0], P[7] - P[1], P[8] - P[2]};
        const T ap[3] = {x[0] - P[0], x[1] - P[1], x[2] - P[2]};
        const T d1 = ab[0] * ap[0] + ab[1] * ap[1] + ab[2] * ap[2];
        const T d2 = ac[0] * ap[0] + ac[1] * ap[1] + ac[2] * ap[2];
        T v, w;
        if (d1 <= T(0) && d2 <= T(0)) { v = T(0); w = T(0); }
        else {
            const T bp[3] = {x[0] - P[3], x[1] - P[4], x[2] - P[5]};
            const T d3 = ab[0] * bp[0] + ab[1] * bp[1] + ab[2] * bp[2];
            const T d4 = ac[0] * bp[0] + ac[1] * bp[1] + ac[2] * bp[2];
            if (d3 >= T(0) && d4 <= d3) { v = T(1); w = T(0); }
            else {
                const T vc = d1 * d4 - d3 * d2;
                if (vc <= T(0) && d1 >= T(0) && d3 <= T(0)) { v = quot<T>(d1, d1 - d3); w = T(0); }
                else {
                    const T cp[3] = {x[0] - P[6], x[1] - P[7], x[2] - P[8]};
                    const T d5 = ab[0] * cp[0] + ab[1] * cp[1] + ab[2] * cp[2];
                    const T d6 = ac[0] * cp[0] + ac[1] * cp[1] + ac[2] * cp[2];
                    if (d6 >= T(0) && d5 <= d6) { v = T(0); w = T(1); }
                    else {
                        const T vb = d5 * d2 - d1 * d6;
                        if (vb <= T(0) && d2 >= T(0) && d6 <= T(0)) { v = T(0); w = quot<T>(d2, d2 - d6); }
                        else {
                            const T va = d3 * d6 - d5 * d4;
                            if (va <= T(0) && (d4 - d3) >= T(0) && (d5 - d6) >= T(0)) {
                                w = quot<T>(d4 - d3, (d4 - d3) + (d5 - d6));
                                v = T(1) - w;
                            } else {
                                const T den = quot<T>(T(1), va + vb + vc);
                                v = vb * den;
                                w = vc * den;
                            }
                        }
                    }
                }
            }
        }
        bary[0] = T(1) - v - w; bary[1] = v; bary[2] = w;
        const T q0 = ap[0] - v * ab[0] - w * ac[0];
        const T q1 = ap[1] - v * ab[1] - w * ac[1];
        const T q2 = ap[2] - v * ab[2] - w * ac[2];
        return q0 * q0 + q1 * q1 + q2 * q2;
    }
}

template <class T, int D>
__device__ __forceinline__ void load_prim(const T* prims, int32_t i, T* P) {
    const T* p = prims + (size_t)i * prim_scalars(D);
    if constexpr (sizeof(T) == 4 && D == 2) {
        const float4 a = *reinterpret_cast<const float4*>(p);
        P[0] = a.x; P[1] = a.y; P[2] = a.z; P[3] = a.w;
    } else if constexpr (sizeof(T) == 4 && D == 3) {
        const float4 a = reinterpret_cast<const float4*>(p)[0];
        const float4 b = reinterpret_cast<const float4*>(p)[1];
        const float4 c = reinterpret_cast<const float4*>(p)[2];
        P[0] = a.x; P[1] = a.y; P[2] = a.z; P[3] = a.w; P[4] = b.x; P[5] = b.y;
        P[6] = b.z; P[7] = b.w; P[8] = c.x;
    } else {
#pragma unroll
        for (int k = 0; k < D * D; ++k) P[k] = p[k];
    }
}

template <class T, int D>
struct NodeData {
    T lo0[D], hi0[D], lo1[D], hi1[D];
    T n0[D], n1[D];
    T o0, t0, o1, t1;
    int32_t c0, c1;
};

// decode a node from 16-byte words (FP32 layout of bvh.hpp)
template <int D>
__device__ __forceinline__ void decode_node_f32(const float4* q, NodeData<float, D>& nd) {
    if constexpr (D == 2) {
        const float4 a = q[0], b = q[1], c = q[2], d = q[3], e = q[4];
        nd.lo0[0] = a.x; nd.lo0[1] = a.y; nd.hi0[0] = a.z; nd.hi0[1] = a.w;
        nd.lo1[0] = b.x; nd.lo1[1] = b.y; nd.hi1[0] = b.z; nd.hi1[1] = b.w;
        nd.n0[0] = c.x; nd.n0[1] = c.y; nd.o0 = c.z; nd.t0 = c.w;
        nd.n1[0] = d.x; nd.n1[1] = d.y; nd.o1 = d.z; nd.t1 = d.w;
        nd.c0 = __float_as_int(e.x); nd.c1 = __float_as_int(e.y);
    } else {
        const float4 a = q[0], b = q[1], c = q[2], d = q[3], e = q[4], f = q[5];
        nd.lo0[0] = a.x; nd.lo0[1] = a.y; nd.lo0[2] = a.z; nd.hi0[0] = a.w;
        nd.hi0[1] = b.x; nd.hi0[2] = b.y; nd.lo1[0] = b.z; nd.lo1[1] = b.w;
        nd.lo1[2] = c.x; nd.hi1[0] = c.y; nd.hi1[1] = c.z; nd.hi1[2] = c.w;
        nd.n0[0] = d.x; nd.n0[1] = d.y; nd.n0[2] = d.z; nd.o0 = d.w;
        nd.t0 = e.x; nd.n1[0] = e.y; nd.n1[1] = e.z; nd.n1[2] = e.w;
        nd.o1 = f.x; nd.t1 = f.y; nd.c0 = __float_as_int(f.z); nd.c1 = __float_as_int(f.w);
    }
}

template <class T, int D>
__device__ __forceinline__ void load_node(const T* nodes, int32_t i, NodeData<T, D>& nd) {
    const T* p = nodes + (size_t)i * node_scalars(D);
    if constexpr (sizeof(T) == 4) {
        decode_node_f32<D>(reinterpret_cast<const float4*>(p), nd);
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            nd.lo0[k] = p[k]; nd.hi0[k] = p[D + k]; nd.lo1[k] = p[2 * D + k]; nd.hi1[k] = p[3 * D + k];
            nd.n0[k] = p[4 * D + k]; nd.n1[k] = p[5 * D + 2 + k];
        }
        nd.o0 = p[5 * D]; nd.t0 = p[5 * D + 1]; nd.o1 = p[6 * D + 2]; nd.t1 = p[6 * D + 3];
        const int32_t* r = reinterpret_cast<const int32_t*>(p + ref_offset(D));
        nd.c0 = r[0]; nd.c1 = r[1];
    }
}

template <class T>
__device__ __forceinline__ T slab_pad(T scale) {
    return T(16) * (sizeof(T) == 4 ? T(5.9604644775390625e-08) : T(1.1102230246251565e-16)) * scale;
}

// squared distance from x to the slab {y : |n.y - o| <= t}
template <class T, int D>
__device__ __forceinline__ T slab_d2(const T* n, T o, T t, const T* x) {
    T pr = -o;
#pragma unroll
    for (int i = 0; i < D; ++i) pr += n[i] * x[i];
    const T e = fmax(fabs(pr) - t, T(0));
    return e * e;
}

// Dynamic LDS of the staged walk kernel: the first n_lnodes pair nodes, then
// (optionally) every primitive, as 16-byte words.
extern __shared__ float4 g_stage[];

// Where a traversal reads nodes and primitives: LDS below the staged prefix,
// global memory otherwise.  prim_off4 < 0: primitives stay in global memory.
struct StageView {
    int32_t n_lnodes;
    int64_t prim_off4;
};

template <class T, int D>
__device__ __forceinline__ void scene_node(const Scene<T>& s, const StageView& v, int32_t i,
                                           NodeData<T, D>& nd) {
    if constexpr (sizeof(T) == 4) {
        if (i < v.n_lnodes) {
            decode_node_f32<D>(g_stage + (int64_t)i * (node_scalars(D) / 4), nd);
            return;
        }
    }
    load_node<T, D>(s.nodes, i, nd);
}

template <class T, int D>
__device__ __forceinline__ void scene_prim(const Scene<T>& s, const StageView& v, int32_t i, T* P) {
    if constexpr (sizeof(T) == 4) {
        if (v.prim_off4 >= 0) {
            const float4* q = g_stage + v.prim_off4 + (int64_t)i * (prim_scalars(D) / 4);
            if constexpr (D == 2) {
                const float4 a = q[0];
                P[0] = a.x; P[1] = a.y; P[2] = a.z; P[3] = a.w;
            } else {
                const float4 a = q[0], b = q[1], c = q[2];
                P[0] = a.x; P[1] = a.y; P[2] = a.z; P[3] = a.w; P[4] = b.x; P[5] = b.y;
                P[6] = b.z; P[7] = b.w; P[8] = c.x;
            }
            return;
        }
    }
    load_prim<T, D>(s.prims, i, P);
}

struct QueryCount { unsigned int nodes, prims, overflow; };

// Traversal stack of (node, squared box distance) entries: per-lane private
// arrays, or a slice of LDS interleaved across the block's lanes.
template <class T, bool LDS> struct TravStack;
template <class T> struct TravStack<T, false> {
    int32_t node[kStackSize];
    T d[kStackSize];
    __device__ __forceinline__ void put(int i, int32_t n, T v) { node[i] = n; d[i] = v; }
    __device__ __forceinline__ int32_t get_node(int i) const { return node[i]; }
    __device__ __forceinline__ T get_d(int i) const { return d[i]; }
};
template <class T> struct TravStack<T, true> {
    int32_t* node;   // node[i * kBlock]
    T* d;
    __device__ __forceinline__ void put(int i, int32_t n, T v) { node[i * kBlock] = n; d[i * kBlock] = v; }
    __device__ __forceinline__ int32_t get_node(int i) const { return node[i * kBlock]; }
    __device__ __forceinline__ T get_d(int i) const { return d[i * kBlock]; }
};

// DistanceToBoundary: nearest primitive to x through the pair-node BVH, as a
// resumable query so that a wavefront can stop traversing when enough of its
// lanes have their answer (see walk_kernel).  The query starts from the upper
// bound given by a previously closest primitive (`warm`, leaf position, or
// -1): the new closest point can only be at that distance or nearer, so the
// result is unchanged while most of the tree is pruned.  Ties go to the
// lowest original primitive index.
//
// One round alternates two phases over the wavefront: expand nodes until
// every lane holds a leaf or has finished, then test the held leaves
// together, so that node and primitive work are not interleaved within one
// iteration.
// The traversal stack's R most recent entries are kept in registers (rn,
// rd; rn[0] the newest); a push moves the oldest of them to the stack
// memory only when all are in use, and a pop reads memory only when none is
// left.  Depth-first descent alternates pushes and pops, so most entries
// never reach memory (the stack's order is unchanged).  R = 8 in 2D: the
// star's differential launch writes 0.56 GB of stack instead of 6.1 GB at
// R = 3, for 4% more time; R = 5 in 3D, as fast as 3 on the icosphere (at
// 8 the 3D kernel spills and slows by 6-8%).
#ifndef DWOS_STACK_REGS_2D
#define DWOS_STACK_REGS_2D 8
#endif
#ifndef DWOS_STACK_REGS_3D
#define DWOS_STACK_REGS_3D 5
#endif
template <class T, int D>
struct Query {
    static constexpr int R = D == 2 ? DWOS_STACK_REGS_2D : DWOS_STACK_REGS_3D;
    T best;          // squared distance of the best primitive so far
    int32_t bleaf;   // its leaf position, -1 none
    int32_t node;    // internal node to expand next, or -1 (pop)
    int32_t leaf;    // held leaf reference
    int32_t sp;      // entries in stack memory
    int32_t rt;      // register-held entries in use
    int32_t rn[R];   // register-held entries: node reference
    T rd[R];         // ... and squared bound distance
    bool has_leaf, done;
};

template <class T, int D>
__device__ __forceinline__ void query_test_prim(const Scene<T>& s, const StageView& sv, const T* x,
                                                int32_t i, Query<T, D>& q, QueryCount& qc) {
    T P[9], bb[3];
    scene_prim<T, D>(s, sv, i, P);
    const T d2 = prim_closest<T, D>(P, x, bb);
    qc.prims++;
    if (d2 < q.best * (T(1) - TieBand<T>::v)) { q.best = d2; q.bleaf = i; }
    else if (d2 <= q.best * (T(1) + TieBand<T>::v) && i != q.bleaf && q.bleaf >= 0 &&
             s.orig[i] < s.orig[q.bleaf]) {
        q.best = d2;
        q.bleaf = i;
    }
}

template <class T, int D>
__device__ __forceinline__ void query_begin(const Scene<T>& s, const StageView& sv, int32_t root,
                                            const T* x, int32_t warm, Query<T, D>& q) {
    q.best = T(INFINITY);
    q.bleaf = -1;
    if (warm >= 0) {
        T P[9], bb[3];
        scene_prim<T, D>(s, sv, warm, P);
        q.best = prim_closest<T, D>(P, x, bb);
        q.bleaf = warm;
    }
    q.node = root;
    q.leaf = 0;
    q.sp = 0;
    q.has_leaf = false;
    q.done = false;
    q.rt = 0;
}

// One round for the lanes with `active` set (a query in progress).
// Phase 1 ends when no lane is descending, or (s.tail > 0) when at most
// s.tail lanes are still descending while some lane holds a leaf for
// phase 2; the descending lanes keep their position and go on in the next
// round.  A round in which no lane holds a leaf always expands at least one
// node per descending lane, so every query progresses.
// Measured on the 200,000-triangle icosphere (65536 points x 1024 walks):
// a tail of 8 lanes cuts the forward launch from 150 to 124 ms and the
// differential launch from 171 to 141 ms (tails of 4 to 24 lanes give
// 123-129 / 140-146 ms); on the 4096-gon star the differential launch goes
// from 60 to 49 ms.  With three register-held stack entries instead of two
// the icosphere launches take a further 1-2% less.
#ifndef DWOS_DESCEND_TAIL
#define DWOS_DESCEND_TAIL 8
#endif
constexpr int kDescendTail = DWOS_DESCEND_TAIL;
template <class T, int D, class Stack>
__device__ __forceinline__ void query_round(const Scene<T>& s, const StageView& sv, const T* x, bool active,
                                            Query<T, D>& q, QueryCount& qc, Stack& st) {
    using Q = Query<T, D>;
    constexpr T slack = Slack<T>::v;
    // phase 1: expand nodes until this lane holds a leaf or is finished
#pragma unroll 1
    while (true) {
        const bool go = active && !q.has_leaf && !q.done;
        if (s.tail > 0) {
            const unsigned long long gm = __ballot(go);
            if (gm == 0ull) break;
            if (__popcll(gm) <= s.tail && __ballot(active && q.has_leaf) != 0ull) break;
            if (!go) continue;
        } else if (!go) {
            break;
        }
        int32_t cur = q.node;
        if (cur < 0) {
            T dd;
            if (q.rt > 0) {
                cur = q.rn[0];
                dd = q.rd[0];
#pragma unroll
                for (int i = 0; i + 1 < Q::R; ++i) { q.rn[i] = q.rn[i + 1]; q.rd[i] = q.rd[i + 1]; }
                --q.rt;
            } else {
                if (q.sp == 0) { q.done = true; continue; }
                --q.sp;
                cur = st.get_node(q.sp);
                dd = st.get_d(q.sp);
            }
            if (dd > q.best * slack) continue;
            if (cur < 0) { q.leaf = cur; q.has_leaf = true; continue; }   // a postponed leaf
        }
        NodeData<T, D> nd;
        scene_node<T, D>(s, sv, cur, nd);
        qc.nodes++;
        const T d0 = fmax(box_d2<T, D>(nd.lo0, nd.hi0, x), slab_d2<T, D>(nd.n0, nd.o0, nd.t0, x));
        const T d1 = fmax(box_d2<T, D>(nd.lo1, nd.hi1, x), slab_d2<T, D>(nd.n1, nd.o1, nd.t1, x));
        const T lim = q.best * slack;
        const bool h0 = d0 <= lim, h1 = d1 <= lim;
        const bool near0 = d0 <= d1;
        int32_t next = -1;
        if (h0 && h1) {
            if (q.sp + q.rt < kStackSize) {
                if (q.rt == Q::R) {
                    st.put(q.sp, q.rn[Q::R - 1], q.rd[Q::R - 1]);
                    ++q.sp;
                }
#pragma unroll
                for (int i = Q::R - 1; i > 0; --i) { q.rn[i] = q.rn[i - 1]; q.rd[i] = q.rd[i - 1]; }
                q.rn[0] = near0 ? nd.c1 : nd.c0;
                q.rd[0] = near0 ? d1 : d0;
                q.rt = q.rt < Q::R ? q.rt + 1 : Q::R;
            } else {
                qc.overflow++;
            }
            next = near0 ? nd.c0 : nd.c1;
        } else if (h0) {
            next = nd.c0;
        } else if (h1) {
            next = nd.c1;
        }
        q.node = -1;
        if (next >= 0) q.node = next;
        else if (h0 || h1) { q.leaf = next; q.has_leaf = true; }   // -1 is the leaf {0}
    }
    // phase 2: every lane holding a leaf tests it
    if (active && q.has_leaf) {
        const int32_t v = -1 - q.leaf;
        const int32_t start = v >> 3, n = (v & 7) + 1;
        for (int32_t i = start; i < start + n; ++i) query_test_prim<T, D>(s, sv, x, i, q, qc);
        q.has_leaf = false;
    }
}

// A whole query (every lane runs its own to completion).
template <class T, int D, class Stack>
__device__ __forceinline__ int32_t closest_leaf(const Scene<T>& s, const StageView& sv, int32_t root,
                                                const T* x, int32_t warm, T& best, QueryCount& qc,
                                                Stack& st) {
    Query<T, D> q;
    query_begin<T, D>(s, sv, root, x, warm, q);
#pragma unroll 1
    while (!q.done) query_round<T, D>(s, sv, x, true, q, qc, st);
    best = q.best;
    return q.bleaf;
}

// A query limited to primitives nearer than sqrt(bound2): the same leaf and
// squared distance as closest_leaf when the closest primitive lies within
// the bound, else -1 (best = bound2).  warm (or -1) with its squared
// distance warm_d2 seeds the search as in closest_leaf.
template <class T, int D, class Stack>
__device__ __forceinline__ int32_t closest_leaf_within(const Scene<T>& s, const StageView& sv, int32_t root,
                                                       const T* x, int32_t warm, T warm_d2, T bound2, T& best,
                                                       QueryCount& qc, Stack& st) {
    Query<T, D> q;
    query_begin<T, D>(s, sv, root, x, -1, q);
    if (warm >= 0 && warm_d2 < bound2) {
        q.best = warm_d2;
        q.bleaf = warm;
    } else {
        q.best = bound2;
    }
#pragma unroll 1
    while (!q.done) query_round<T, D>(s, sv, x, true, q, qc, st);
    best = q.best;
    return q.bleaf;
}

// ---------------------------------------------------------------------------
// boundary data and normals
// ---------------------------------------------------------------------------
template <class T, int D>
__device__ __forceinline__ void prim_vertices(const Scene<T>& s, int32_t orig, T* V, int32_t* vid) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
        vid[k] = s.pverts[(size_t)orig * D + k];
#pragma unroll
        for (int c = 0; c < D; ++c) V[k * D + c] = s.verts[(size_t)vid[k] * D + c];
    }
}

// geometric normal of a primitive from its vertices (unit length)
template <class T, int D>
__device__ __forceinline__ void geo_normal(const T* V, T* n) {
    if constexpr (D == 2) {
        const T tx = V[2] - V[0], ty = V[3] - V[1];
        const T inv = T(1) / sqrt(tx * tx + ty * ty);
        n[0] = ty * inv; n[1] = -tx * inv;
    } else {
        const T e1[3] = {V[3] - V[0], V[4] - V[1], V[5] - V[2]};
        const T e2[3] = {V[6] - V[0], V[7] - V[1], V[8] - V[2]};
        T c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const T inv = T(1) / sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        n[0] = c[0] * inv; n[1] = c[1] * inv; n[2] = c[2] * inv;
    }
}

// g at a closest point (restricted field or interpolated mapped values)
template <class T, int D>
__device__ __forceinline__ T boundary_value(const Scene<T>& s, const Params<T>& prm, int32_t orig,
                                            const T* bary, const T* xbar, const int32_t* vid) {
    const int L = s.label[orig];
    if (prm.kind[L] == 1) {
        T v = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) v += bary[k] * s.gvert[vid[k]];
        return v;
    }
    T v = prm.gc[L];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        v += prm.gb[L][i] * xbar[i];
#pragma unroll
        for (int j = 0; j < D; ++j) v += xbar[i] * prm.gA[L][i * 3 + j] * xbar[j];
    }
    return v;
}

template <class T, int D>
__device__ __forceinline__ T source_f(const Params<T>& prm, const T* y) {
    T v = prm.src_c0;
    for (int i = 0; i < prm.n_gauss; ++i) {
        T d2 = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) { const T e = y[k] - prm.gauss[i][1 + k]; d2 += e * e; }
        v += prm.gauss[i][0] * exp(-d2 / (T(2) * prm.gauss[i][4] * prm.gauss[i][4]));
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned lo = (unsigned)__shfl_xor((int)(unsigned)(v & 0xffffffffull), o);
        const unsigned hi = (unsigned)__shfl_xor((int)(unsigned)(v >> 32), o);
        v += ((unsigned long long)hi << 32) | lo;
    }
    return v;
}

// ---------------------------------------------------------------------------
// wave-level work queue
// ---------------------------------------------------------------------------
// v of lane src (wave-uniform src), as a wave-uniform value (scalar registers)
__device__ __forceinline__ unsigned long long bcast64(unsigned long long v, int src) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v & 0xffffffffull), src);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// the walk kernel
//   MODE 0: Algorithm 1 (forward walks): rec_u = walk estimate
//   MODE 1: Algorithm 2 (differential walks) with the joint u estimate and K
//           nested forward walks from xbar - delta n at the terminal point;
//           rec_uoff = their mean (eq. (dudn_fd_estimate) follows from it)
//   MODE 2: as MODE 1 with the offset-point gradient estimator of
//           eq. (dudn_mc_estimate) (Laplace only): the first step of each
//           nested walk goes from xoff to y = xoff + R s (R the largest empty
//           ball), and D/R (s.n) (u(y) - g(xbar)) estimates du/dn; rec_uoff
//           is g - delta times their mean, so that (g - rec_uoff)/delta is
//           that estimate
// The unstaged 3D kernel asks for six wavefronts per SIMD (at most 80
// registers per lane, a few spilled): its closest-point queries wait on L2
// and Infinity-Cache gathers, and the extra wavefronts hide that latency
// (200,000-triangle icosphere: forward launch 117 -> 100 ms, differential
// 162 -> 133 ms, against 106 / 136 ms at five and 107 / 156 ms at seven
// wavefronts).  Since the registers were trimmed, the differential build
// (MODE 1) is faster at five (at most 96 registers, fewer spills): 120.0 ->
// 118.5 ms on the icosphere and 88.2 -> 86.9 ms on the 256-instance batch,
// while the forward build loses 9-10% at five and stays at six.  The staged
// kernel's 1024-thread block, the 2D scenes' LDS-resident trees and the FP64
// reference build keep the compiler's choice.
template <class T, int D, int MODE, bool STAGED>
struct WalkWaves {
    static constexpr int v = (sizeof(T) == 4 && !STAGED && D == 3) ? (MODE == 1 ? 5 : 6) : 1;
};

// CV: the build with the control variate's bookkeeping (MODE >= 1 with
// a.cv_run set); without it the kernel carries none of that state.
template <class T, int D, int MODE, bool STAGED, bool CV = false>
__global__ void __launch_bounds__(STAGED ? kBlockStaged : kBlock) __attribute__((amdgpu_waves_per_eu(WalkWaves<T, D, MODE, STAGED>::v)))
walk_kernel(WalkArgs<T> a) {
    const int lane = threadIdx.x & 63;
    TravStack<T, kLdsStack && !STAGED> stack;
    if constexpr (kLdsStack && !STAGED) {
        __shared__ int32_t s_node[kStackSize * kBlock];
        __shared__ T s_d[kStackSize * kBlock];
        stack.node = s_node + threadIdx.x;
        stack.d = s_d + threadIdx.x;
    }
    StageView sv{0, -1};
    if constexpr (STAGED) {
        // copy the top BVH levels (and, if they fit, all primitives) into LDS
        // once per persistent block; every later node or primitive fetch
        // below the staged prefix is an LDS read
        const int64_t nn4 = (int64_t)a.s.n_stage_nodes * node_scalars(D) * (int64_t)sizeof(T) / 16;
        const float4* gn = reinterpret_cast<const float4*>(a.s.nodes);
        for (int64_t i = threadIdx.x; i < nn4; i += blockDim.x) g_stage[i] = gn[i];
        if (a.s.stage_prims) {
            const int64_t np4 = a.s.n_prims * prim_scalars(D) * (int64_t)sizeof(T) / 16;
            const float4* gp = reinterpret_cast<const float4*>(a.s.prims);
            for (int64_t i = threadIdx.x; i < np4; i += blockDim.x) g_stage[nn4 + i] = gp[i];
        }
        __syncthreads();
        sv.n_lnodes = a.s.n_stage_nodes;
        sv.prim_off4 = a.s.stage_prims ? nn4 : -1;
    }
    uint32_t key0 = a.key0, key1 = a.key1;
    if (a.seed_ptr) {
        const unsigned long long sd = *a.seed_ptr + (((unsigned long long)a.key1 << 32) | a.key0);
        key0 = (uint32_t)sd;
        key1 = (uint32_t)(sd >> 32);
    }
    unsigned long long pool_next = 0, pool_end = 0;   // wave-uniform
    bool done = false;
    int64_t wid = -1;          // logical walk id (relative to wid_offset)
    // walk state
    T x[D], xoff[D];
    T acc = T(0), u_main = T(0), usum = T(0);
    T kappa = T(0), eps = T(1);   // the instance's delta is read at the terminal
    uint32_t k = 0, m = 0, p = 0, inst_tag = 0;
    int64_t first_row = 0;
    int32_t root = 0, warm = -1, term_leaf = -1, term_code = -1, phase = 0;
    T term_b1 = T(0), term_b2 = T(0);
    int64_t wsteps = 0;
    // MODE 2: terminal normal and data, and the current nested walk's weight
    T bvc_n[D], bvc_g = T(0), bvc_w = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) bvc_n[c] = T(0);
    // closest-point query in progress (resumable across iterations)
    Query<T, D> q;
    bool qpend = false;
    // control-variate trace of the current nested walk
    T cv_S = T(0);
    T ysel[D], rho_sel = T(0), d_sel = T(0);
#pragma unroll
    for (int c = 0; c < D; ++c) ysel[c] = T(0);
    // lane statistics
    // (32 bits per lane keeps registers free; the node, primitive and step
    // counts move to the device totals before they could wrap)
    // (walks cut at the cap, stack overflows and non-finite positions are
    // rare: each goes to the device totals when it happens)
    uint32_t c_walks = 0, c_nested = 0, c_steps = 0, c_term = 0, c_nodes = 0, c_prims = 0;
    auto count_rare = [&](unsigned long long Counters::*field, unsigned long long v) {
        atomicAdd(&(a.cnt->*field), v);
        atomicAdd(&(a.tot->*field), v);
    };
#pragma unroll 1
    while (true) {
        // ---- hand new walks to idle lanes ------------------------------------
        const bool need = (wid < 0) && !done;
        const unsigned long long mask = __ballot(need);
        if (mask) {
            const int n = __popcll(mask);
            const int rank = __popcll(mask & ((1ull << lane) - 1ull));
            const unsigned long long avail = pool_end - pool_next;
            unsigned long long myid;
            if (avail >= (unsigned long long)n) {
                myid = pool_next + rank;
                pool_next += n;
            } else {
                const int leader = __ffsll((long long)mask) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)a.chunk);
                base = bcast64(base, leader);
                myid = (unsigned long long)rank < avail ? pool_next + rank : base + (rank - avail);
                pool_next = base + (n - avail);
                pool_end = base + a.chunk;
            }
            if (need) {
                if (myid >= (unsigned long long)a.total) {
                    done = true;
                } else {
                    wid = (int64_t)myid;
                    const int64_t gid = wid + a.wid_offset;
                    int ii = 0;
                    if (a.n_inst > 1) {   // instance containing walk gid
                        int lo = 0, hi = a.n_inst - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (a.inst[mid].walk_begin <= gid) lo = mid; else hi = mid - 1;
                        }
                        ii = lo;
                    }
                    const Instance<T> in = a.inst[ii];
                    const int64_t local = gid - in.walk_begin;
                    int64_t pin = local / a.W;
                    m = (uint32_t)(local - pin * a.W);
                    if (a.perm) {   // the slot's point; records stay indexed by point
                        pin = a.perm[pin];
                        wid = pin * a.W + m;
                    }
                    p = (uint32_t)(pin + in.p_counter);
                    root = in.root;
                    kappa = in.kappa; eps = in.eps;
                    inst_tag = (uint32_t)ii << 16;
                    const double* xp = a.X + (size_t)(in.point_begin + pin) * D;
                    first_row = in.point_begin + pin - a.x_base;
#pragma unroll
                    for (int i = 0; i < D; ++i) x[i] = T(xp[i]);
                    acc = T(0); k = 0; warm = -1; phase = 0; usum = T(0); wsteps = 0;
                    c_walks++;
                }
            }
        }
        if (__ballot(!done) == 0ull) break;
        if (done) continue;

        // ---- one walk step: closest-point query -----------------------------
        // A lane without a query in progress starts one at x.  The wavefront
        // then traverses until at least a.park of its lanes have their
        // answer (or none is still searching); lanes whose query is
        // unfinished skip the rest of this iteration and resume it in the
        // next, so that fast queries do not wait for the slowest one.
        bool ready = false;
        bool shared = false;   // answered by the point's shared first query
        T d2 = T(0);
        int32_t leaf = -1;
        if (!qpend) {
            if (a.first_leaf && phase == 0 && k == 0) {
                leaf = a.first_leaf[first_row];
                d2 = a.first_d2[first_row];
                ready = true;
                shared = true;
            } else {
                query_begin<T, D>(a.s, sv, root, x, warm, q);
                qpend = true;
            }
        }
        {
            QueryCount qc{0, 0, 0};
#pragma unroll 1
            while (true) {
                const bool searching = qpend && !q.done;
                const unsigned long long sm = __ballot(searching);
                const unsigned long long rm = __ballot(ready || (qpend && q.done));
                if (sm == 0ull || __popcll(rm) >= a.park) break;
                query_round<T, D>(a.s, sv, x, searching, q, qc, stack);
            }
            c_nodes += qc.nodes; c_prims += qc.prims;
            if (qc.overflow) count_rare(&Counters::overflow, qc.overflow);
            if ((c_nodes | c_prims | c_steps) >= 0x80000000u) {   // rare: move to the totals
                Counters* dst[2] = {a.cnt, a.tot};
                for (int t = 0; t < 2; ++t) {
                    atomicAdd(&dst[t]->nodes, (unsigned long long)c_nodes);
                    atomicAdd(&dst[t]->prims, (unsigned long long)c_prims);
                    atomicAdd(&dst[t]->steps, (unsigned long long)c_steps);
                }
                c_nodes = 0; c_prims = 0; c_steps = 0;
            }
        }
        if (qpend && q.done) {
            leaf = q.bleaf;
            d2 = q.best;
            qpend = false;
            ready = true;
        }
        if (!ready) continue;
        // executed queries: the shared first query of a point (run once for
        // all its walks) counts once, on the point's walk 0
        if (!shared || m == 0) c_steps++;
        wsteps++;
        if (leaf < 0 || !(d2 >= T(0))) {
            // non-finite position (e.g. a NaN query point): end the walk with
            // a NaN result instead of touching primitive -1
            count_rare(&Counters::invalid, 1ull);
            const T nanv = T(NAN);
            a.rec_u[wid] = nanv;
            if (MODE >= 1) {
                a.rec_prim[wid] = -1;
                a.rec_uoff[wid] = nanv;
                if (CV && a.cv_run) a.cv_run[wid] = -1;
            }
            if (a.rec_steps) a.rec_steps[wid] = wsteps;
            wid = -1;
            continue;
        }
        const T d = sqrt(d2);
        const bool cap = (int)(k + 1) >= a.prm.kmax;
        const bool nested = MODE >= 1 && phase > 0;
        bool finished = false;     // the current (main or nested) walk ended
        bool alive = false;        // ... in the shell or at the cap (not by roulette)
        T result = T(0);           // its value
        if (d < eps || cap) {
            if (cap && !(d < eps)) count_rare(&Counters::truncated, 1ull);
            // closest point, barycentrics, boundary value
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
                for (int kk = 0; kk < D; ++kk) v += bary[kk] * V[kk * D + c];
                xbar[c] = v;
            }
            const T g = boundary_value<T, D>(a.s, a.prm, orig, bary, xbar, vid);
            if (MODE >= 1 && phase == 0) {
                // BoundaryNormal, oriented out of the domain: away from the
                // walk's previous position (held in xoff until now), which
                // lies inside by at least eps; the terminal position itself
                // may sit within rounding of the boundary, or past it, where
                // the side test has no reliable sign.  A walk that starts in
                // the shell uses its start point.
                T n[3] = {T(0), T(0), T(0)};
                geo_normal<T, D>(V, n);
                T dn = T(0);
#pragma unroll
                for (int c = 0; c < D; ++c) dn += n[c] * (xbar[c] - (k > 0 ? xoff[c] : x[c]));
                const int flip = dn < T(0) ? 1 : 0;
                if (flip) {
#pragma unroll
                    for (int c = 0; c < D; ++c) n[c] = -n[c];
                }
                u_main = acc + g;
                if constexpr (MODE == 2) {
#pragma unroll
                    for (int c = 0; c < D; ++c) bvc_n[c] = n[c];
                    bvc_g = g;
                    bvc_w = T(0);
                }
                term_code = orig * 2 + flip;
                term_b1 = bary[1]; term_b2 = bary[2];
                term_leaf = leaf;
                {
                    const T delta = a.inst[inst_tag >> 16].delta;
#pragma unroll
                    for (int c = 0; c < D; ++c) xoff[c] = xbar[c] - delta * n[c];
                }
                c_term++;
                if (a.prim_dep && !a.prim_dep[orig]) {
                    a.rec_u[wid] = u_main;
                    a.rec_prim[wid] = term_code;
                    a.rec_b[(size_t)wid * (D - 1)] = term_b1;
                    if constexpr (D == 3) a.rec_b[(size_t)wid * 2 + 1] = term_b2;
                    a.rec_uoff[wid] = g;
                    if (CV && a.cv_run) a.cv_run[wid] = -1;
                    if (a.rec_steps) a.rec_steps[wid] = wsteps;
                    wid = -1;
                    continue;
                }
                if (CV && a.cv_run) {
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        a.cv_xoff[(size_t)wid * D + c] = xoff[c];
                        a.cv_xbar[(size_t)wid * D + c] = xbar[c];
                    }
                    a.cv_g[wid] = g;
                    int run = 1;
                    if (a.cv_qthresh < (1u << 24)) {
                        // run the nested walks with probability q
                        const u4 rq = philox10(u4{k, m, p, inst_tag | 4u}, key0, key1);
                        run = (rq.x >> 8) < a.cv_qthresh ? 1 : 0;
                    }
                    a.cv_run[wid] = run;
                    if (!run) {
                        a.rec_u[wid] = u_main;
                        a.rec_prim[wid] = term_code;
                        a.rec_b[(size_t)wid * (D - 1)] = term_b1;
                        if constexpr (D == 3) a.rec_b[(size_t)wid * 2 + 1] = term_b2;
                        a.rec_uoff[wid] = T(0);
                        if (a.rec_steps) a.rec_steps[wid] = wsteps;
                        wid = -1;
                        continue;
                    }
                }
                // the walk's own records now (only the nested mean is left)
                a.rec_u[wid] = u_main;
                a.rec_prim[wid] = term_code;
                a.rec_b[(size_t)wid * (D - 1)] = term_b1;
                if constexpr (D == 3) a.rec_b[(size_t)wid * 2 + 1] = term_b2;
                // start the first nested forward walk at the offset point
                phase = 1;
                cv_S = T(0); rho_sel = T(0); d_sel = T(0);
#pragma unroll
                for (int c = 0; c < D; ++c) x[c] = xoff[c];
                acc = T(0); k = 0; warm = term_leaf;
                c_nested++;
                continue;
            }
            finished = true;
            alive = true;
            result = acc + g;
        } else {
            const uint32_t tag = inst_tag | (nested ? (1u | ((uint32_t)(phase - 1) << 8)) : 0u);
            const u4 r = philox10(u4{k, m, p, tag}, key0, key1);
            if (MODE >= 1 && CV && nested && a.cv_run) {
                // weighted reservoir choice of one source step (probability
                // proportional to its ball's Green's-function mass) with one
                // uniform point of its ball
                const T mj = green_mass<D, T>(kappa, d);
                cv_S += mj;
                const u4 r3 = philox10(u4{k, m, p, tag | 4u}, key0, key1);
                if (unif<T>(r3.x) * cv_S < mj) {
                    T dir[3];
                    unit_dir<T, D>(r3.y, r3.z, dir);
                    T rho;
                    if constexpr (D == 2) rho = sqrt(unif_pos<T>(r3.w));
                    else rho = cbrt(unif_pos<T>(r3.w));
#pragma unroll
                    for (int c = 0; c < D; ++c) ysel[c] = x[c] + rho * d * dir[c];
                    rho_sel = rho;
                    d_sel = d;
                }
            }
            if (a.prm.has_source) {
                // ball-point direction: 2D uses the step draw's second word
                // (the step direction needs only the first), 3D a second draw
                T dir[3];
                if constexpr (D == 2) {
                    unit_dir<T, D>(r.y, 0u, dir);
                } else {
                    const u4 r2 = philox10(u4{k, m, p, tag | 2u}, key0, key1);
                    unit_dir<T, D>(r2.x, r2.y, dir);
                }
                T rho;
                if constexpr (D == 2) rho = sqrt(unif_pos<T>(r.w));
                else rho = cbrt(unif_pos<T>(r.w));
                T y[3];
#pragma unroll
                for (int c = 0; c < D; ++c) y[c] = x[c] + rho * d * dir[c];
                acc += green_ball_t<D, T>(kappa, rho, d) * source_f<T, D>(a.prm, y);
            }
            const T alpha = poisson_scale<T, D>(kappa, d);
            if (a.prm.rr && alpha < unif<T>(r.z)) {
                finished = true;
                result = acc;
                if (MODE >= 1 && phase == 0) term_code = -1;
            } else {
                T dir[3];
                unit_dir<T, D>(r.x, r.y, dir);
                if constexpr (MODE == 2) {
                    if (nested && k == 0) {
                        T sn = T(0);
#pragma unroll
                        for (int c = 0; c < D; ++c) sn += dir[c] * bvc_n[c];
                        bvc_w = T(D) / d * sn;
                    }
                }
                if (MODE >= 1 && phase == 0) {
#pragma unroll
                    for (int c = 0; c < D; ++c) xoff[c] = x[c];   // previous position
                }
#pragma unroll
                for (int c = 0; c < D; ++c) x[c] += d * dir[c];
                ++k;
                warm = leaf;
            }
        }
        if (!finished) continue;

        if (MODE == 0) {
            a.rec_u[wid] = result;
            if (a.rec_steps) a.rec_steps[wid] = wsteps;
            wid = -1;
        } else if (phase == 0) {
            // differential walk stopped by roulette: udot = 0, u = sources
            a.rec_u[wid] = result;
            a.rec_prim[wid] = -1;
            a.rec_uoff[wid] = T(0);
            if (CV && a.cv_run) a.cv_run[wid] = -1;
            if (a.rec_steps) a.rec_steps[wid] = wsteps;
            wid = -1;
        } else {
            if constexpr (MODE == 2) usum += bvc_w * (result - bvc_g);
            else usum += result;
            if (CV && a.cv_run) {
                const size_t q = (size_t)wid * a.prm.K + (phase - 1);
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    a.cv_stop[q * D + c] = x[c];
                    a.cv_y[q * D + c] = ysel[c];
                }
                a.cv_rho[q] = rho_sel;
                a.cv_d[q] = d_sel;
                a.cv_S[q] = cv_S;
                a.cv_alive[q] = alive ? 1 : 0;
            }
            if (phase >= a.prm.K) {
                if constexpr (MODE == 2) a.rec_uoff[wid] = bvc_g - a.inst[inst_tag >> 16].delta * (usum / T(a.prm.K));
                else a.rec_uoff[wid] = usum / T(a.prm.K);
                if (a.rec_steps) a.rec_steps[wid] = wsteps;
                wid = -1;
            } else {
                ++phase;
                if constexpr (MODE == 2) bvc_w = T(0);
#pragma unroll
                for (int c = 0; c < D; ++c) x[c] = xoff[c];
                acc = T(0); k = 0; warm = term_leaf;
                cv_S = T(0); rho_sel = T(0); d_sel = T(0);
                c_nested++;
            }
        }
    }
    // ---- statistics: wave sums, then one atomic per counter per wave -------
    const unsigned long long s_walks = wave_sum_u64(c_walks);
    const unsigned long long s_nested = wave_sum_u64(c_nested);
    const unsigned long long s_steps = wave_sum_u64(c_steps);
    const unsigned long long s_term = wave_sum_u64(c_term);
    const unsigned long long s_nodes = wave_sum_u64(c_nodes);
    const unsigned long long s_prims = wave_sum_u64(c_prims);
    if (lane == 0) {
        Counters* dst[2] = {a.cnt, a.tot};
        for (int q = 0; q < 2; ++q) {
            Counters* c = dst[q];
            atomicAdd(&c->walks, s_walks);
            atomicAdd(&c->nested, s_nested);
            atomicAdd(&c->steps, s_steps);
            atomicAdd(&c->terminal, s_term);
            atomicAdd(&c->nodes, s_nodes);
            atomicAdd(&c->prims, s_prims);
        }
    }
}

}  // namespace dwos
