// Walk on stars on gfx950 in 3D: the screened Poisson problem with a
// Dirichlet triangle mesh and a fixed reflecting triangle mesh carrying the
// Robin condition du/dn - mu u = h (n into the domain; mu = 0, h = 0: zero
// flux), the mixed problem of Sec. 3.4, and its differential version of
// Sec. 4.4, which nests through the Dirichlet boundary only.  One step, as
// in the 2D kernel (wost_kernels.hpp) with 3D geometry:
//   * d = distance to the Dirichlet boundary; in its eps-shell the walk ends
//     as in Algorithm 1 / Algorithm 2.
//   * star radius R = min(d, distance to the closest silhouette edge of the
//     reflecting mesh[, 1/mu]).  Seen from x, an edge shared by two
//     triangles is a silhouette when both lie on the same side of the plane
//     through x and the edge; an edge with one triangle (a rim) or more than
//     two always is.  A triangle seen edge-on does not decide (see
//     sil3_test).
//   * a direction v uniform on the sphere (at a wall point: on the half that
//     enters the domain, by reflecting the other half); the first reflecting
//     triangle entered from its domain side along v before R gives the next
//     point with weight reflect_weight(t, R), else x + R v with alpha(R).
//   * source: y = x + rho v along the same direction, rho = R U^(1/3),
//     counted if rho < t.
//   * Robin terms: the triangles that reach into B(x, R) with their whole
//     areas A_i, L = sum A_i; an order-free exponential race with weights
//     A_i picks one (each triangle o draws from its own Philox counter
//     (k, m, p, tag | 8 | o << 16)) and z is uniform on it (words 1, 2 of
//     the winner's draw); a z outside the ball adds nothing.  The data term
//     adds -c L G(|z - x|; R) h(z) (c = 2 on a wall, else 1); with
//     probability q = min(1/2, c mu L G) the walk continues at z with weight
//     -c mu L G / q (branch on word 3 of the winner's draw), else the step's
//     weight is divided by 1 - q.  Roulette keeps the walk with probability
//     min(1, |w|) and the throughput carries w / keep.
// Random numbers: one Philox draw per step, words 0 and 1 the direction,
// word 2 the roulette, word 3 the source radius.
//
// The reflecting mesh has two BVHs in the layout of bvh.hpp: one over its
// triangles (rays, Robin samples) and one over its edges (silhouettes).
// Every reflecting triangle must have the domain on its left normal
// (b - a) x (c - a); walls are one-way, met only from their domain side.
#pragma once
#include "wost_kernels.hpp"

namespace dwos {

// Per reflecting triangle in leaf order: a[3] b[3] c[3] and 3 pad scalars.
constexpr int kTriGeo = 12;
// Per reflecting edge in leaf order: p[3] q[3] (its vertices) and w0[3],
// w1[3] (the third vertex of its first and second triangle; w1 unused for
// a rim).  einfo: {flags (1: always a silhouette), leaf position of the
// first triangle, of the second (-1 none), original edge index}.
constexpr int kEdgeGeo = 12;

// Normal cones of the silhouette query, per edge-BVH node and child (8
// scalars: a unit axis a[3], sin and cos of s0 = theta + margin, the range
// [omin, omax] of a.p over the child's edge vertices p, and kappa), theta
// the largest angle between a and the left normals of the triangles at the
// child's edges.  Seen from x, an edge of two consistently wound triangles
// is a silhouette only if x is in front of one triangle's plane and behind
// the other's (or sees one edge-on).  Two tests show a child holds none:
// (view cone) the normals' dot products with the view direction then
// differ in sign, so some normal of the cone is perpendicular to a view
// direction; a child whose view cone from x (half-angle beta over the child
// box's bounding sphere) keeps every such dot product of one sign --
// |cos angle(a, c - x)| > sin(s0 + beta) with s0 + beta < pi/2 -- holds
// none.  (planes) For a triangle with unit normal n through edge vertex p,
// n.(x - p) >= a.x - omax - 2 sin(s0/2) |x - p|, so a.x - omax > (2
// sin(s0/2) + kappa) dmax (dmax >= |x - p| over the child's box) puts x in
// front of every such plane by more than kappa |x - p|, and omin - a.x
// beyond the same bound puts it behind all of them; kappa = 4 tol / sin phi
// over the child's edges, phi the angle at the edge's first vertex between
// the edge and a triangle's third vertex, keeps every triangle clear of the
// edge-on tolerance tol.  The cone margin covers the edge-on tolerance and
// rounding, the plane test a floor of 32 units of rounding; children with a
// rim, a non-manifold or inconsistently wound edge, or normals spread by
// pi/2 or more, store sin = 2, cos = -1 (never pruned).
constexpr int kEdgeCone = 8;

template <class T>
struct RefScene3 {
    const T* tnodes;          // triangle BVH
    const T* tgeo;
    const int32_t* torig;     // leaf position -> original triangle
    const int32_t* tleaf_of;  // original triangle -> leaf position
    int64_t nt;
    const T* enodes;          // edge BVH
    const T* egeo;
    const int4* einfo;
    const T* econes;          // per edge node: child 0 then child 1, kEdgeCone each
    int64_t ne;
    // FP32: the edge BVH's first n_estage nodes (breadth-first order) and
    // their cones in LDS at g_stage + estage_off4 (16-byte words: the nodes,
    // then the cones); 0: none
    int32_t n_estage;
    int64_t estage_off4;
    // Robin condition: h = hq[0] + hq[1..3] . z + z^T A z, A = hq[4..12] row
    // major; robin = 0: zero flux
    int32_t robin;
    T mu;
    T hq[13];
};

template <class T>
__device__ __forceinline__ T robin_data3(const RefScene3<T>& r, const T* z) {
    T v = r.hq[0] + r.hq[1] * z[0] + r.hq[2] * z[1] + r.hq[3] * z[2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) v += z[i] * r.hq[4 + 3 * i + j] * z[j];
    return v;
}

template <class T>
__device__ __forceinline__ void tri_load(const RefScene3<T>& r, int32_t i, T* P) {
    const T* g = r.tgeo + (size_t)i * kTriGeo;
#pragma unroll
    for (int k = 0; k < 9; ++k) P[k] = g[k];
}

template <class T>
__device__ __forceinline__ void cross3d(const T* a, const T* b, T* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

template <class T>
__device__ __forceinline__ T dot3d(const T* a, const T* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// unit left normal (b - a) x (c - a) of leaf triangle i
template <class T>
__device__ __forceinline__ void tri_left_normal(const RefScene3<T>& r, int32_t i, T* n) {
    T P[9];
    tri_load<T>(r, i, P);
    const T e1[3] = {P[3] - P[0], P[4] - P[1], P[5] - P[2]};
    const T e2[3] = {P[6] - P[0], P[7] - P[1], P[8] - P[2]};
    cross3d<T>(e1, e2, n);
    const T inv = T(1) / sqrt(dot3d<T>(n, n));
    n[0] *= inv; n[1] *= inv; n[2] *= inv;
}

// Keep a point on leaf triangle i a few units of rounding in front of its
// plane (domain side nin), as keep_on_domain_side does for 2D segments.
template <class T>
__device__ __forceinline__ void keep_on_domain_side3(const RefScene3<T>& r, int32_t i, const T* nin, T* x) {
    const T* g = r.tgeo + (size_t)i * kTriGeo;
    const T s = nin[0] * (x[0] - g[0]) + nin[1] * (x[1] - g[1]) + nin[2] * (x[2] - g[2]);
    const T ulp = sizeof(T) == 4 ? T(1.1920929e-07) : T(2.220446049250313e-16);
    const T margin = T(8) * ulp * (fabs(x[0]) + fabs(x[1]) + fabs(x[2]) + fabs(g[0]) + fabs(g[1]) + fabs(g[2]));
    if (s < margin) {
#pragma unroll
        for (int c = 0; c < 3; ++c) x[c] += (margin - s) * nin[c];
    }
}

// Is the edge p-q a silhouette seen from x?  w0, w1: the third vertices of
// its two triangles; own = 1 if x lies on the first triangle, 2 if on the
// second, else 0; nin the domain side of the triangle x lies on (on).  Both
// triangles on the same side of the plane through x and the edge: the
// surface turns back there.  An edge of the triangle x lies on is a
// silhouette iff the other triangle leaves to the outside of that
// triangle's plane.  Otherwise a triangle seen edge-on does not decide: both
// edge-on (a flat part of the surface through x) is not a silhouette, one
// edge-on is decided by the other triangle's side of the plane x lies on
// (x on a wall) or counted (x inside).
template <class T>
__device__ __forceinline__ bool sil3_test(const T* p, const T* q, const T* w0, const T* w1, int own, const T* x,
                                          const T* nin, bool on) {
    auto outside = [&](const T* w) {
        return nin[0] * (w[0] - p[0]) + nin[1] * (w[1] - p[1]) + nin[2] * (w[2] - p[2]) < T(0);
    };
    if (own == 1) return outside(w1);
    if (own == 2) return outside(w0);
    const T t[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
    const T rr[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
    T m[3];
    cross3d<T>(t, rr, m);
    const T lm = sqrt(dot3d<T>(m, m));
    const T d0[3] = {w0[0] - p[0], w0[1] - p[1], w0[2] - p[2]};
    const T d1[3] = {w1[0] - p[0], w1[1] - p[1], w1[2] - p[2]};
    const T c0 = dot3d<T>(m, d0), c1 = dot3d<T>(m, d1);
    const bool z0 = fabs(c0) <= SilTol<T>::v * lm * sqrt(dot3d<T>(d0, d0));
    const bool z1 = fabs(c1) <= SilTol<T>::v * lm * sqrt(dot3d<T>(d1, d1));
    if (z0 && z1) return false;
    if (z0 || z1) return on ? outside(z0 ? w1 : w0) : true;
    return (c0 > T(0)) == (c1 > T(0));
}

// Leaf edge i: if it is nearer to x than sqrt(best) and a silhouette seen
// from x (x on leaf triangle `on` with domain side nin, or inside: -1),
// lower best to its squared distance and return true.
template <class T>
__device__ __forceinline__ bool sil3_edge_nearer(const RefScene3<T>& r, int32_t i, const T* x, int32_t on,
                                                 const T* nin, T& best) {
    const T* g = r.egeo + (size_t)i * kEdgeGeo;
    const T e[3] = {g[3] - g[0], g[4] - g[1], g[5] - g[2]};
    const T ax[3] = {x[0] - g[0], x[1] - g[1], x[2] - g[2]};
    const T ee = dot3d<T>(e, e);
    const T t = ee > T(0) ? fmin(T(1), fmax(T(0), quot<T>(dot3d<T>(ax, e), ee))) : T(0);
    const T dx = ax[0] - t * e[0], dy = ax[1] - t * e[1], dz = ax[2] - t * e[2];
    const T d2 = dx * dx + dy * dy + dz * dz;
    if (!(d2 < best)) return false;
    const int4 inf = r.einfo[i];
    const int own = on < 0 ? 0 : (on == inf.y ? 1 : (on == inf.z ? 2 : 0));
    if ((inf.x & 1) || sil3_test<T>(g, g + 3, g + 6, g + 9, own, x, nin, on >= 0)) {
        best = d2;
        return true;
    }
    return false;
}

// Can the child with box lo..hi and cone q hold a silhouette edge seen from x?
template <class T>
__device__ __forceinline__ bool cone3_may_hold(const T* lo, const T* hi, const T* q, const T* x) {
    if (!(q[3] <= T(1))) return true;      // never pruned
    T c[3], r2 = T(0), d2 = T(0), mag = T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c[k] = T(0.5) * (lo[k] + hi[k]) - x[k];
        const T e = T(0.5) * (hi[k] - lo[k]);
        r2 += e * e;
        d2 += c[k] * c[k];
        mag += fabs(x[k]) + fabs(lo[k]) + fabs(hi[k]);
    }
    {   // planes: x in front of (or behind) every triangle plane of the child
        const T ulp = sizeof(T) == 4 ? T(1.1920929e-07) : T(2.220446049250313e-16);
        const T ax = q[0] * x[0] + q[1] * x[1] + q[2] * x[2];
        const T dmax = sqrt(d2) + sqrt(r2);
        const T marg = (sqrt(fmax(T(0), T(2) - T(2) * q[4])) + q[7]) * dmax + T(32) * ulp * (mag + dmax);
        if (ax - q[6] > marg || q[5] - ax > marg) return false;
    }
    if (!(d2 > r2)) return true;           // x inside the bounding sphere
    const T inv = T(1) / sqrt(d2);
    const T sb = sqrt(r2) * inv, cb = sqrt(T(1) - sb * sb);
    const T cs = q[4] * cb - q[3] * sb;   // cos(s0 + beta)
    if (!(cs > T(0))) return true;
    const T ss = q[3] * cb + q[4] * sb;   // sin(s0 + beta)
    return !(fabs((q[0] * c[0] + q[1] * c[1] + q[2] * c[2]) * inv) > ss);
}

// An edge-BVH node and its children's cones, from LDS for the staged prefix.
template <class T>
__device__ __forceinline__ void edge_node3(const RefScene3<T>& r, int32_t i, NodeData<T, 3>& nd, T* cq) {
    if constexpr (sizeof(T) == 4) {
        if (i < r.n_estage) {
            const float4* w = g_stage + r.estage_off4;
            decode_node_f32<3>(w + (int64_t)i * (node_scalars(3) / 4), nd);
            const float4* c = w + (int64_t)r.n_estage * (node_scalars(3) / 4) + (int64_t)i * (2 * kEdgeCone / 4);
#pragma unroll
            for (int k = 0; k < 2 * kEdgeCone / 4; ++k) {
                const float4 v = c[k];
                cq[4 * k] = v.x; cq[4 * k + 1] = v.y; cq[4 * k + 2] = v.z; cq[4 * k + 3] = v.w;
            }
            return;
        }
    }
    load_node<T, 3>(r.enodes, i, nd);
    const T* g = r.econes + (size_t)i * (2 * kEdgeCone);
#pragma unroll
    for (int k = 0; k < 2 * kEdgeCone; ++k) cq[k] = g[k];
}

// Closest silhouette edge as a resumable query, as sil_round in 2D; x lies
// on leaf triangle `on` (domain side nin) or inside (-1).  A round expands
// nodes until the lane holds a leaf or is answered, then the lanes holding
// leaves test them together; with tail > 0 the expansion stops once at most
// `tail` lanes still descend while some lane holds a leaf (those go on in
// the next round), as in the closest-point query.  Each lane visits the same
// nodes and edges in the same order whatever the tail, so the answer and
// the edge found do not depend on it.
template <class T, class Stack>
__device__ __forceinline__ void sil3_round(const RefScene3<T>& r, const T* x, int32_t on, const T* nin,
                                           SilQuery<T>& q, QueryCount& qc, Stack& st, int tail = 0) {
    // phase 1: expand nodes
#pragma unroll 1
    while (true) {
        const bool go = q.have && q.cur >= 0;
        if (tail > 0) {
            const unsigned long long gm = __ballot(go);
            if (gm == 0ull) break;
            if (__popcll(gm) <= tail && __ballot(q.have && q.cur < 0) != 0ull) break;
            if (!go) continue;
        } else if (!go) {
            break;
        }
        NodeData<T, 3> nd;
        T cq[2 * kEdgeCone];
        edge_node3<T>(r, q.cur, nd, cq);
        qc.nodes++;
        const T d0 = fmax(box_d2<T, 3>(nd.lo0, nd.hi0, x), slab_d2<T, 3>(nd.n0, nd.o0, nd.t0, x));
        const T d1 = fmax(box_d2<T, 3>(nd.lo1, nd.hi1, x), slab_d2<T, 3>(nd.n1, nd.o1, nd.t1, x));
        const bool h0 = !(nd.t0 < T(0)) && d0 < q.best && cone3_may_hold<T>(nd.lo0, nd.hi0, cq, x);
        const bool h1 = !(nd.t1 < T(0)) && d1 < q.best && cone3_may_hold<T>(nd.lo1, nd.hi1, cq + kEdgeCone, x);
        if (h0 && h1) {
            const bool n0 = d0 <= d1;
            if (q.sp < kStackSize) {
                st.put(q.sp, n0 ? nd.c1 : nd.c0, n0 ? d1 : d0);
                ++q.sp;
            } else {
                qc.overflow++;
            }
            q.cur = n0 ? nd.c0 : nd.c1;
        } else if (h0) {
            q.cur = nd.c0;
        } else if (h1) {
            q.cur = nd.c1;
        } else {
            sil_pop<T>(q, st);
        }
    }
    // phase 2: the lanes holding a leaf test its edges
    if (q.have && q.cur < 0) {
        const int32_t v = -1 - q.cur;
        const int32_t start = v >> 3, n = (v & 7) + 1;
        for (int32_t i = start; i < start + n; ++i) {
            qc.prims++;
            if (sil3_edge_nearer<T>(r, i, x, on, nin, q.best)) q.bsil = i;
        }
        sil_pop<T>(q, st);
    }
}

template <class T, class Stack>
__device__ T silhouette3_d2(const RefScene3<T>& r, const T* x, int32_t on, const T* nin, T best, QueryCount& qc,
                            Stack& st) {
    SilQuery<T> q;
    sil_begin<T>(q, best);
#pragma unroll 1
    while (q.have) sil3_round<T>(r, x, on, nin, q, qc, st);
    return q.best;
}

// Entry distance of the ray x + t dir (t in [0, tmax]) into a child's box
// and oriented slab (3D), or +inf if it misses them.
template <class T>
__device__ __forceinline__ T ray_child3(const T* lo, const T* hi, const T* n, T o, T th, const T* x, const T* dir,
                                        const T* inv, T tmax) {
    if (th < T(0)) return T(INFINITY);   // empty child
    T tn = T(0), tf = tmax;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (dir[k] != T(0)) {
            const T t1 = (lo[k] - x[k]) * inv[k], t2 = (hi[k] - x[k]) * inv[k];
            tn = fmax(tn, fmin(t1, t2));
            tf = fmin(tf, fmax(t1, t2));
        } else if (x[k] < lo[k] || x[k] > hi[k]) {
            return T(INFINITY);
        }
    }
    const T pn = n[0] * dir[0] + n[1] * dir[1] + n[2] * dir[2];
    const T q = n[0] * x[0] + n[1] * x[1] + n[2] * x[2] - o;
    if (pn != T(0)) {
        const T s1 = (-th - q) / pn, s2 = (th - q) / pn;
        tn = fmax(tn, fmin(s1, s2));
        tf = fmin(tf, fmax(s1, s2));
    } else if (fabs(q) > th) {
        return T(INFINITY);
    }
    return tn <= tf * Slack<T>::v + T(1e-30) ? tn : T(INFINITY);
}

// Barycentric slack of the ray-triangle test: a ray through an edge shared
// by two triangles is taken by at least one of them despite rounding.
template <class T> struct BaryTol;
template <> struct BaryTol<float> { static constexpr float v = 1e-6f; };
template <> struct BaryTol<double> { static constexpr double v = 1e-13; };

// First reflecting triangle (leaf position) entered from its domain side by
// x + t dir, 0 <= t < tmax, skipping leaf `skip`; -1 if none.  t_out: its t,
// or tmax.  Equal t go to the lowest original index.
template <class T, class Stack>
__device__ int32_t ray3_first(const RefScene3<T>& r, const T* x, const T* dir, T tmax, int32_t skip, T& t_out,
                              QueryCount& qc, Stack& st) {
    T inv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) inv[k] = dir[k] != T(0) ? T(1) / dir[k] : T(0);
    T best = tmax;
    int32_t hit = -1;
    int sp = 0;
    int32_t cur = 0;
    bool have = true;
#pragma unroll 1
    while (have) {
        if (cur >= 0) {
            NodeData<T, 3> nd;
            load_node<T, 3>(r.tnodes, cur, nd);
            qc.nodes++;
            const T e0 = ray_child3<T>(nd.lo0, nd.hi0, nd.n0, nd.o0, nd.t0, x, dir, inv, best);
            const T e1 = ray_child3<T>(nd.lo1, nd.hi1, nd.n1, nd.o1, nd.t1, x, dir, inv, best);
            const bool h0 = e0 <= best, h1 = e1 <= best;
            if (h0 && h1) {
                const bool n0 = e0 <= e1;
                if (sp < kStackSize) {
                    st.put(sp, n0 ? nd.c1 : nd.c0, n0 ? e1 : e0);
                    ++sp;
                } else {
                    qc.overflow++;
                }
                cur = n0 ? nd.c0 : nd.c1;
            } else if (h0) {
                cur = nd.c0;
            } else if (h1) {
                cur = nd.c1;
            } else {
                have = false;
            }
        } else {
            const int32_t v = -1 - cur;
            const int32_t start = v >> 3, n = (v & 7) + 1;
            for (int32_t i = start; i < start + n; ++i) {
                if (i == skip) continue;
                T P[9];
                tri_load<T>(r, i, P);
                qc.prims++;
                const T e1[3] = {P[3] - P[0], P[4] - P[1], P[5] - P[2]};
                const T e2[3] = {P[6] - P[0], P[7] - P[1], P[8] - P[2]};
                T nrm[3];
                cross3d<T>(e1, e2, nrm);
                // one-way: only a ray entering from the domain side (the left
                // normal's side) is stopped
                if (!(dot3d<T>(dir, nrm) < T(0))) continue;
                // an origin further behind the plane than rounding explains is
                // not on this wall's domain side
                const T tv[3] = {x[0] - P[0], x[1] - P[1], x[2] - P[2]};
                const T h = dot3d<T>(nrm, tv);
                const T sc = fabs(x[0]) + fabs(x[1]) + fabs(x[2]) + fabs(P[0]) + fabs(P[1]) + fabs(P[2]);
                if (h < T(0) && h * h > kBehind<T>::v * kBehind<T>::v * dot3d<T>(nrm, nrm) * sc * sc) continue;
                // Moller-Trumbore barycentrics and distance
                T pv[3];
                cross3d<T>(dir, e2, pv);
                const T det = dot3d<T>(e1, pv);
                if (det == T(0)) continue;
                const T id = T(1) / det;
                const T u = dot3d<T>(tv, pv) * id;
                if (u < -BaryTol<T>::v || u > T(1) + BaryTol<T>::v) continue;
                T qv[3];
                cross3d<T>(tv, e1, qv);
                const T vv = dot3d<T>(dir, qv) * id;
                if (vv < -BaryTol<T>::v || u + vv > T(1) + BaryTol<T>::v) continue;
                const T t = fmax(T(0), dot3d<T>(e2, qv) * id);
                if (t < best || (t == best && hit >= 0 && r.torig[i] < r.torig[hit])) {
                    best = t;
                    hit = i;
                }
            }
            have = false;
        }
        if (!have) {
#pragma unroll 1
            while (sp > 0) {
                --sp;
                if (st.get_d(sp) <= best) {
                    cur = st.get_node(sp);
                    have = true;
                    break;
                }
            }
        }
    }
    t_out = best;
    return hit;
}

// Robin sample (see the header): returns the leaf of z's triangle or -1
// (nothing in the ball, or z outside it); L = the summed areas of the
// triangles that reach into the ball; branch = word 3 of the winner's draw.
template <class T, class Stack>
__device__ int32_t ref3_boundary_sample(const RefScene3<T>& r, const T* x, T R, u4 ctr, uint32_t key0,
                                        uint32_t key1, T& L, T* z, uint32_t& branch, QueryCount& qc, Stack& st) {
    const T R2 = R * R;
    L = T(0);
    int32_t win = -1;
    T best = T(INFINITY);
    u4 ww{0, 0, 0, 0};
    int sp = 0;
    int32_t cur = 0;
    bool have = true;
#pragma unroll 1
    while (have) {
        if (cur >= 0) {
            NodeData<T, 3> nd;
            load_node<T, 3>(r.tnodes, cur, nd);
            qc.nodes++;
            const bool h0 = !(nd.t0 < T(0)) &&
                            fmax(box_d2<T, 3>(nd.lo0, nd.hi0, x), slab_d2<T, 3>(nd.n0, nd.o0, nd.t0, x)) < R2;
            const bool h1 = !(nd.t1 < T(0)) &&
                            fmax(box_d2<T, 3>(nd.lo1, nd.hi1, x), slab_d2<T, 3>(nd.n1, nd.o1, nd.t1, x)) < R2;
            if (h0 && h1) {
                if (sp < kStackSize) {
                    st.put(sp, nd.c1, T(0));
                    ++sp;
                } else {
                    qc.overflow++;
                }
                cur = nd.c0;
            } else if (h0) {
                cur = nd.c0;
            } else if (h1) {
                cur = nd.c1;
            } else {
                have = false;
            }
        } else {
            const int32_t v = -1 - cur;
            const int32_t start = v >> 3, n = (v & 7) + 1;
            for (int32_t i = start; i < start + n; ++i) {
                T P[9], bb[3];
                tri_load<T>(r, i, P);
                qc.prims++;
                if (!(prim_closest<T, 3>(P, x, bb) < R2)) continue;
                const T e1[3] = {P[3] - P[0], P[4] - P[1], P[5] - P[2]};
                const T e2[3] = {P[6] - P[0], P[7] - P[1], P[8] - P[2]};
                T cr[3];
                cross3d<T>(e1, e2, cr);
                const T A = T(0.5) * sqrt(dot3d<T>(cr, cr));
                L += A;
                const uint32_t o = (uint32_t)r.torig[i];
                const u4 w = philox10(u4{ctr.x, ctr.y, ctr.z, ctr.w | 8u | (o << 16)}, key0, key1);
                const T e = -log(unif_pos<T>(w.x)) / A;
                if (e < best) {
                    best = e;
                    win = i;
                    ww = w;
                }
            }
            have = false;
        }
        if (!have && sp > 0) {
            --sp;
            cur = st.get_node(sp);
            have = true;
        }
    }
    if (win < 0) return -1;
    T P[9];
    tri_load<T>(r, win, P);
    const T rr = sqrt(unif<T>(ww.y)), tt = unif<T>(ww.z);
    T d2 = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        z[c] = (T(1) - rr) * P[c] + rr * (T(1) - tt) * P[3 + c] + rr * tt * P[6 + c];
        d2 += (z[c] - x[c]) * (z[c] - x[c]);
    }
    branch = ww.w;
    return d2 < R2 ? win : -1;
}

// ---------------------------------------------------------------------------
// the walk-on-stars kernel (3D)
//   MODE 0: forward walks, rec_u = walk estimate
//   MODE 1: differential walks with the joint u estimate and K nested
//           walks on stars from xbar - delta n at the Dirichlet terminal
// start_tri (per point row of X: original reflecting triangle or -1; NULL:
// none): walks of that point start on the triangle with the domain on its
// left normal.
// ---------------------------------------------------------------------------
// FP32: four wavefronts per SIMD (at most 128 registers per lane; the
// compiler took 150 for the differential kernel, three wavefronts).  The
// LDS staging of about 40 KB per 256-thread block admits four blocks per
// CU, i.e. four wavefronts per SIMD, so asking for more only spills: on the
// 3D thermal stand-in (W = 32, three runs each) 791 / 805 ms against 814 /
// 824 ms at five / six wavefronts (937 / 996 ms at the compiler's choice).
template <class T, int MODE>
struct Wost3Waves { static constexpr int v = sizeof(T) == 4 ? 4 : 1; };

template <class T, int MODE>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(Wost3Waves<T, MODE>::v)))
wost3_kernel(WalkArgs<T> a, RefScene3<T> ref, const int32_t* start_tri) {
    constexpr int D = 3;
    const int lane = threadIdx.x & 63;
    TravStack<T, false> stack;
    StageView sv{0, -1};
    if constexpr (sizeof(T) == 4) {
        // LDS: the Dirichlet BVH's first nodes (and its primitives when they fit)
        const int64_t nn4 = (int64_t)a.s.n_stage_nodes * (node_scalars(D) / 4);
        const float4* gn = reinterpret_cast<const float4*>(a.s.nodes);
        for (int64_t i = threadIdx.x; i < nn4; i += blockDim.x) g_stage[i] = gn[i];
        if (a.s.stage_prims) {
            const int64_t np4 = a.s.n_prims * (prim_scalars(D) / 4);
            const float4* gp = reinterpret_cast<const float4*>(a.s.prims);
            for (int64_t i = threadIdx.x; i < np4; i += blockDim.x) g_stage[nn4 + i] = gp[i];
        }
        // ... and the edge BVH's first nodes with their cones
        if (ref.n_estage > 0) {
            const int64_t en4 = (int64_t)ref.n_estage * (node_scalars(D) / 4);
            const int64_t ec4 = (int64_t)ref.n_estage * (2 * kEdgeCone / 4);
            const float4* ge = reinterpret_cast<const float4*>(ref.enodes);
            const float4* gc = reinterpret_cast<const float4*>(ref.econes);
            for (int64_t i = threadIdx.x; i < en4; i += blockDim.x) g_stage[ref.estage_off4 + i] = ge[i];
            for (int64_t i = threadIdx.x; i < ec4; i += blockDim.x) g_stage[ref.estage_off4 + en4 + i] = gc[i];
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
    int64_t wid = -1;
    T x[D], xoff[D], nin[D];
    T acc = T(0), u_main = T(0), usum = T(0);
    T tau = T(1), tau_main = T(1);
    T kappa = T(0), eps = T(1), delta = T(1);
    uint32_t k = 0, m = 0, p = 0;
    int64_t first_row = 0;
    int32_t root = 0, warm = -1, term_leaf = -1, term_code = -1, phase = 0, on = -1;
    T term_b1 = T(0), term_b2 = T(0);
    int64_t wsteps = 0;
    SilQuery<T> sq;
    sq.have = false;
    bool spend = false;
    bool sexact = true;    // sd2 is the Dirichlet distance (else an upper bound)
    int32_t swarm = -1;    // the previous step's closest silhouette edge, or -1
    T sd2 = T(0);
    int32_t sleaf = -1;
    unsigned long long c_walks = 0, c_nested = 0, c_steps = 0, c_term = 0, c_trunc = 0,
                       c_nodes = 0, c_prims = 0, c_ovf = 0, c_invalid = 0;
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
                    const Instance<T> in = a.inst[0];
                    const int64_t local = gid - in.walk_begin;
                    int64_t pin = local / a.W;
                    m = (uint32_t)(local - pin * a.W);
                    if (a.perm) {   // the slot's point; records stay indexed by point
                        pin = a.perm[pin];
                        wid = pin * a.W + m;
                    }
                    p = (uint32_t)(pin + in.p_counter);
                    root = in.root;
                    kappa = in.kappa; eps = in.eps; delta = in.delta;
                    const int64_t row = in.point_begin + pin;
                    const double* xp = a.X + (size_t)row * D;
                    first_row = row - a.x_base;
#pragma unroll
                    for (int i = 0; i < D; ++i) x[i] = T(xp[i]);
                    on = -1;
                    if (start_tri && start_tri[row] >= 0) {
                        on = ref.tleaf_of[start_tri[row]];
                        tri_left_normal<T>(ref, on, nin);
                        keep_on_domain_side3<T>(ref, on, nin, x);
                    }
                    acc = T(0); k = 0; warm = -1; phase = 0; usum = T(0); wsteps = 0;
                    tau = T(1);
                    c_walks++;
                }
            }
        }
        if (__ballot(!done) == 0ull) break;
        if (done) continue;

        QueryCount qc{0, 0, 0};
        bool finished = false;
        T result = T(0);
        bool at_term = false;   // the walk reached the Dirichlet boundary (or the cap)
        T td2 = T(0);
        int32_t tleaf = -1;
        const bool cap = (int)(k + 1) >= a.prm.kmax;
        if (!spend) {
            // ---- Dirichlet distance, or an upper bound of it -------------------
            // The step's radius is min(Dirichlet distance, closest silhouette).
            // Away from the cap and the walk's first step the silhouette query
            // runs first, bounded by the distance to the previous step's
            // closest primitive (warm), and the Dirichlet query afterwards
            // only within max(silhouette distance, eps): nearer primitives
            // are found exactly as by the full query, and when there is none
            // the radius is the silhouette distance.  Same radius, same
            // terminals.
            T d2 = T(0);
            int32_t leaf = -1;
            bool executed = true;
            sexact = true;
            if (a.first_leaf && phase == 0 && k == 0) {
                leaf = a.first_leaf[first_row];
                d2 = a.first_d2[first_row];
                executed = m == 0;
            } else if (warm >= 0 && !cap) {
                T P[9], bb[3];
                scene_prim<T, D>(a.s, sv, warm, P);
                d2 = prim_closest<T, D>(P, x, bb);
                qc.prims++;
                leaf = warm;
                sexact = false;
            } else {
                leaf = closest_leaf<T, D>(a.s, sv, root, x, warm, d2, qc, stack);
            }
            if (executed) c_steps++;
            wsteps++;
            if (leaf < 0 || !(d2 >= T(0))) {
                c_invalid++;
                const T nanv = T(NAN);
                a.rec_u[wid] = nanv;
                if (MODE == 1) {
                    a.rec_prim[wid] = -1;
                    a.rec_uoff[wid] = nanv;
                    if (a.rec_w) a.rec_w[wid] = T(1);
                }
                if (a.rec_steps) a.rec_steps[wid] = wsteps;
                wid = -1;
                c_nodes += qc.nodes; c_prims += qc.prims; c_ovf += qc.overflow;
                continue;
            }
            if (sexact && (sqrt(d2) < eps || cap)) {
                at_term = true;
                td2 = d2;
                tleaf = leaf;
            } else {
                // seed: the previous closest silhouette edge, if it still is one
                T sb = d2;
                int32_t bs = -1;
                if (swarm >= 0) {
                    qc.prims++;
                    if (sil3_edge_nearer<T>(ref, swarm, x, on, nin, sb)) bs = swarm;
                }
                sil_begin<T>(sq, sb, bs);
                spend = true;
                sd2 = d2;
                sleaf = leaf;
            }
        }
        // ---- closest silhouette edge (resumable) -------------------------------
        {
#pragma unroll 1
            while (true) {
                const bool trav = spend && sq.have;
                const unsigned long long sm = __ballot(trav);
                const unsigned long long present = __ballot(true);
                if (sm == 0ull || __popcll(present & ~sm) >= a.park) break;
                if (trav) sil3_round<T>(ref, x, on, nin, sq, qc, stack, a.s.tail);
            }
        }
        if (spend && sq.have) {
            c_nodes += qc.nodes; c_prims += qc.prims; c_ovf += qc.overflow;
            continue;
        }
        if (spend) {
            spend = false;
            swarm = sq.bsil;
            // radius floor of 16 units of rounding of the position (see the 2D
            // kernel); sfl: the silhouette distance with that floor
            const T ulp = sizeof(T) == 4 ? T(1.1920929e-07) : T(2.220446049250313e-16);
            const T rmin = T(16) * ulp * (fabs(x[0]) + fabs(x[1]) + fabs(x[2]));
            const T sfl = fmax(sqrt(sq.best), rmin);
            T d;   // the Dirichlet distance, or a lower bound of it that is >= sfl
            if (sexact) {
                d = sqrt(sd2);
            } else {
                // primitives nearer than B = max(sfl, eps); the bound is padded
                // so that finding none proves a distance above B
                const T B = fmax(sfl, eps);
                const T B2 = B * B * (sizeof(T) == 4 ? T(1.00001) : T(1.0000000001));
                T d2b;
                const int32_t lb = closest_leaf_within<T, D>(a.s, sv, root, x, sleaf, sd2, B2, d2b, qc, stack);
                if (lb >= 0) {
                    d = sqrt(d2b);
                    sleaf = lb;
                    if (d < eps) {
                        at_term = true;
                        td2 = d2b;
                        tleaf = lb;
                    }
                } else {
                    d = B;
                }
            }
            if (!at_term) {
                const bool nested = MODE == 1 && phase > 0;
                // ---- one step on the star-shaped region ---------------------------
                T R = fmin(d, sfl);
                if (ref.mu > T(0)) R = fmin(R, fmax(T(1) / ref.mu, rmin));
                const uint32_t tag = nested ? (1u | ((uint32_t)(phase - 1) << 8)) : 0u;
                const u4 r = philox10(u4{k, m, p, tag}, key0, key1);
                T dir[3];
                unit_dir<T, D>(r.x, r.y, dir);
                if (on >= 0) {
                    const T c = dot3d<T>(dir, nin);
                    if (c < T(0)) {
#pragma unroll
                        for (int cc = 0; cc < 3; ++cc) dir[cc] -= T(2) * c * nin[cc];
                    }
                }
                T t;
                const T reach = R + T(8) * ulp * (fabs(x[0]) + fabs(x[1]) + fabs(x[2]) + R);
                int32_t tri = ray3_first<T>(ref, x, dir, reach, on, t, qc, stack);
                if (tri < 0) t = R;
                if (a.prm.has_source) {
                    const T rho = cbrt(unif_pos<T>(r.w));
                    if (tri < 0 || rho * R < t) {
                        T y[3];
#pragma unroll
                        for (int c = 0; c < D; ++c) y[c] = x[c] + rho * R * dir[c];
                        acc += tau * green_ball_t<D, T>(kappa, rho, R) * source_f<T, D>(a.prm, y);
                    }
                }
                T zr[3] = {T(0), T(0), T(0)}, Lz = T(0), Gz = T(0);
                int32_t zleaf = -1;
                uint32_t wbranch = 0;
                const T cx = on >= 0 ? T(2) : T(1);
                if (ref.robin) {
                    zleaf = ref3_boundary_sample<T>(ref, x, R, u4{k, m, p, tag}, key0, key1, Lz, zr, wbranch, qc, stack);
                    if (zleaf >= 0) {
                        const T dz[3] = {zr[0] - x[0], zr[1] - x[1], zr[2] - x[2]};
                        const T rz = fmax(sqrt(dot3d<T>(dz, dz)), rmin);
                        // G(r; R) = (G |B_R|) / |B_R|
                        Gz = green_ball_t<D, T>(kappa, fmin(rz / R, T(1)), R) /
                             (T(4.18879020478639098462) * R * R * R);
                        acc -= tau * cx * Lz * Gz * robin_data3<T>(ref, zr);
                    }
                }
                const T q = (ref.mu > T(0) && zleaf >= 0) ? fmin(T(0.5), cx * ref.mu * Lz * Gz) : T(0);
                const bool to_z = q > T(0) && unif<T>(wbranch) < q;
                const T wgt = to_z ? -cx * ref.mu * Lz * Gz / q
                                   : (tri >= 0 ? reflect_weight<D, T>(kappa, t, R) : poisson_scale<T, D>(kappa, R)) /
                                         (T(1) - q);
                const T keep = fmin(T(1), fabs(wgt));
                if (a.prm.rr && (!(keep > T(0)) || keep < unif<T>(r.z))) {
                    finished = true;
                    result = acc;
                    if (MODE == 1 && phase == 0) term_code = -1;
                } else {
                    tau *= a.prm.rr ? wgt / keep : wgt;
                    if (MODE == 1 && phase == 0) {
#pragma unroll
                        for (int c = 0; c < D; ++c) xoff[c] = x[c];   // previous position
                    }
                    if (to_z) {   // continue on the wall at z
#pragma unroll
                        for (int c = 0; c < D; ++c) x[c] = zr[c];
                        on = zleaf;
                    } else {
#pragma unroll
                        for (int c = 0; c < D; ++c) x[c] += t * dir[c];
                        on = tri;
                    }
                    if (on >= 0) {   // the domain is on the wall's left normal side
                        tri_left_normal<T>(ref, on, nin);
                        keep_on_domain_side3<T>(ref, on, nin, x);
                    }
                    ++k;
                    warm = sleaf;
                }
            }
        }
        if (at_term) {
            const T d = sqrt(td2);
            const int32_t leaf = tleaf;
            if (cap && !(d < eps)) c_trunc++;
            T P[9], bary[3];
            scene_prim<T, D>(a.s, sv, leaf, P);
            prim_closest<T, D>(P, x, bary);
            const int32_t orig = a.s.orig[leaf];
            T V[9];
            int32_t vid[3];
            prim_vertices<T, D>(a.s, orig, V, vid);
            T xbar[3];
#pragma unroll
            for (int c = 0; c < D; ++c) {
                T v = T(0);
#pragma unroll
                for (int kk = 0; kk < D; ++kk) v += bary[kk] * V[kk * D + c];
                xbar[c] = v;
            }
            const T g = boundary_value<T, D>(a.s, a.prm, orig, bary, xbar, vid);
            if (MODE == 1 && phase == 0) {
                T n[3] = {T(0), T(0), T(0)};
                geo_normal<T, D>(V, n);
                // oriented away from the previous position (held in xoff
                // until now), or the start point
                T dn = T(0);
#pragma unroll
                for (int c = 0; c < D; ++c) dn += n[c] * (xbar[c] - (k > 0 ? xoff[c] : x[c]));
                const int flip = dn < T(0) ? 1 : 0;
                if (flip) {
#pragma unroll
                    for (int c = 0; c < D; ++c) n[c] = -n[c];
                }
                u_main = acc + tau * g;
                tau_main = tau;
                term_code = orig * 2 + flip;
                term_b1 = bary[1];
                term_b2 = bary[2];
                term_leaf = leaf;
#pragma unroll
                for (int c = 0; c < D; ++c) xoff[c] = xbar[c] - delta * n[c];
                c_term++;
                if (a.prim_dep && !a.prim_dep[orig]) {
                    a.rec_u[wid] = u_main;
                    a.rec_prim[wid] = term_code;
                    a.rec_b[(size_t)wid * 2] = term_b1;
                    a.rec_b[(size_t)wid * 2 + 1] = term_b2;
                    a.rec_uoff[wid] = g;
                    if (a.rec_w) a.rec_w[wid] = tau_main;
                    if (a.rec_steps) a.rec_steps[wid] = wsteps;
                    wid = -1;
                    c_nodes += qc.nodes; c_prims += qc.prims; c_ovf += qc.overflow;
                    continue;
                }
                // the first nested walk on stars starts at the offset point
                phase = 1;
#pragma unroll
                for (int c = 0; c < D; ++c) x[c] = xoff[c];
                acc = T(0); k = 0; warm = term_leaf; on = -1; tau = T(1);
                c_nested++;
                c_nodes += qc.nodes; c_prims += qc.prims; c_ovf += qc.overflow;
                continue;
            }
            finished = true;
            result = acc + tau * g;
        }
        c_nodes += qc.nodes; c_prims += qc.prims; c_ovf += qc.overflow;
        if (!finished) continue;

        if (MODE == 0) {
            a.rec_u[wid] = result;
            if (a.rec_steps) a.rec_steps[wid] = wsteps;
            wid = -1;
        } else if (phase == 0) {
            a.rec_u[wid] = result;
            a.rec_prim[wid] = -1;
            a.rec_uoff[wid] = T(0);
            if (a.rec_w) a.rec_w[wid] = T(1);
            if (a.rec_steps) a.rec_steps[wid] = wsteps;
            wid = -1;
        } else {
            usum += result;
            if (phase >= a.prm.K) {
                a.rec_u[wid] = u_main;
                a.rec_prim[wid] = term_code;
                a.rec_b[(size_t)wid * 2] = term_b1;
                a.rec_b[(size_t)wid * 2 + 1] = term_b2;
                a.rec_uoff[wid] = usum / T(a.prm.K);
                if (a.rec_w) a.rec_w[wid] = tau_main;
                if (a.rec_steps) a.rec_steps[wid] = wsteps;
                wid = -1;
            } else {
                ++phase;
#pragma unroll
                for (int c = 0; c < D; ++c) x[c] = xoff[c];
                acc = T(0); k = 0; warm = term_leaf; on = -1; tau = T(1);
                c_nested++;
            }
        }
    }
    c_walks = wave_sum_u64(c_walks);
    c_nested = wave_sum_u64(c_nested);
    c_steps = wave_sum_u64(c_steps);
    c_term = wave_sum_u64(c_term);
    c_nodes = wave_sum_u64(c_nodes);
    c_prims = wave_sum_u64(c_prims);
    c_trunc = wave_sum_u64(c_trunc);
    c_ovf = wave_sum_u64(c_ovf);
    c_invalid = wave_sum_u64(c_invalid);
    if (lane == 0) {
        Counters* dst[2] = {a.cnt, a.tot};
        for (int q = 0; q < 2; ++q) {
            Counters* c = dst[q];
            atomicAdd(&c->walks, c_walks);
            atomicAdd(&c->nested, c_nested);
            atomicAdd(&c->steps, c_steps);
            atomicAdd(&c->terminal, c_term);
            atomicAdd(&c->nodes, c_nodes);
            atomicAdd(&c->prims, c_prims);
            if (c_trunc) atomicAdd(&c->truncated, c_trunc);
            if (c_ovf) atomicAdd(&c->overflow, c_ovf);
            if (c_invalid) atomicAdd(&c->invalid, c_invalid);
        }
    }
}

// Closest silhouette distance and first ray hit for query rows (parity
// checks of the two 3D reflecting-boundary queries).  out per row: {silhouette
// distance capped at cap[row], ray t (cap[row] if none), hit as an original
// triangle index or -1}.  on: original triangle or -1; a row with any other
// value gets NaN outputs.
template <class T>
__global__ void ref3_query_kernel(RefScene3<T> ref, const double* X, const double* dir, const double* cap,
                                  const int32_t* on_orig, const double* nin, int64_t n, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T x[3], dv[3], nn[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = T(X[3 * i + c]);
        dv[c] = T(dir[3 * i + c]);
        nn[c] = T(nin[3 * i + c]);
    }
    const int32_t oo = on_orig[i];
    if (oo < -1 || oo >= ref.nt) {
        out[3 * i] = out[3 * i + 1] = out[3 * i + 2] = NAN;
        return;
    }
    const int32_t on = oo >= 0 ? ref.tleaf_of[oo] : -1;
    QueryCount qc{0, 0, 0};
    TravStack<T, false> st;
    const T c = T(cap[i]);
    out[3 * i] = double(sqrt(silhouette3_d2<T>(ref, x, on, nn, c * c, qc, st)));
    T t;
    const int32_t hit = ray3_first<T>(ref, x, dv, c, on, t, qc, st);
    out[3 * i + 1] = double(t);
    out[3 * i + 2] = hit >= 0 ? double(ref.torig[hit]) : -1.0;
}

}  // namespace dwos
