// Walk on stars on gfx950: the screened Poisson problem with a Dirichlet
// boundary and a fixed zero-flux (reflecting) boundary, 2D (the mixed
// problem of Sec. 3.4 with Robin coefficient and data 0, and its
// differential version of Sec. 4.4, which nests through the Dirichlet
// boundary only).  The paper defers the estimator to the walk-on-stars
// papers; one step, as implemented here:
//   * d = distance to the Dirichlet boundary (the Dirichlet BVH); in its
//     eps-shell the walk ends as in Algorithm 1 / Algorithm 2.
//   * star radius R = min(d, distance to the closest silhouette vertex of the
//     reflecting boundary), so that the part of B(x, R) visible from x is
//     star-shaped and bounded by the sphere and the reflecting boundary only.
//   * a direction v uniform on the circle (at a reflecting boundary point:
//     the half entering the domain, by reflection of the other half); the
//     first reflecting segment hit along v before R is the next point, with
//     weight reflect_weight(t, R), else x + R v with weight alpha(R);
//     Russian roulette on the weight.
//   * source: y = x + rho v along the same direction, counted if rho < t.
// Random numbers: one Philox draw per step, word 0 the direction, word 2 the
// roulette, word 3 the source radius.
//
// The persistent kernel and its records are those of the walk-on-spheres
// kernel (one walk per lane, wave-level work queue, per-walk records reduced
// afterwards), so every reduction kernel applies unchanged.
#pragma once
#include "walk_kernels.hpp"

namespace dwos {

// Reflecting segments with a pair-node BVH in the layout of bvh.hpp.  Per
// segment in leaf order:
//   geo  (8 scalars): a[2] b[2] na[2] nb[2] -- the endpoints and, for each,
//        the far end of the other segment at that vertex (unused if none);
//   info (int4): flags, leaf of the other segment at a, at b (-1 none),
//        original index.
// flags: 1 this segment tests vertex a, 2 vertex b (every vertex is tested
// by one of its segments); 4 vertex a is always a silhouette (an open end or
// a vertex of more than two segments), 8 the same for b.
constexpr int kRefGeo = 8;

// Normal cones of the silhouette query, per node and child (8 scalars
// each): a unit axis a, sin and cos of s0 = theta + margin, the range
// [omin, omax] of a.p over the child's segment endpoints p, kappa and a pad;
// theta the largest angle between a and the normals involved in the child's
// vertex tests (its segments' and, at each vertex it tests, the other
// segment's, all oriented along the polyline through that vertex).  A
// vertex is a silhouette only if x is in front of one of its segments'
// lines and behind the other's (or sees one edge-on).  Two tests show a
// child holds none: (view cone) the view direction v - x is then
// perpendicular to some normal of the cone, so a child whose view cone
// (from x, half-angle beta over the child box's bounding circle) keeps every
// such dot product of one sign, i.e. |cos angle(a, c - x)| > sin(s0 + beta)
// with s0 + beta < pi/2, holds none; (lines) for a segment with unit normal
// n through the tested vertex p, n.(x - p) >= a.x - omax - 2 sin(s0/2)
// |x - p|, so a.x - omax > (2 sin(s0/2) + kappa) dmax (dmax >= |x - p| over
// the child's box) puts x in front of every such line by more than kappa
// |x - p|, and omin - a.x beyond the same bound behind all of them; kappa =
// 4 tol keeps every segment clear of the edge-on tolerance tol (seen
// edge-on means a distance from the line below tol |x - p|).  The cone
// margin covers the edge-on tolerance and rounding, the line test a floor
// of 32 units of rounding; children that hold an always-silhouette vertex,
// or whose normals spread by pi/2 or more, store sin = 2, cos = -1 (never
// pruned).
constexpr int kRefCone = 8;

template <class T>
struct RefScene {
    const T* nodes;
    const T* geo;
    const int4* info;
    const int32_t* leaf_of;   // original segment -> leaf position
    const T* cones;           // per node: child 0 then child 1, kRefCone each
    int64_t n;
    // FP32 walk kernel: the first n_stage nodes (breadth-first, the top
    // levels every query visits) and their cones are copied to LDS at
    // g_stage + stage_off4 (16-byte words: nodes, then cones); 0: none
    int32_t n_stage;
    int64_t stage_off4;
    // Robin condition du/dn - mu u = h on the reflecting boundary (n into
    // the domain) with h = hq[0] + hq[1] x + hq[2] y + [x y] [hq[3] hq[4];
    // hq[5] hq[6]] [x y]^T; robin = 0: zero flux (mu = 0, h = 0)
    int32_t robin;
    T mu;
    T hq[7];
};

// Robin data h at a reflecting boundary point z
template <class T>
__device__ __forceinline__ T robin_data(const RefScene<T>& r, const T* z) {
    T v = r.hq[0] + r.hq[1] * z[0] + r.hq[2] * z[1];
    v += z[0] * r.hq[3] * z[0] + z[0] * r.hq[4] * z[1];
    v += z[1] * r.hq[5] * z[0] + z[1] * r.hq[6] * z[1];
    return v;
}

// Length of the part of leaf segment i inside the disk |z - x| < R, and its
// parameter interval [t0, t1] along the segment from its first vertex.
template <class T>
__device__ __forceinline__ T ref_clip(const RefScene<T>& r, int32_t i, const T* x, T R, T& t0, T& t1) {
    const T* g = r.geo + (size_t)i * kRefGeo;
    const T ex = g[2] - g[0], ey = g[3] - g[1];
    const T ax = g[0] - x[0], ay = g[1] - x[1];
    const T ee = ex * ex + ey * ey, ea = ex * ax + ey * ay;
    const T disc = ea * ea - ee * (ax * ax + ay * ay - R * R);
    if (!(disc > T(0))) return T(0);
    const T sq = sqrt(disc);
    t0 = fmax(T(0), (-ea - sq) / ee);
    t1 = fmin(T(1), (-ea + sq) / ee);
    if (!(t1 > t0)) return T(0);
    return sqrt(ee) * (t1 - t0);
}

// A point z uniform by length on the reflecting boundary inside the disk
// B(x, R) and that length L; returns the leaf of z's segment, or -1 (L = 0)
// when the disk holds no reflecting point.  The segment is chosen with
// probability proportional to its clipped length by an exponential race:
// every segment o in the disk draws E_o = -ln(U_o) / l_o from its own
// Philox counter (k, m, p, tag | 8 | o << 16) -- `ctr` holds the step's
// (k, m, p, tag) -- and the smallest E_o wins, so the choice does not
// depend on the order of the traversal; the position along the winner's
// clipped part is word 1 of the same draw.
template <class T, class Stack>
__device__ int32_t ref_boundary_sample(const RefScene<T>& r, const T* x, T R, u4 ctr, uint32_t key0,
                                       uint32_t key1, T& L, T* z, QueryCount& qc, Stack& st) {
    const T R2 = R * R;
    L = T(0);
    int32_t win = -1;
    T best = T(INFINITY), wt0 = T(0), wt1 = T(0);
    uint32_t wpos = 0;
    int sp = 0;
    int32_t cur = 0;
    bool have = true;
#pragma unroll 1
    while (have) {
        if (cur >= 0) {
            NodeData<T, 2> nd;
            ref_node<T>(r, cur, nd);
            qc.nodes++;
            const bool h0 = !(nd.t0 < T(0)) &&
                            fmax(box_d2<T, 2>(nd.lo0, nd.hi0, x), slab_d2<T, 2>(nd.n0, nd.o0, nd.t0, x)) < R2;
            const bool h1 = !(nd.t1 < T(0)) &&
                            fmax(box_d2<T, 2>(nd.lo1, nd.hi1, x), slab_d2<T, 2>(nd.n1, nd.o1, nd.t1, x)) < R2;
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
                T t0 = T(0), t1 = T(0);
                const T l = ref_clip<T>(r, i, x, R, t0, t1);
                qc.prims++;
                if (!(l > T(0))) continue;
                L += l;
                const uint32_t o = (uint32_t)r.info[i].w;
                const u4 w = philox10(u4{ctr.x, ctr.y, ctr.z, ctr.w | 8u | (o << 16)}, key0, key1);
                const T e = -log(unif_pos<T>(w.x)) / l;
                if (e < best) {
                    best = e;
                    win = i;
                    wt0 = t0;
                    wt1 = t1;
                    wpos = w.y;
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
    if (win >= 0) {
        const T* g = r.geo + (size_t)win * kRefGeo;
        const T t = wt0 + unif<T>(wpos) * (wt1 - wt0);
        z[0] = g[0] + t * (g[2] - g[0]);
        z[1] = g[1] + t * (g[3] - g[1]);
    }
    return win;
}

// A reflecting-BVH node and its children's cones, from LDS for the staged
// prefix, from global memory otherwise.
template <class T>
__device__ __forceinline__ void ref_node(const RefScene<T>& r, int32_t i, NodeData<T, 2>& nd) {
    if constexpr (sizeof(T) == 4) {
        if (i < r.n_stage) {
            decode_node_f32<2>(g_stage + r.stage_off4 + (int64_t)i * (node_scalars(2) / 4), nd);
            return;
        }
    }
    load_node<T, 2>(r.nodes, i, nd);
}

template <class T>
__device__ __forceinline__ void ref_cones(const RefScene<T>& r, int32_t i, T* q) {
    if constexpr (sizeof(T) == 4) {
        if (i < r.n_stage) {
            const float4* w = g_stage + r.stage_off4 + (int64_t)r.n_stage * (node_scalars(2) / 4) +
                              (int64_t)i * (2 * kRefCone / 4);
#pragma unroll
            for (int k = 0; k < 2 * kRefCone / 4; ++k) {
                const float4 v = w[k];
                q[4 * k] = v.x; q[4 * k + 1] = v.y; q[4 * k + 2] = v.z; q[4 * k + 3] = v.w;
            }
            return;
        }
    }
    const T* g = r.cones + (size_t)i * (2 * kRefCone);
#pragma unroll
    for (int k = 0; k < 2 * kRefCone; ++k) q[k] = g[k];
}

// Can the child with box lo..hi and cone q hold a silhouette seen from x?
template <class T>
__device__ __forceinline__ bool cone_may_hold(const T* lo, const T* hi, const T* q, const T* x) {
    if (!(q[2] <= T(1))) return true;     // never pruned
    const T cx = T(0.5) * (lo[0] + hi[0]) - x[0], cy = T(0.5) * (lo[1] + hi[1]) - x[1];
    const T ex = T(0.5) * (hi[0] - lo[0]), ey = T(0.5) * (hi[1] - lo[1]);
    const T d2 = cx * cx + cy * cy, r2 = ex * ex + ey * ey;
    {   // lines: x in front of (or behind) every segment line of the child
        const T ulp = sizeof(T) == 4 ? T(1.1920929e-07) : T(2.220446049250313e-16);
        const T ax = q[0] * x[0] + q[1] * x[1];
        const T dmax = sqrt(d2) + sqrt(r2);
        const T mag = fabs(x[0]) + fabs(x[1]) + fabs(lo[0]) + fabs(lo[1]) + fabs(hi[0]) + fabs(hi[1]);
        const T marg = (sqrt(fmax(T(0), T(2) - T(2) * q[3])) + q[6]) * dmax + T(32) * ulp * (mag + dmax);
        if (ax - q[5] > marg || q[4] - ax > marg) return false;
    }
    if (!(d2 > r2)) return true;          // x inside the bounding circle
    const T inv = T(1) / sqrt(d2);
    const T sb = sqrt(r2) * inv, cb = sqrt(T(1) - sb * sb);
    const T cs = q[3] * cb - q[2] * sb;   // cos(s0 + beta)
    if (!(cs > T(0))) return true;
    const T ss = q[2] * cb + q[3] * sb;   // sin(s0 + beta)
    return !(fabs((q[0] * cx + q[1] * cy) * inv) > ss);
}

// Relative size below which a cross product counts as zero in the silhouette
// test (an edge seen edge-on): well above the rounding of the working
// precision, far below any geometric angle of interest.
template <class T> struct SilTol;
template <> struct SilTol<float> { static constexpr float v = 1e-4f; };
template <> struct SilTol<double> { static constexpr double v = 1e-10; };

// How far (relative to the coordinates' magnitude) a ray origin may lie
// behind a wall and still be taken as on its domain side: a few units of
// rounding of the working precision.
template <class T> struct kBehind;
template <> struct kBehind<float> { static constexpr float v = 16 * 1.1920929e-07f; };
template <> struct kBehind<double> { static constexpr double v = 16 * 2.220446049250313e-16; };

// Is vertex v a silhouette point seen from x?  u, w: the far ends of its two
// segments; own = 1 if u's segment is the one x lies on, 2 if w's, else 0.
// Seen from x the boundary turns back at v iff both segments leave v on the
// same side of the line through x and v.  A segment seen edge-on does not
// decide: on the reflecting boundary (domain side nin) v is then a silhouette
// iff the other segment leaves to the outside of that line; off it, an
// edge-on view counts as a silhouette.
template <class T>
__device__ __forceinline__ bool sil_test(const T* v, const T* u, const T* w, int own, const T* x,
                                         const T* nin, bool on) {
    auto outside = [&](const T* q) { return nin[0] * (q[0] - v[0]) + nin[1] * (q[1] - v[1]) < T(0); };
    if (own == 1) return outside(w);
    if (own == 2) return outside(u);
    const T vx = v[0] - x[0], vy = v[1] - x[1];
    const T lv = sqrt(vx * vx + vy * vy);
    const T ux = u[0] - v[0], uy = u[1] - v[1], wx = w[0] - v[0], wy = w[1] - v[1];
    const T cu = vx * uy - vy * ux, cw = vx * wy - vy * wx;
    const bool zu = fabs(cu) <= SilTol<T>::v * lv * sqrt(ux * ux + uy * uy);
    const bool zw = fabs(cw) <= SilTol<T>::v * lv * sqrt(wx * wx + wy * wy);
    if (zu && zw) return false;
    if (zu || zw) return on ? outside(zu ? w : u) : true;
    return (cu > T(0)) == (cw > T(0));
}

// Closest silhouette vertex as a resumable query: the traversal state of one
// lane (node to visit next or a held leaf, stack depth, best squared
// distance so far).  sil_round expands nodes, then tests a leaf; a lane keeps
// its state (and its entries in the traversal stack) across iterations of
// the walk loop, so a wavefront can take its step once enough lanes are
// answered (see wost_kernel).  x lies on leaf segment `on` (domain side nin)
// or inside (-1).
template <class T>
struct SilQuery {
    int32_t cur;   // node (>= 0) or leaf reference (< 0) to process next
    int32_t sp;    // entries in the traversal stack
    bool have;     // cur is valid; false once the query is answered
    T best;        // squared distance of the closest silhouette so far
    int32_t bsil;  // the silhouette at that distance (3D: leaf edge), or -1
};

template <class T>
__device__ __forceinline__ void sil_begin(SilQuery<T>& q, T best, int32_t bsil = -1) {
    q.cur = 0;   // the root pair node
    q.sp = 0;
    q.have = true;
    q.best = best;
    q.bsil = bsil;
}

// Answer the next entry of the traversal stack still nearer than the best
// distance, or end the query when none is left.
template <class T, class Stack>
__device__ __forceinline__ void sil_pop(SilQuery<T>& q, Stack& st) {
    q.have = false;
#pragma unroll 1
    while (q.sp > 0) {
        --q.sp;
        if (st.get_d(q.sp) < q.best) {
            q.cur = st.get_node(q.sp);
            q.have = true;
            break;
        }
    }
}

// One round of the query: expand nodes until the lane holds a leaf or is
// answered, then the lanes holding leaves test them together; with tail > 0
// the expansion stops once at most `tail` lanes still descend while some
// lane holds a leaf (those go on in the next round), as in the closest-point
// query.  Each lane visits the same nodes and vertices in the same order
// whatever the tail, so the answer does not depend on it.
template <class T, class Stack>
__device__ __forceinline__ void sil_round(const RefScene<T>& r, const T* x, int32_t on, const T* nin,
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
        NodeData<T, 2> nd;
        ref_node<T>(r, q.cur, nd);
        qc.nodes++;
        const T d0 = fmax(box_d2<T, 2>(nd.lo0, nd.hi0, x), slab_d2<T, 2>(nd.n0, nd.o0, nd.t0, x));
        const T d1 = fmax(box_d2<T, 2>(nd.lo1, nd.hi1, x), slab_d2<T, 2>(nd.n1, nd.o1, nd.t1, x));
        T qn[2 * kRefCone];
        ref_cones<T>(r, q.cur, qn);
        const bool h0 = d0 < q.best && cone_may_hold<T>(nd.lo0, nd.hi0, qn, x);
        const bool h1 = d1 < q.best && cone_may_hold<T>(nd.lo1, nd.hi1, qn + kRefCone, x);
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
    // phase 2: the lanes holding a leaf test its vertices
    if (q.have && q.cur < 0) {
        const int32_t v = -1 - q.cur;
        const int32_t start = v >> 3, n = (v & 7) + 1;
        for (int32_t i = start; i < start + n; ++i) {
            const int4 inf = r.info[i];
            const T* g = r.geo + (size_t)i * kRefGeo;
            qc.prims++;
            if (inf.x & 1) {   // vertex a: segments i (far end b) and inf.y (far end na)
                const T dx = g[0] - x[0], dy = g[1] - x[1];
                const T d2 = dx * dx + dy * dy;
                if (d2 < q.best) {
                    const int own = on < 0 ? 0 : (on == i ? 1 : (on == inf.y ? 2 : 0));
                    if ((inf.x & 4) || sil_test<T>(g, g + 2, g + 4, own, x, nin, on >= 0)) q.best = d2;
                }
            }
            if (inf.x & 2) {   // vertex b: segments i (far end a) and inf.z (far end nb)
                const T dx = g[2] - x[0], dy = g[3] - x[1];
                const T d2 = dx * dx + dy * dy;
                if (d2 < q.best) {
                    const int own = on < 0 ? 0 : (on == i ? 1 : (on == inf.z ? 2 : 0));
                    if ((inf.x & 8) || sil_test<T>(g + 2, g, g + 6, own, x, nin, on >= 0)) q.best = d2;
                }
            }
        }
        sil_pop<T>(q, st);
    }
}

// Squared distance from x to its closest silhouette vertex, if below `best`
// (else `best`): the whole query.
template <class T, class Stack>
__device__ T silhouette_d2(const RefScene<T>& r, const T* x, int32_t on, const T* nin, T best,
                           QueryCount& qc, Stack& st) {
    SilQuery<T> q;
    sil_begin<T>(q, best);
#pragma unroll 1
    while (q.have) sil_round<T>(r, x, on, nin, q, qc, st);
    return q.best;
}

// Entry distance of the ray x + t dir (t in [0, tmax]) into a child's box
// and oriented slab, or +inf if it misses them.  inv = 1/dir per axis.
template <class T>
__device__ __forceinline__ T ray_child(const T* lo, const T* hi, const T* n, T o, T th, const T* x,
                                       const T* dir, const T* inv, T tmax) {
    if (th < T(0)) return T(INFINITY);   // empty child
    T tn = T(0), tf = tmax;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (dir[k] != T(0)) {
            const T t1 = (lo[k] - x[k]) * inv[k], t2 = (hi[k] - x[k]) * inv[k];
            tn = fmax(tn, fmin(t1, t2));
            tf = fmin(tf, fmax(t1, t2));
        } else if (x[k] < lo[k] || x[k] > hi[k]) {
            return T(INFINITY);
        }
    }
    const T pn = n[0] * dir[0] + n[1] * dir[1];
    const T q = n[0] * x[0] + n[1] * x[1] - o;
    if (pn != T(0)) {
        const T s1 = (-th - q) / pn, s2 = (th - q) / pn;
        tn = fmax(tn, fmin(s1, s2));
        tf = fmin(tf, fmax(s1, s2));
    } else if (fabs(q) > th) {
        return T(INFINITY);
    }
    return tn <= tf * Slack<T>::v + T(1e-30) ? tn : T(INFINITY);
}

// First reflecting segment (leaf position) entered from its domain side
// (its left) by x + t dir with 0 <= t < tmax, skipping leaf `skip`; -1 if
// none.  t_out: its t, or tmax.  Equal t go to the lowest original index.
template <class T, class Stack>
__device__ int32_t ray_first(const RefScene<T>& r, const T* x, const T* dir, T tmax, int32_t skip, T& t_out,
                             QueryCount& qc, Stack& st) {
    T inv[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) inv[k] = dir[k] != T(0) ? T(1) / dir[k] : T(0);
    T best = tmax;
    int32_t hit = -1;
    int sp = 0;
    int32_t cur = 0;
    bool have = true;
#pragma unroll 1
    while (have) {
        if (cur >= 0) {
            NodeData<T, 2> nd;
            ref_node<T>(r, cur, nd);
            qc.nodes++;
            const T e0 = ray_child<T>(nd.lo0, nd.hi0, nd.n0, nd.o0, nd.t0, x, dir, inv, best);
            const T e1 = ray_child<T>(nd.lo1, nd.hi1, nd.n1, nd.o1, nd.t1, x, dir, inv, best);
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
                const T* g = r.geo + (size_t)i * kRefGeo;
                qc.prims++;
                // walls are one-way: only a ray entering the wall from the
                // domain side (the segment's left) is stopped, so a walk that
                // rounding left just behind a wall passes back into the domain
                const T ex = g[2] - g[0], ey = g[3] - g[1];
                const T dn = ey * dir[0] - ex * dir[1];          // -dir . left normal (times |e|)
                if (!(dn > T(0))) continue;
                const T ax = g[0] - x[0], ay = g[1] - x[1];
                const T h = ey * ax - ex * ay;                   // height of x over the wall (times |e|)
                // an origin further behind the wall than rounding explains
                // is not on the domain side of this wall
                if (h < T(0) && h * h > kBehind<T>::v * kBehind<T>::v * (ex * ex + ey * ey) *
                                            (fabs(x[0]) + fabs(x[1]) + fabs(g[0]) + fabs(g[1])) *
                                            (fabs(x[0]) + fabs(x[1]) + fabs(g[0]) + fabs(g[1])))
                    continue;
                // the segment is crossed iff its endpoints lie on opposite
                // sides of the ray's line; a shared vertex gets the same side
                // from both of its segments (same operands, same rounding),
                // so no ray slips between two segments
                const T bx = g[2] - x[0], by = g[3] - x[1];
                const T sa = dir[0] * ay - dir[1] * ax;
                const T sb = dir[0] * by - dir[1] * bx;
                if ((sa >= T(0)) == (sb >= T(0))) continue;
                const T t = fmax(T(0), quot<T>(h, dn));
                if (t < best || (t == best && hit >= 0 && r.info[i].w < r.info[hit].w)) {
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

// unit normal to the left of leaf segment i (from its first to its second vertex)
template <class T>
__device__ __forceinline__ void ref_left_normal(const RefScene<T>& r, int32_t i, T* n) {
    const T* g = r.geo + (size_t)i * kRefGeo;
    const T tx = g[2] - g[0], ty = g[3] - g[1];
    const T inv = T(1) / sqrt(tx * tx + ty * ty);
    n[0] = -ty * inv;
    n[1] = tx * inv;
}

// Keep a point on leaf segment i a few units of rounding in front of the
// segment's line (on the domain side nin): the rounded hit point may land
// on or just behind the line, and a later step almost parallel to the wall
// would otherwise round to either side.
template <class T>
__device__ __forceinline__ void keep_on_domain_side(const RefScene<T>& r, int32_t i, const T* nin, T* x) {
    const T* g = r.geo + (size_t)i * kRefGeo;
    const T s = nin[0] * (x[0] - g[0]) + nin[1] * (x[1] - g[1]);
    const T ulp = sizeof(T) == 4 ? T(1.1920929e-07) : T(2.220446049250313e-16);
    const T margin = T(8) * ulp * (fabs(x[0]) + fabs(x[1]) + fabs(g[0]) + fabs(g[1]));
    if (s < margin) {
        x[0] += (margin - s) * nin[0];
        x[1] += (margin - s) * nin[1];
    }
}

// ---------------------------------------------------------------------------
// the walk-on-stars kernel (2D)
//   MODE 0: forward walks, rec_u = walk estimate
//   MODE 1: differential walks with the joint u estimate and K nested
//           walks on stars from xbar - delta n at the Dirichlet terminal
// start_seg (per point row of X, original reflecting segment or -1; NULL:
// none): walks of that point start on the segment with the domain on its
// left.
// ---------------------------------------------------------------------------
// FP32 differential kernel: four wavefronts per SIMD (at most 128 registers
// per lane instead of the compiler's 130, which gave three).  On the 2D
// thermal workload (W = 128, three runs each) the differential launch takes
// 306 ms against 315 ms at five wavefronts (96 registers, more spilling) and
// 333 ms at six; the forward kernel keeps the compiler's choice (four; five
// was slower, 362 against 337 ms).
template <class T, int MODE>
struct WostWaves { static constexpr int v = (sizeof(T) == 4 && MODE == 1) ? 4 : 1; };

template <class T, int MODE>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(WostWaves<T, MODE>::v)))
wost_kernel(WalkArgs<T> a, RefScene<T> ref, const int32_t* start_seg) {
    constexpr int D = 2;
    const int lane = threadIdx.x & 63;
    TravStack<T, false> stack;
    StageView sv{0, -1};
    if constexpr (sizeof(T) == 4) {
        // LDS: the Dirichlet BVH's first nodes (and its primitives when they
        // fit), then the reflecting BVH's top nodes and their cones
        const int64_t nn4 = (int64_t)a.s.n_stage_nodes * (node_scalars(D) / 4);
        const float4* gn = reinterpret_cast<const float4*>(a.s.nodes);
        for (int64_t i = threadIdx.x; i < nn4; i += blockDim.x) g_stage[i] = gn[i];
        if (a.s.stage_prims) {
            const int64_t np4 = a.s.n_prims * (prim_scalars(D) / 4);
            const float4* gp = reinterpret_cast<const float4*>(a.s.prims);
            for (int64_t i = threadIdx.x; i < np4; i += blockDim.x) g_stage[nn4 + i] = gp[i];
        }
        const int64_t rn4 = (int64_t)ref.n_stage * (node_scalars(D) / 4);
        const float4* rn = reinterpret_cast<const float4*>(ref.nodes);
        for (int64_t i = threadIdx.x; i < rn4; i += blockDim.x) g_stage[ref.stage_off4 + i] = rn[i];
        const float4* rc = reinterpret_cast<const float4*>(ref.cones);
        for (int64_t i = threadIdx.x; i < (2 * kRefCone / 4) * (int64_t)ref.n_stage; i += blockDim.x)
            g_stage[ref.stage_off4 + rn4 + i] = rc[i];
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
    // throughput of the current walk (Robin steps may flip its sign or
    // exceed 1) and, during nested walks, that of the main walk
    T tau = T(1), tau_main = T(1);
    T kappa = T(0), eps = T(1), delta = T(1);
    uint32_t k = 0, m = 0, p = 0, inst_tag = 0;
    int64_t first_row = 0;
    int32_t root = 0, warm = -1, term_leaf = -1, term_code = -1, phase = 0, on = -1;
    T term_b1 = T(0);
    int64_t wsteps = 0;
    // silhouette query in progress (resumable across iterations) and the
    // Dirichlet answer of its step
    SilQuery<T> sq;
    sq.have = false;
    bool spend = false;
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
                    const int64_t pin = local / a.W;
                    m = (uint32_t)(local - pin * a.W);
                    p = (uint32_t)(pin + in.p_counter);
                    root = in.root;
                    kappa = in.kappa; eps = in.eps; delta = in.delta;
                    inst_tag = 0;
                    const int64_t row = in.point_begin + pin;
                    const double* xp = a.X + (size_t)row * D;
                    first_row = row - a.x_base;
#pragma unroll
                    for (int i = 0; i < D; ++i) x[i] = T(xp[i]);
                    on = -1;
                    if (start_seg && start_seg[row] >= 0) {
                        on = ref.leaf_of[start_seg[row]];
                        ref_left_normal<T>(ref, on, nin);
                        keep_on_domain_side<T>(ref, on, nin, x);
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
        if (!spend) {
            // ---- Dirichlet distance ----------------------------------------------
            T d2;
            int32_t leaf;
            // the first query of a point is run once for all its walks: it
            // counts as one executed query, on the point's walk 0
            bool executed = true;
            if (a.first_leaf && phase == 0 && k == 0) {
                leaf = a.first_leaf[first_row];
                d2 = a.first_d2[first_row];
                executed = m == 0;
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
            const T d = sqrt(d2);
            const bool cap = (int)(k + 1) >= a.prm.kmax;
            if (d < eps || cap) {
                if (cap && !(d < eps)) c_trunc++;
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
                if (MODE == 1 && phase == 0) {
                    T n[3] = {T(0), T(0), T(0)};
                    geo_normal<T, D>(V, n);
                    // oriented away from the previous position (inside by at
                    // least eps; held in xoff until now), or the start point
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
                    term_leaf = leaf;
#pragma unroll
                    for (int c = 0; c < D; ++c) xoff[c] = xbar[c] - delta * n[c];
                    c_term++;
                    if (a.prim_dep && !a.prim_dep[orig]) {
                        a.rec_u[wid] = u_main;
                        a.rec_prim[wid] = term_code;
                        a.rec_b[wid] = term_b1;
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
            } else {
                sil_begin<T>(sq, d2);
                spend = true;
                sd2 = d2;
                sleaf = leaf;
            }
        }
        // ---- closest silhouette point (resumable) -----------------------------
        // The wavefront runs rounds of the lanes' silhouette queries until at
        // least a.park of its lanes are not traversing (answered, or at a
        // terminal); the others keep their query state and resume it in the
        // next iteration instead of starting a new step.
        {
#pragma unroll 1
            while (true) {
                const bool trav = spend && sq.have;
                const unsigned long long sm = __ballot(trav);
                const unsigned long long present = __ballot(true);
                if (sm == 0ull || __popcll(present & ~sm) >= a.park) break;
                if (trav) sil_round<T>(ref, x, on, nin, sq, qc, stack, a.s.tail);
            }
        }
        if (spend && sq.have) {
            c_nodes += qc.nodes; c_prims += qc.prims; c_ovf += qc.overflow;
            continue;
        }
        if (spend) {
            spend = false;
            const T d = sqrt(sd2);
            const int32_t leaf = sleaf;
            const bool nested = MODE == 1 && phase > 0;
            // ---- one step on the star-shaped region ---------------------------
            // The star radius is kept above 16 units of rounding of the
            // position: a walk next to a silhouette vertex must still move
            // (a step below the position's resolution would leave it in
            // place).  Rays still stop at the first wall, so the walk stays
            // in the domain; the region may lose star shape only at that
            // scale.  In FP64 the floor is ~1e-15 and never binds in practice.
            const T ulp = sizeof(T) == 4 ? T(1.1920929e-07) : T(2.220446049250313e-16);
            const T rmin = T(16) * ulp * (fabs(x[0]) + fabs(x[1]));
            T R = fmin(d, fmax(sqrt(sq.best), rmin));
            // a Robin coefficient also caps the radius at 1/mu (a variance
            // choice: it bounds the Robin term's mass per step)
            if (ref.mu > T(0)) R = fmin(R, fmax(T(1) / ref.mu, rmin));
            const uint32_t tag = inst_tag | (nested ? (1u | ((uint32_t)(phase - 1) << 8)) : 0u);
            const u4 r = philox10(u4{k, m, p, tag}, key0, key1);
            T dir[2];
            unit_dir<T, D>(r.x, r.y, dir);
            if (on >= 0) {
                const T c = dir[0] * nin[0] + dir[1] * nin[1];
                if (c < T(0)) {
                    dir[0] -= T(2) * c * nin[0];
                    dir[1] -= T(2) * c * nin[1];
                }
            }
            // The march looks a few units of rounding past R: a wall that the
            // rounded end point x + R v could land behind counts as hit.
            T t;
            const T reach = R + T(8) * ulp * (fabs(x[0]) + fabs(x[1]) + R);
            int32_t seg = ray_first<T>(ref, x, dir, reach, on, t, qc, stack);
            if (seg < 0) t = R;
            if (a.prm.has_source) {
                const T rho = sqrt(unif_pos<T>(r.w));
                if (seg < 0 || rho * R < t) {
                    T y[3];
#pragma unroll
                    for (int c = 0; c < D; ++c) y[c] = x[c] + rho * R * dir[c];
                    acc += tau * green_ball_t<D, T>(kappa, rho, R) * source_f<T, D>(a.prm, y);
                }
            }
            // Robin terms of the star-shaped region's integral equation over
            // the reflecting boundary in the ball, -int G (mu u + h): z
            // uniform by length on that part (length Lz); the data term
            // directly, the mu term by continuing at z with probability q;
            // both doubled at a wall point (the equation's u/2 there)
            T zr[2] = {T(0), T(0)}, Lz = T(0), Gz = T(0);
            int32_t zleaf = -1;
            const T cx = on >= 0 ? T(2) : T(1);
            if (ref.robin) {
                zleaf = ref_boundary_sample<T>(ref, x, R, u4{k, m, p, tag}, key0, key1, Lz, zr, qc, stack);
                if (zleaf >= 0) {
                    const T rz = fmax(sqrt((zr[0] - x[0]) * (zr[0] - x[0]) + (zr[1] - x[1]) * (zr[1] - x[1])), rmin);
                    // G(r; R) = (G |B_R|) / |B_R|
                    Gz = green_ball_t<D, T>(kappa, fmin(rz / R, T(1)), R) / (T(3.14159265358979323846) * R * R);
                    acc -= tau * cx * Lz * Gz * robin_data<T>(ref, zr);
                }
            }
            const T q = (ref.mu > T(0) && zleaf >= 0) ? fmin(T(0.5), cx * ref.mu * Lz * Gz) : T(0);
            const bool to_z = q > T(0) && unif<T>(r.y) < q;
            const T wgt = to_z ? -cx * ref.mu * Lz * Gz / q
                               : (seg >= 0 ? reflect_weight<D, T>(kappa, t, R) : poisson_scale<T, D>(kappa, R)) /
                                     (T(1) - q);
            // roulette keeps the walk with probability min(1, |wgt|), and the
            // throughput carries the rest of the weight
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
                    x[0] = zr[0];
                    x[1] = zr[1];
                    on = zleaf;
                } else {
#pragma unroll
                    for (int c = 0; c < D; ++c) x[c] += t * dir[c];
                    on = seg;
                }
                if (on >= 0) {   // the domain is on the wall's left
                    ref_left_normal<T>(ref, on, nin);
                    keep_on_domain_side<T>(ref, on, nin, x);
                }
                ++k;
                warm = leaf;
            }
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
                a.rec_b[wid] = term_b1;
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
// checks of the two reflecting-boundary queries).  out per row:
// {silhouette distance capped at cap[row], ray t (cap[row] if none), ray
// hit as an original segment index or -1}.  on: original segment or -1;
// a row with any other value gets NaN outputs.
template <class T>
__global__ void ref_query_kernel(RefScene<T> ref, const double* X, const double* dir, const double* cap,
                                 const int32_t* on_orig, const double* nin, int64_t n, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T x[2] = {T(X[2 * i]), T(X[2 * i + 1])};
    T dv[2] = {T(dir[2 * i]), T(dir[2 * i + 1])};
    T nn[2] = {T(nin[2 * i]), T(nin[2 * i + 1])};
    const int32_t oo = on_orig[i];
    if (oo < -1 || oo >= ref.n) {
        out[3 * i] = out[3 * i + 1] = out[3 * i + 2] = NAN;
        return;
    }
    const int32_t on = oo >= 0 ? ref.leaf_of[oo] : -1;
    QueryCount qc{0, 0, 0};
    TravStack<T, false> st;
    const T c = T(cap[i]);
    out[3 * i] = double(sqrt(silhouette_d2<T>(ref, x, on, nn, c * c, qc, st)));
    T t;
    const int32_t hit = ray_first<T>(ref, x, dv, c, on, t, qc, st);
    out[3 * i + 1] = double(t);
    out[3 * i + 2] = hit >= 0 ? double(ref.info[hit].w) : -1.0;
}

template <class T, int D>
__global__ void reflect_weight_eval(const double* r, const double* R, int64_t n, T kappa, double* w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    w[i] = double(reflect_weight<D, T>(kappa, T(r[i]), T(R[i])));
}

}  // namespace dwos
