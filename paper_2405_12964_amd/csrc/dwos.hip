// C ABI of the differential walk-on-spheres library (declared in include/dwos.h).
//
// A context owns one boundary (or a batch of instance boundaries), its BVH in
// the working precision, the problem constants, the parameter Jacobian and
// grow-only workspaces.  Every entry point validates its arguments on the
// host, enqueues kernels on the context stream and returns a status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dwos.h"
#include "aux_kernels.hpp"
#include "cv_kernels.hpp"
#include "host_common.hpp"
#include "mlp.hpp"
#include "bvh.hpp"
#include "wost_kernels.hpp"
#include "wost3_kernels.hpp"
#include "implicit_kernels.hpp"
#include "adjoint_kernels.hpp"

#include <map>
#include <mutex>
#include <tuple>

namespace {

using dwos_host::fail;
using dwos_host::DevBuf;
using dwos_host::upload;
using dwos_host::blocks_for;

constexpr int64_t kMaxWalksPerChunk = int64_t(1) << 26;

// Workspace of the allocation-free solve (dwos_solve_noalloc): one fixed
// array per device, held from module load to process exit.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol); it uses the device address resolved per device by
// resolve_scratch() when a context is created.
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` on device `dev` (which must be current),
// resolved once per device.
dwos_status resolve_scratch(int dev) {
    if (dev < 0 || dev >= kScratchMaxDevices) return fail(DWOS_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return DWOS_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(DWOS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
    return DWOS_OK;
}

void* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kScratchMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[dev];
}

struct InstanceHost {
    int32_t root;            // root pair node in the combined node array
    int64_t nv_off, np_off;  // first vertex / primitive of the instance
    double sigma, eps, delta;
};

}  // namespace

struct dwos_ctx {
    int D = 0;
    int prec = DWOS_FP32;
    hipStream_t stream = nullptr;
    int device = 0;
    int cu_count = 0;
    size_t max_smem = 0;      // LDS bytes a block may use
    // geometry
    bool has_boundary = false;
    int64_t nv = 0, np = 0, n_nodes = 0;
    DevBuf nodes, prims, orig, verts, pverts, label, gvert, leaf_of;
    DevBuf node_ranges;   // leaf-order primitive range of each node's two children
    // batch contexts: instances accumulated on the host, uploaded together
    std::vector<InstanceHost> instances;
    std::vector<double> hostV, hostG;
    std::vector<int32_t> hostP, hostL;
    std::vector<dwos::HostNode> hostNodes;
    std::vector<int32_t> hostOrder;
    bool batch_dirty = false;
    std::vector<unsigned char> inst_host;     // last uploaded instance table
    // per-instance parameter Jacobians (instance-local vertices), combined
    // into one Jacobian of the batch's vertex array before a batch gradient
    struct BatchParams { int64_t N = 0; std::vector<int64_t> rowptr; std::vector<int32_t> pid; std::vector<double> vel; };
    std::vector<BatchParams> batch_params;
    bool batch_params_dirty = false;
    // problem
    bool has_problem = false;
    dwos_problem prob{};
    // parameters
    bool has_params = false;
    int64_t N = 0;
    DevBuf rowptr, pid, vel, bc_pid, colptr, cvert, cvel, bcptr, bcvert;
    bool has_bc_params = false;
    // workspaces
    DevBuf rec_u, rec_prim, rec_b, rec_uoff, rec_steps, accA, accB, queue, counters, instbuf, export_u;
    DevBuf vtmp;   // V(pi) for dwos_apply_parameters
    DevBuf first_leaf, first_d2;   // shared first query of each start point
    // first_leaf holds primitives of this context's own (single-instance)
    // scene, so the next first queries may start from them
    bool first_warm = false;
    DevBuf inst_prange;   // batch: per instance its leaf positions [begin, end)
    DevBuf order_cell, order_perm, order_hist;   // spatial scheduling order of a chunk's points
    const uint64_t* seed_dev = nullptr;   // optional device seed offset
    int variant = 0;                      // walk-kernel launch shape (FP32; 3D contexts start at 1)
    // scheduling knobs of the walk kernels (dwos_set_tuning, dwos_autotune)
    int park = dwos::kParkLanes;
    int tail = dwos::kDescendTail;
    int chunk = (int)dwos::kQueueChunk;
    int stage_cap = -1;                   // cap on LDS-staged nodes (-1: all that fit)
    // timing and cumulative counters per walk kind (0 forward, 1 differential)
    struct Pending { hipEvent_t e0, e1; int kind; };
    std::vector<Pending> pending;
    double timed_ms[3] = {0.0, 0.0, 0.0};
    int64_t timed_launches[3] = {0, 0, 0};
    DevBuf totals;   // 3 x Counters (kind 2: adjoint walks)
    // learned control variate of the nested walks (not owned)
    dwos_mlp* cv = nullptr;
    uint32_t cv_qthresh = 1u << 24;
    DevBuf cv_run, cv_xoff, cv_xbar, cv_g, cv_stop, cv_y, cv_rho, cv_d, cv_S, cv_alive;
    DevBuf cv_Noff, cv_Nstop, cv_Ny, cv_Ly, cv_target, cv_uplain;
    DevBuf cv_bx, cv_bN, cv_bL, cv_bNbar, cv_bLbar, cv_bs, cv_bvalid;   // training batch
    DevBuf cv_beta, cv_stats;     // control-variate coefficient; sums for the next one
    DevBuf vparam;                // per vertex: 1 if it moves or carries a parameter value
    DevBuf prim_dep;              // per primitive: 1 if a vertex of it does
    bool cv_fresh = true;         // beta must be reset to 1 before the next use
    int64_t cv_nrec = 0;          // walks recorded by the last differential chunk
    // reflecting (zero-flux) boundary, 2D: walks on stars when present
    bool has_ref = false;
    int64_t ref_n = 0, ref_nn = 0;   // reflecting segments, pair nodes
    DevBuf ref_nodes, ref_geo, ref_info, ref_leaf_of, ref_cones;
    DevBuf start_seg;             // per query point: reflecting segment or -1
    int64_t start_n = 0;          // points covered by start_seg (0: none)
    // Robin condition on the reflecting boundary (mu, data h as c, b, A)
    // 3D reflecting mesh: ref_nodes / ref_geo / ref_leaf_of hold its triangle
    // BVH, ref_torig the leaf -> original triangle map; its edges have a BVH
    // of their own
    DevBuf ref_torig, ref_enodes, ref_egeo, ref_einfo, ref_econes;
    int64_t ref_ne = 0, ref_enn = 0;
    bool robin = false;
    double robin_mu = 0.0;
    double robin_hq[13] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};   // c, b[3], A[9] (row major)
    DevBuf rec_w;                 // per differential walk: throughput at the terminal
    // implicit boundary (2D): zero set of c + sum_n a_n / |x - p_n|
    bool has_imp = false;
    int64_t imp_n = 0;
    double imp_c = 0.0;
    DevBuf imp_mono;              // n x 3 in the working precision
    DevBuf imp_xbar, imp_s, imp_coef;   // per-walk terminal data and reverse-mode weights
    DevBuf imp_bx, imp_bs;              // band points and their 1/|grad h|
    // adjoint formulation: per-walk weights of udot and of V_n
    DevBuf adj_w, adj_e;
};

namespace {

template <class T>
dwos::Params<T> make_params(const dwos_problem& p) {
    dwos::Params<T> q{};
    q.K = p.K;
    q.kmax = p.kmax;
    q.rr = p.rr;
    q.n_gauss = p.n_gauss;
    q.n_labels = p.n_labels;
    q.src_c0 = T(p.src_c0);
    q.has_source = (p.src_c0 != 0.0 || p.n_gauss > 0) ? 1 : 0;
    for (int i = 0; i < dwos::kMaxGauss; ++i)
        for (int k = 0; k < 5; ++k) q.gauss[i][k] = T(p.gauss[i][k]);
    for (int l = 0; l < dwos::kMaxLabels; ++l) {
        q.kind[l] = p.bc[l].kind;
        q.gc[l] = T(p.bc[l].c);
        for (int i = 0; i < 3; ++i) q.gb[l][i] = T(p.bc[l].b[i]);
        for (int i = 0; i < 9; ++i) q.gA[l][i] = T(p.bc[l].A[i]);
    }
    return q;
}

template <class T>
dwos::Scene<T> make_scene(dwos_ctx* c) {
    dwos::Scene<T> s;
    s.nodes = c->nodes.as<T>();
    s.prims = c->prims.as<T>();
    s.orig = c->orig.as<int32_t>();
    s.verts = c->verts.as<T>();
    s.pverts = c->pverts.as<int32_t>();
    s.label = c->label.as<int32_t>();
    s.gvert = c->gvert.as<T>();
    s.n_prims = c->np;
    // LDS staging plan: the whole BVH and all primitives if they fit, else a
    // prefix of the (breadth-first ordered) nodes
    const size_t budget = c->max_smem >= 1024 ? c->max_smem - 512 : 0;
    const size_t nb = (size_t)dwos::node_scalars(c->D) * sizeof(T);
    const size_t pb = (size_t)dwos::prim_scalars(c->D) * sizeof(T);
    const size_t all_nodes = (size_t)c->n_nodes * nb, all_prims = (size_t)c->np * pb;
    if (!c->instances.empty()) {
        // batches: every instance has its own tree, so no common prefix
        s.n_stage_nodes = 0;
        s.stage_prims = 0;
    } else if (all_nodes + all_prims <= budget) {
        s.n_stage_nodes = (int32_t)c->n_nodes;
        s.stage_prims = 1;
    } else {
        s.n_stage_nodes = (int32_t)std::min<size_t>((size_t)c->n_nodes, budget / nb);
        s.stage_prims = 0;
    }
    // a tuning cap shortens the staged node prefix (primitives, if staged,
    // follow the prefix in LDS)
    if (c->stage_cap >= 0 && s.n_stage_nodes > c->stage_cap) s.n_stage_nodes = c->stage_cap;
    s.tail = c->tail;
    return s;
}

template <class T>
size_t stage_bytes(const dwos::Scene<T>& s, int D) {
    return (size_t)s.n_stage_nodes * dwos::node_scalars(D) * sizeof(T) +
           (s.stage_prims ? (size_t)s.n_prims * dwos::prim_scalars(D) * sizeof(T) : 0);
}

dwos::ParamCSR make_csr(dwos_ctx* c) {
    dwos::ParamCSR J{};
    J.rowptr = c->rowptr.as<int64_t>();
    J.pid = c->pid.as<int32_t>();
    J.vel = c->vel.as<double>();
    J.bc_pid = c->has_bc_params ? c->bc_pid.as<int32_t>() : nullptr;
    J.colptr = c->colptr.as<int64_t>();
    J.cvert = c->cvert.as<int32_t>();
    J.cvel = c->cvel.as<double>();
    J.bcptr = c->has_bc_params ? c->bcptr.as<int64_t>() : nullptr;
    J.bcvert = c->has_bc_params ? c->bcvert.as<int32_t>() : nullptr;
    J.N = c->N;
    return J;
}


// Pair nodes of a built BVH in the device layout of bvh.hpp (working precision T).
template <class T>
std::vector<T> pack_nodes(int D, const std::vector<dwos::HostNode>& hn) {
    const int NS = dwos::node_scalars(D);
    std::vector<T> nodes((size_t)hn.size() * NS, T(0));
    for (size_t i = 0; i < hn.size(); ++i) {
        T* p = &nodes[i * NS];
        for (int k = 0; k < D; ++k) {
            p[k] = T(hn[i].lo[0][k]); p[D + k] = T(hn[i].hi[0][k]);
            p[2 * D + k] = T(hn[i].lo[1][k]); p[3 * D + k] = T(hn[i].hi[1][k]);
        }
        for (int c = 0; c < 2; ++c) {
            T* sl = p + dwos::slab_offset(D) + c * (D + 2);
            double scale = std::fabs(hn[i].o[c]);
            for (int k = 0; k < D; ++k) {
                sl[k] = T(hn[i].n[c][k]);
                scale += std::max(std::fabs(hn[i].lo[c][k]), std::fabs(hn[i].hi[c][k]));
            }
            sl[D] = T(hn[i].o[c]);
            sl[D + 1] = hn[i].t[c] < 0 ? T(hn[i].t[c]) : T(hn[i].t[c]) + dwos::slab_pad_host<T>(T(scale));
        }
        int32_t* r = reinterpret_cast<int32_t*>(p + dwos::ref_offset(D));
        r[0] = hn[i].child[0];
        r[1] = hn[i].child[1];
    }
    return nodes;
}

// Reflecting segments: BVH nodes, per-segment geometry and adjacency in
// leaf order (the layout of wost_kernels.hpp's RefScene).  inc[v]: the
// segments at vertex v.
template <class T>
dwos_status upload_reflecting(dwos_ctx* c, const double* V, const int32_t* segs, int64_t ns,
                              const std::vector<std::vector<int32_t>>& inc, const dwos::HostBVH& bvh) {
    std::vector<T> nodes = pack_nodes<T>(2, bvh.nodes);
    std::vector<int32_t> leaf_of(ns);
    for (int64_t i = 0; i < ns; ++i) leaf_of[bvh.order[i]] = (int32_t)i;
    std::vector<T> geo((size_t)ns * dwos::kRefGeo, T(0));
    std::vector<int32_t> info((size_t)ns * 4, -1);
    for (int64_t lp = 0; lp < ns; ++lp) {
        const int32_t o = bvh.order[lp];
        T* g = &geo[(size_t)lp * dwos::kRefGeo];
        int32_t* f = &info[(size_t)lp * 4];
        f[0] = 0;
        f[3] = o;
        for (int e = 0; e < 2; ++e) {
            const int32_t v = segs[2 * o + e];
            for (int k = 0; k < 2; ++k) g[2 * e + k] = T(V[2 * (size_t)v + k]);
            const std::vector<int32_t>& at = inc[v];
            if (at[0] == o) f[0] |= 1 << e;                 // lowest segment at v tests it
            if (at.size() != 2) { f[0] |= 4 << e; continue; }
            const int32_t j = at[0] == o ? at[1] : at[0];  // the other segment at v
            const int32_t far = segs[2 * j] == v ? segs[2 * j + 1] : segs[2 * j];
            for (int k = 0; k < 2; ++k) g[4 + 2 * e + k] = T(V[2 * (size_t)far + k]);
            f[1 + e] = leaf_of[j];
        }
    }
    // normal cones of every node's two children (layout in wost_kernels.hpp)
    const double margin = sizeof(T) == 4 ? 2e-3 : 1e-8;
    std::vector<T> cones(bvh.nodes.size() * 2 * dwos::kRefCone);
    for (size_t ni = 0; ni < bvh.nodes.size(); ++ni)
        for (int ch = 0; ch < 2; ++ch) {
            T* q = &cones[(ni * 2 + ch) * dwos::kRefCone];
            q[0] = T(0); q[1] = T(0); q[2] = T(2); q[3] = T(-1);   // never pruned
            q[4] = T(0); q[5] = T(0); q[6] = T(0); q[7] = T(0);
            const int32_t b0 = bvh.nodes[ni].range[ch][0], b1 = bvh.nodes[ni].range[ch][1];
            std::vector<double> nrm;
            bool forced = b1 <= b0;
            auto add = [&](double tx, double ty) {
                const double L = std::sqrt(tx * tx + ty * ty);
                nrm.push_back(ty / L);
                nrm.push_back(-tx / L);
            };
            for (int32_t lp = b0; lp < b1 && !forced; ++lp) {
                const T* g = &geo[(size_t)lp * dwos::kRefGeo];
                const int32_t f = info[(size_t)lp * 4];
                const int32_t o = bvh.order[lp];
                const double* a = V + 2 * (size_t)segs[2 * o];
                const double* b = V + 2 * (size_t)segs[2 * o + 1];
                add(b[0] - a[0], b[1] - a[1]);
                if ((f & 1) && (f & 4)) forced = true;
                if ((f & 2) && (f & 8)) forced = true;
                if (forced) break;
                // the other segment at a tested vertex, along the polyline through it
                if (f & 1) add(a[0] - double(g[4]), a[1] - double(g[5]));
                if (f & 2) add(double(g[6]) - b[0], double(g[7]) - b[1]);
            }
            if (forced || nrm.empty()) continue;
            double ax = 0, ay = 0;
            for (size_t k = 0; k < nrm.size(); k += 2) { ax += nrm[k]; ay += nrm[k + 1]; }
            const double L = std::sqrt(ax * ax + ay * ay);
            if (!(L > 1e-9 * (double)nrm.size())) continue;
            ax /= L; ay /= L;
            double th = 0;
            for (size_t k = 0; k < nrm.size(); k += 2)
                th = std::max(th, std::acos(std::min(1.0, std::max(-1.0, ax * nrm[k] + ay * nrm[k + 1]))));
            const double s0 = th + margin;
            if (!(s0 < 1.5707963267948966)) continue;
            // range of a.p over the child's segment endpoints, and kappa
            double omin = HUGE_VAL, omax = -HUGE_VAL;
            for (int32_t lp = b0; lp < b1; ++lp) {
                const int32_t o = bvh.order[lp];
                for (int e = 0; e < 2; ++e) {
                    const double* pv = V + 2 * (size_t)segs[2 * o + e];
                    const double ov = ax * pv[0] + ay * pv[1];
                    omin = std::min(omin, ov);
                    omax = std::max(omax, ov);
                }
            }
            const double tol = sizeof(T) == 4 ? 1e-4 : 1e-10;
            q[0] = T(ax); q[1] = T(ay); q[2] = T(std::sin(s0)); q[3] = T(std::cos(s0));
            q[4] = T(omin); q[5] = T(omax); q[6] = T(4.0 * tol); q[7] = T(0);
        }
    hipStream_t s = c->stream;
    HIP_OK(upload(c->ref_cones, cones.data(), cones.size(), s));
    HIP_OK(upload(c->ref_nodes, nodes.data(), nodes.size(), s));
    HIP_OK(upload(c->ref_geo, geo.data(), geo.size(), s));
    HIP_OK(upload(c->ref_info, info.data(), info.size(), s));
    HIP_OK(upload(c->ref_leaf_of, leaf_of.data(), leaf_of.size(), s));
    c->ref_n = ns;
    c->ref_nn = (int64_t)bvh.nodes.size();
    return DWOS_OK;
}

template <class T>
dwos::RefScene<T> make_ref(dwos_ctx* c) {
    dwos::RefScene<T> r{};
    r.nodes = c->ref_nodes.as<T>();
    r.geo = c->ref_geo.as<T>();
    r.info = c->ref_info.as<int4>();
    r.leaf_of = c->ref_leaf_of.as<int32_t>();
    r.cones = c->ref_cones.as<T>();
    r.n = c->ref_n;
    r.robin = c->robin ? 1 : 0;
    r.mu = T(c->robin_mu);
    // 2D: c, b0, b1, A00, A01, A10, A11
    const int pick[7] = {0, 1, 2, 4, 5, 7, 8};
    for (int i = 0; i < 7; ++i) r.hq[i] = T(c->robin_hq[pick[i]]);
    return r;
}

// Reflecting triangles (3D): the triangle BVH with each leaf's vertices,
// and the edge BVH with each edge's vertices, the third vertices of its
// (first two) triangles and their leaf positions (layout of
// wost3_kernels.hpp's RefScene3).
template <class T>
dwos_status upload_reflecting3(dwos_ctx* c, const double* V, const int32_t* tris, int64_t nt,
                               const dwos::HostBVH& tb) {
    std::vector<T> tnodes = pack_nodes<T>(3, tb.nodes);
    std::vector<int32_t> leaf_of(nt), torig(nt);
    for (int64_t i = 0; i < nt; ++i) {
        leaf_of[tb.order[i]] = (int32_t)i;
        torig[i] = tb.order[i];
    }
    std::vector<T> tgeo((size_t)nt * dwos::kTriGeo, T(0));
    for (int64_t lp = 0; lp < nt; ++lp) {
        const int32_t o = tb.order[lp];
        for (int k = 0; k < 3; ++k)
            for (int cc = 0; cc < 3; ++cc) tgeo[(size_t)lp * dwos::kTriGeo + 3 * k + cc] = T(V[3 * (size_t)tris[3 * o + k] + cc]);
    }
    // edges: sorted (low vertex, high vertex, triangle) triples, grouped
    struct E { int32_t a, b, f; };
    std::vector<E> es;
    es.reserve(3 * (size_t)nt);
    for (int64_t i = 0; i < nt; ++i)
        for (int k = 0; k < 3; ++k) {
            const int32_t u = tris[3 * i + k], v = tris[3 * i + (k + 1) % 3];
            es.push_back({std::min(u, v), std::max(u, v), (int32_t)i});
        }
    std::sort(es.begin(), es.end(), [](const E& x, const E& y) {
        return x.a != y.a ? x.a < y.a : (x.b != y.b ? x.b < y.b : x.f < y.f);
    });
    struct Edge { int32_t a, b, f0, f1, nf; };
    std::vector<Edge> edges;
    for (size_t j = 0; j < es.size(); ++j) {
        if (j == 0 || es[j].a != es[j - 1].a || es[j].b != es[j - 1].b) edges.push_back({es[j].a, es[j].b, es[j].f, -1, 0});
        Edge& e = edges.back();
        if (e.nf == 1) e.f1 = es[j].f;
        e.nf++;
    }
    // does triangle f traverse the edge a -> b (in its winding order)?
    auto forward = [&](int32_t f, int32_t a, int32_t b) {
        for (int k = 0; k < 3; ++k)
            if (tris[3 * (size_t)f + k] == a && tris[3 * (size_t)f + (k + 1) % 3] == b) return true;
        return false;
    };
    auto unit_normal = [&](int32_t f, double* n) {
        const double* A = V + 3 * (size_t)tris[3 * (size_t)f];
        const double* B = V + 3 * (size_t)tris[3 * (size_t)f + 1];
        const double* Cc = V + 3 * (size_t)tris[3 * (size_t)f + 2];
        const double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        const double e2[3] = {Cc[0] - A[0], Cc[1] - A[1], Cc[2] - A[2]};
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double L = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int k = 0; k < 3; ++k) n[k] /= L;
    };
    const int64_t ne = (int64_t)edges.size();
    if (ne > (int64_t(1) << 27)) return fail(DWOS_EINVAL, "set_reflecting: too many edges");
    std::vector<int32_t> eprims(3 * (size_t)ne);
    for (int64_t i = 0; i < ne; ++i) {
        eprims[3 * i] = edges[i].a;
        eprims[3 * i + 1] = edges[i].b;
        eprims[3 * i + 2] = edges[i].b;
    }
    dwos::HostBVH eb = dwos::build_bvh(V, eprims.data(), ne, 3);
    if (eb.max_depth >= dwos::kMaxDepth) return fail(DWOS_EINVAL, "set_reflecting: edge BVH too deep");
    dwos::reorder_bfs(eb);
    std::vector<T> enodes = pack_nodes<T>(3, eb.nodes);
    std::vector<T> egeo((size_t)ne * dwos::kEdgeGeo, T(0));
    std::vector<int32_t> einfo((size_t)ne * 4, -1);
    auto third = [&](int32_t f, int32_t a, int32_t b) {
        for (int k = 0; k < 3; ++k) {
            const int32_t v = tris[3 * (size_t)f + k];
            if (v != a && v != b) return v;
        }
        return tris[3 * (size_t)f];
    };
    for (int64_t lp = 0; lp < ne; ++lp) {
        const Edge& e = edges[eb.order[lp]];
        T* g = &egeo[(size_t)lp * dwos::kEdgeGeo];
        const int32_t w0 = third(e.f0, e.a, e.b), w1 = e.nf >= 2 ? third(e.f1, e.a, e.b) : w0;
        const int32_t vs[4] = {e.a, e.b, w0, w1};
        for (int k = 0; k < 4; ++k)
            for (int cc = 0; cc < 3; ++cc) g[3 * k + cc] = T(V[3 * (size_t)vs[k] + cc]);
        int32_t* f = &einfo[(size_t)lp * 4];
        f[0] = e.nf != 2 ? 1 : 0;
        f[1] = leaf_of[e.f0];
        f[2] = e.nf >= 2 ? leaf_of[e.f1] : -1;
        f[3] = eb.order[lp];
    }
    // normal cones of every edge node's two children (layout in wost3_kernels.hpp)
    const double margin = sizeof(T) == 4 ? 2e-3 : 1e-8;
    std::vector<T> cones(eb.nodes.size() * 2 * dwos::kEdgeCone, T(0));
    std::vector<double> nrm;
    for (size_t ni = 0; ni < eb.nodes.size(); ++ni)
        for (int ch = 0; ch < 2; ++ch) {
            T* q = &cones[(ni * 2 + ch) * dwos::kEdgeCone];
            q[3] = T(2); q[4] = T(-1);   // never pruned
            const int32_t b0 = eb.nodes[ni].range[ch][0], b1 = eb.nodes[ni].range[ch][1];
            if (b1 <= b0) continue;
            nrm.clear();
            bool forced = false;
            double min_sin = 1.0;   // sin of the smallest angle at an edge's first vertex
            for (int32_t lp = b0; lp < b1 && !forced; ++lp) {
                const Edge& e = edges[eb.order[lp]];
                // a rim or non-manifold edge, or two triangles wound the same
                // way along it, is never pruned
                if (e.nf != 2 || forward(e.f0, e.a, e.b) == forward(e.f1, e.a, e.b)) { forced = true; break; }
                double n[3];
                unit_normal(e.f0, n);
                nrm.insert(nrm.end(), n, n + 3);
                unit_normal(e.f1, n);
                nrm.insert(nrm.end(), n, n + 3);
                const double* pa = V + 3 * (size_t)e.a;
                const double* pb = V + 3 * (size_t)e.b;
                const double t[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
                for (int32_t f : {e.f0, e.f1}) {
                    const double* pw = V + 3 * (size_t)third(f, e.a, e.b);
                    const double d[3] = {pw[0] - pa[0], pw[1] - pa[1], pw[2] - pa[2]};
                    const double cr[3] = {t[1] * d[2] - t[2] * d[1], t[2] * d[0] - t[0] * d[2], t[0] * d[1] - t[1] * d[0]};
                    const double tt = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
                    const double dd = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                    const double sn = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]) / (tt * dd);
                    min_sin = std::min(min_sin, std::isfinite(sn) ? sn : 0.0);
                }
            }
            if (forced || nrm.empty()) continue;
            double ax = 0, ay = 0, az = 0;
            for (size_t k = 0; k < nrm.size(); k += 3) { ax += nrm[k]; ay += nrm[k + 1]; az += nrm[k + 2]; }
            const double L = std::sqrt(ax * ax + ay * ay + az * az);
            if (!(L > 1e-9 * (double)nrm.size())) continue;
            ax /= L; ay /= L; az /= L;
            double th = 0;
            for (size_t k = 0; k < nrm.size(); k += 3)
                th = std::max(th, std::acos(std::min(1.0, std::max(-1.0, ax * nrm[k] + ay * nrm[k + 1] + az * nrm[k + 2]))));
            const double s0 = th + margin;
            if (!(s0 < 1.5707963267948966)) continue;
            // range of a.p over the child's edge vertices, and kappa (an edge
            // of zero angle leaves the plane test unable to prune: kappa inf)
            double omin = HUGE_VAL, omax = -HUGE_VAL;
            for (int32_t lp = b0; lp < b1; ++lp) {
                const Edge& e = edges[eb.order[lp]];
                for (int32_t v : {e.a, e.b}) {
                    const double* pv = V + 3 * (size_t)v;
                    const double o = ax * pv[0] + ay * pv[1] + az * pv[2];
                    omin = std::min(omin, o);
                    omax = std::max(omax, o);
                }
            }
            const double tol = sizeof(T) == 4 ? 1e-4 : 1e-10;
            const double kappa = min_sin > 0.0 ? 4.0 * tol / min_sin : HUGE_VAL;
            q[0] = T(ax); q[1] = T(ay); q[2] = T(az); q[3] = T(std::sin(s0)); q[4] = T(std::cos(s0));
            q[5] = T(omin); q[6] = T(omax); q[7] = T(kappa);
        }
    hipStream_t s = c->stream;
    HIP_OK(upload(c->ref_econes, cones.data(), cones.size(), s));
    HIP_OK(upload(c->ref_nodes, tnodes.data(), tnodes.size(), s));
    HIP_OK(upload(c->ref_geo, tgeo.data(), tgeo.size(), s));
    HIP_OK(upload(c->ref_leaf_of, leaf_of.data(), leaf_of.size(), s));
    HIP_OK(upload(c->ref_torig, torig.data(), torig.size(), s));
    HIP_OK(upload(c->ref_enodes, enodes.data(), enodes.size(), s));
    HIP_OK(upload(c->ref_egeo, egeo.data(), egeo.size(), s));
    HIP_OK(upload(c->ref_einfo, einfo.data(), einfo.size(), s));
    c->ref_n = nt;
    c->ref_nn = (int64_t)tb.nodes.size();
    c->ref_ne = ne;
    c->ref_enn = (int64_t)eb.nodes.size();
    return DWOS_OK;
}

template <class T>
dwos::RefScene3<T> make_ref3(dwos_ctx* c) {
    dwos::RefScene3<T> r{};
    r.tnodes = c->ref_nodes.as<T>();
    r.tgeo = c->ref_geo.as<T>();
    r.torig = c->ref_torig.as<int32_t>();
    r.tleaf_of = c->ref_leaf_of.as<int32_t>();
    r.nt = c->ref_n;
    r.enodes = c->ref_enodes.as<T>();
    r.egeo = c->ref_egeo.as<T>();
    r.einfo = c->ref_einfo.as<int4>();
    r.econes = c->ref_econes.as<T>();
    r.ne = c->ref_ne;
    r.robin = c->robin ? 1 : 0;
    r.mu = T(c->robin_mu);
    for (int i = 0; i < 13; ++i) r.hq[i] = T(c->robin_hq[i]);
    return r;
}

// Upload a built BVH + geometry in the working precision T.
template <class T>
dwos_status upload_geometry(dwos_ctx* c, const std::vector<double>& V, const std::vector<int32_t>& prims,
                            const std::vector<int32_t>& label, const std::vector<double>& gvert,
                            const std::vector<dwos::HostNode>& hn, const std::vector<int32_t>& order) {
    const int D = c->D;
    const int PS = dwos::prim_scalars(D);
    const int64_t np = (int64_t)prims.size() / D, nv = (int64_t)V.size() / D;
    std::vector<T> nodes = pack_nodes<T>(D, hn);
    std::vector<int32_t> ranges((size_t)hn.size() * 4);
    for (size_t i = 0; i < hn.size(); ++i)
        for (int c = 0; c < 2; ++c) {
            ranges[i * 4 + 2 * c] = hn[i].range[c][0];
            ranges[i * 4 + 2 * c + 1] = hn[i].range[c][1];
        }
    std::vector<T> pr((size_t)np * PS, T(0));
    for (int64_t lp = 0; lp < np; ++lp) {
        const int32_t o = order[lp];
        for (int k = 0; k < D; ++k)
            for (int cc = 0; cc < D; ++cc) pr[lp * PS + k * D + cc] = T(V[(size_t)prims[(size_t)o * D + k] * D + cc]);
    }
    std::vector<int32_t> origv(order.begin(), order.end());
    std::vector<int32_t> leaf_of(np);
    for (int64_t i = 0; i < np; ++i) leaf_of[order[i]] = (int32_t)i;
    std::vector<T> vt(V.size());
    for (size_t i = 0; i < V.size(); ++i) vt[i] = T(V[i]);
    std::vector<T> gv(gvert.size());
    for (size_t i = 0; i < gvert.size(); ++i) gv[i] = T(gvert[i]);
    hipStream_t s = c->stream;
    c->first_warm = false;
    HIP_OK(upload(c->nodes, nodes.data(), nodes.size(), s));
    HIP_OK(upload(c->node_ranges, ranges.data(), ranges.size(), s));
    HIP_OK(upload(c->prims, pr.data(), pr.size(), s));
    HIP_OK(upload(c->orig, origv.data(), origv.size(), s));
    HIP_OK(upload(c->leaf_of, leaf_of.data(), leaf_of.size(), s));
    HIP_OK(upload(c->verts, vt.data(), vt.size(), s));
    HIP_OK(upload(c->pverts, prims.data(), prims.size(), s));
    HIP_OK(upload(c->label, label.data(), label.size(), s));
    HIP_OK(upload(c->gvert, gv.data(), gv.size(), s));
    c->nv = nv;
    c->np = np;
    c->n_nodes = (int64_t)hn.size();
    return DWOS_OK;
}

dwos_status check_geometry(int D, const double* V, int64_t nv, const int32_t* prims, int64_t np,
                           const int32_t* label, int n_labels_limit) {
    if (!V || !prims || nv <= 0 || np <= 0) return fail(DWOS_EINVAL, "set_boundary: empty or NULL geometry");
    if (nv > INT32_MAX || np > (int64_t(1) << 27)) return fail(DWOS_EINVAL, "set_boundary: too many vertices/primitives");
    for (int64_t i = 0; i < nv * D; ++i)
        if (!std::isfinite(V[i])) return fail(DWOS_EINVAL, "set_boundary: non-finite vertex coordinate");
    for (int64_t p = 0; p < np; ++p) {
        for (int k = 0; k < D; ++k) {
            const int32_t v = prims[p * D + k];
            if (v < 0 || v >= nv) return fail(DWOS_EINVAL, "set_boundary: vertex index out of range");
        }
        double e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
        const double* a = V + (size_t)prims[p * D] * D;
        const double* b = V + (size_t)prims[p * D + 1] * D;
        for (int c = 0; c < D; ++c) e1[c] = b[c] - a[c];
        double area2;
        if (D == 2) {
            area2 = e1[0] * e1[0] + e1[1] * e1[1];
        } else {
            const double* cc = V + (size_t)prims[p * D + 2] * D;
            for (int c = 0; c < 3; ++c) e2[c] = cc[c] - a[c];
            const double x = e1[1] * e2[2] - e1[2] * e2[1], y = e1[2] * e2[0] - e1[0] * e2[2],
                         z = e1[0] * e2[1] - e1[1] * e2[0];
            area2 = x * x + y * y + z * z;
        }
        if (!(area2 > 0)) return fail(DWOS_EINVAL, "set_boundary: degenerate primitive " + std::to_string(p));
        if (label && (label[p] < 0 || label[p] >= n_labels_limit))
            return fail(DWOS_EINVAL, "set_boundary: label out of range");
    }
    return DWOS_OK;
}

dwos_status drain_events(dwos_ctx* c, double* call_ms, size_t from) {
    double ms_call = 0.0;
    for (size_t i = 0; i < c->pending.size(); ++i) {
        auto& pr = c->pending[i];
        HIP_OK(hipEventSynchronize(pr.e1));
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, pr.e0, pr.e1));
        c->timed_ms[pr.kind] += ms;
        c->timed_launches[pr.kind] += 1;
        if (i >= from) ms_call += ms;
        (void)hipEventDestroy(pr.e0);
        (void)hipEventDestroy(pr.e1);
    }
    c->pending.clear();
    if (call_ms) *call_ms = ms_call;
    return DWOS_OK;
}

dwos_status ensure_totals(dwos_ctx* c) {
    if (c->totals.bytes >= 3 * sizeof(dwos::Counters)) return DWOS_OK;
    HIP_OK(c->totals.reserve(3 * sizeof(dwos::Counters)));
    hipLaunchKernelGGL(dwos::fill_u64_kernel, dim3(1), dim3(64), 0, c->stream,
                       c->totals.as<unsigned long long>(), (int64_t)(3 * sizeof(dwos::Counters) / 8));
    return DWOS_OK;
}

template <class T, int D, int MODE, bool staged, bool cv>
dwos_status launch_shape(dwos_ctx* c, dwos::WalkArgs<T>& a, bool timed);

// Launch the persistent walk kernel over `total` walks.  FP32 uses the
// LDS-staged kernel (one large block per CU); the FP64 debug build keeps
// everything in global memory.  `tot` (cumulative counters of this walk
// kind) defaults to the context's; an untimed launch records no events.
template <class T, int D, int MODE>
dwos_status launch_walks(dwos_ctx* c, dwos::WalkArgs<T>& a, dwos::Counters* tot = nullptr,
                         bool timed = true) {
    hipStream_t s = c->stream;
    a.tot = tot ? tot : c->totals.as<dwos::Counters>() + (MODE ? 1 : 0);
    hipLaunchKernelGGL(dwos::fill_u64_kernel, dim3(1), dim3(64), 0, s, a.queue, (int64_t)1);
    if constexpr (MODE >= 1) {
        if (a.cv_run) {   // the build with the control variate's bookkeeping
            if constexpr (sizeof(T) == 4) {
                if (c->variant == 1) return launch_shape<T, D, MODE, false, true>(c, a, timed);
                return launch_shape<T, D, MODE, true, true>(c, a, timed);
            } else {
                return launch_shape<T, D, MODE, false, true>(c, a, timed);
            }
        }
    }
    if constexpr (sizeof(T) == 4) {
        if (c->variant == 1) return launch_shape<T, D, MODE, false, false>(c, a, timed);
        return launch_shape<T, D, MODE, true, false>(c, a, timed);
    } else {
        return launch_shape<T, D, MODE, false, false>(c, a, timed);
    }
}

template <class T, int D, int MODE, bool staged, bool cv>
dwos_status launch_shape(dwos_ctx* c, dwos::WalkArgs<T>& a, bool timed) {
    hipStream_t s = c->stream;
    constexpr int block = staged ? dwos::kBlockStaged : dwos::kBlock;
    const size_t smem = staged ? stage_bytes<T>(a.s, D) : 0;
    auto kern = dwos::walk_kernel<T, D, MODE, staged, cv>;
    // launch attributes and occupancy are computed once per kernel and LDS
    // size (no runtime queries on later, possibly captured, calls)
    static size_t attr_smem = 0;
    static size_t occ_smem = ~size_t(0);
    static int occ_per_cu = 1;
    if (smem > attr_smem) {
        HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
        attr_smem = smem;
    }
    if (occ_smem != smem) {
        int per = 0;
        HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, smem));
        occ_per_cu = std::max(1, per);
        occ_smem = smem;
    }
    const int per_cu = occ_per_cu;
    const int64_t need = (a.total + block - 1) / block;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)per_cu * c->cu_count));
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_OK(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone || !timed) {   // captured launches are not timed
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), smem, s, a);
        HIP_OK(hipGetLastError());
        return DWOS_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, s));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), smem, s, a);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(e1, s));
    c->pending.push_back({e0, e1, MODE ? 1 : 0});
    if (c->pending.size() > 4096) {
        dwos_status st = drain_events(c, nullptr, c->pending.size());
        if (st) return st;
    }
    return DWOS_OK;
}

// Launch the persistent walk-on-stars kernel (2D, reflecting boundary).
template <class T, int MODE>
dwos_status launch_wost(dwos_ctx* c, dwos::WalkArgs<T>& a0) {
    hipStream_t s = c->stream;
    dwos::WalkArgs<T> a = a0;
    a.tot = c->totals.as<dwos::Counters>() + MODE;
    hipLaunchKernelGGL(dwos::fill_u64_kernel, dim3(1), dim3(64), 0, s, a.queue, (int64_t)1);
    constexpr int block = dwos::kBlock;
    auto kern = dwos::wost_kernel<T, MODE>;
    dwos::RefScene<T> ref = make_ref<T>(c);
    size_t lds = 0;
    if constexpr (sizeof(T) == 4) {
        // LDS per block (a few blocks per CU): up to 256 Dirichlet nodes, its
        // primitives up to 16 KB, the reflecting BVH's first 128 nodes
        a.s.n_stage_nodes = (int32_t)std::min<int64_t>(c->n_nodes, 256);
        a.s.stage_prims = c->np * (int64_t)(dwos::prim_scalars(2) * sizeof(T)) <= 16384 ? 1 : 0;
        ref.n_stage = (int32_t)std::min<int64_t>(c->ref_nn, 128);
        const int64_t w_nodes = dwos::node_scalars(2) / 4;
        ref.stage_off4 = (int64_t)a.s.n_stage_nodes * w_nodes + (a.s.stage_prims ? c->np : 0);
        lds = (size_t)(ref.stage_off4 + (int64_t)ref.n_stage * (w_nodes + 2 * dwos::kRefCone / 4)) * 16;
    } else {
        a.s.n_stage_nodes = 0;
        a.s.stage_prims = 0;
        ref.n_stage = 0;
        ref.stage_off4 = 0;
    }
    static size_t occ_lds = ~size_t(0);
    static int occ_per_cu = 1;
    if (occ_lds != lds) {
        int per = 0;
        HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, lds));
        occ_per_cu = std::max(1, per);
        occ_lds = lds;
    }
    const int64_t need = (a.total + block - 1) / block;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)occ_per_cu * c->cu_count));
    const int32_t* starts = c->start_n > 0 ? c->start_seg.as<int32_t>() : nullptr;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_OK(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, a, ref, starts);
        HIP_OK(hipGetLastError());
        return DWOS_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, s));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, a, ref, starts);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(e1, s));
    c->pending.push_back({e0, e1, MODE});
    if (c->pending.size() > 4096) {
        dwos_status st = drain_events(c, nullptr, c->pending.size());
        if (st) return st;
    }
    return DWOS_OK;
}

// Launch the persistent walk-on-stars kernel (3D reflecting mesh).
template <class T, int MODE>
dwos_status launch_wost3(dwos_ctx* c, dwos::WalkArgs<T>& a0) {
    hipStream_t s = c->stream;
    dwos::WalkArgs<T> a = a0;
    a.tot = c->totals.as<dwos::Counters>() + MODE;
    hipLaunchKernelGGL(dwos::fill_u64_kernel, dim3(1), dim3(64), 0, s, a.queue, (int64_t)1);
    constexpr int block = dwos::kBlock;
    auto kern = dwos::wost3_kernel<T, MODE>;
    size_t lds = 0;
    dwos::RefScene3<T> ref = make_ref3<T>(c);
    if constexpr (sizeof(T) == 4) {
        // LDS per block (40 KB: four 256-thread blocks per CU): up to 64
        // Dirichlet nodes and its primitives up to 16 KB (the Dirichlet query
        // mostly runs bounded by the star radius), then as many of the edge
        // BVH's first nodes with their cones as fit (every silhouette query
        // descends through them)
        a.s.n_stage_nodes = (int32_t)std::min<int64_t>(c->n_nodes, 64);
        a.s.stage_prims = c->np * (int64_t)(dwos::prim_scalars(3) * sizeof(T)) <= 16384 ? 1 : 0;
        lds = (size_t)a.s.n_stage_nodes * dwos::node_scalars(3) * sizeof(T) +
              (a.s.stage_prims ? (size_t)c->np * dwos::prim_scalars(3) * sizeof(T) : 0);
        const size_t per_edge = (size_t)(dwos::node_scalars(3) + 2 * dwos::kEdgeCone) * sizeof(T);
        const size_t budget = 40 * 1024;
        lds = (lds + 15) & ~size_t(15);
        ref.n_estage = lds < budget ? (int32_t)std::min<int64_t>(c->ref_enn, (int64_t)((budget - lds) / per_edge)) : 0;
        if (c->stage_cap >= 0) ref.n_estage = std::min<int32_t>(ref.n_estage, c->stage_cap);
        ref.estage_off4 = (int64_t)(lds / 16);
        lds += (size_t)ref.n_estage * per_edge;
    } else {
        a.s.n_stage_nodes = 0;
        a.s.stage_prims = 0;
    }
    static size_t occ_lds = ~size_t(0);
    static int occ_per_cu = 1;
    if (occ_lds != lds) {
        int per = 0;
        HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, lds));
        occ_per_cu = std::max(1, per);
        occ_lds = lds;
    }
    const int64_t need = (a.total + block - 1) / block;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)occ_per_cu * c->cu_count));
    const int32_t* starts = c->start_n > 0 ? c->start_seg.as<int32_t>() : nullptr;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_OK(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, a, ref, starts);
        HIP_OK(hipGetLastError());
        return DWOS_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, s));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, a, ref, starts);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(e1, s));
    c->pending.push_back({e0, e1, MODE});
    if (c->pending.size() > 4096) {
        dwos_status st = drain_events(c, nullptr, c->pending.size());
        if (st) return st;
    }
    return DWOS_OK;
}

template <class T>
dwos_status ensure_records(dwos_ctx* c, int64_t walks, bool diff, bool steps) {
    HIP_OK(c->rec_u.reserve(walks * sizeof(T)));
    if (diff) {
        HIP_OK(c->rec_prim.reserve(walks * sizeof(int32_t)));
        HIP_OK(c->rec_b.reserve(walks * (c->D - 1) * sizeof(T)));
        HIP_OK(c->rec_uoff.reserve(walks * sizeof(T)));
    }
    if (steps) HIP_OK(c->rec_steps.reserve(walks * sizeof(int64_t)));
    if (diff && c->cv) {
        const int64_t nk = walks * c->prob.K;
        HIP_OK(c->cv_run.reserve(walks * sizeof(int32_t)));
        HIP_OK(c->cv_xoff.reserve(walks * c->D * sizeof(T)));
        HIP_OK(c->cv_xbar.reserve(walks * c->D * sizeof(T)));
        HIP_OK(c->cv_g.reserve(walks * sizeof(T)));
        HIP_OK(c->cv_target.reserve(walks * sizeof(T)));
        HIP_OK(c->cv_uplain.reserve(walks * sizeof(T)));
        HIP_OK(c->cv_Noff.reserve(walks * sizeof(float)));
        HIP_OK(c->cv_stop.reserve(nk * c->D * sizeof(T)));
        HIP_OK(c->cv_y.reserve(nk * c->D * sizeof(T)));
        HIP_OK(c->cv_rho.reserve(nk * sizeof(T)));
        HIP_OK(c->cv_d.reserve(nk * sizeof(T)));
        HIP_OK(c->cv_S.reserve(nk * sizeof(T)));
        HIP_OK(c->cv_alive.reserve(nk * sizeof(int32_t)));
        HIP_OK(c->cv_Nstop.reserve(nk * sizeof(float)));
        HIP_OK(c->cv_Ny.reserve(nk * sizeof(float)));
        HIP_OK(c->cv_Ly.reserve(nk * sizeof(float)));
    }
    HIP_OK(c->queue.reserve(sizeof(unsigned long long)));
    HIP_OK(c->counters.reserve(sizeof(dwos::Counters)));
    return DWOS_OK;
}

template <class T>
dwos::WalkArgs<T> base_args(dwos_ctx* c, const double* X, int32_t W, uint64_t seed) {
    dwos::WalkArgs<T> a{};
    a.s = make_scene<T>(c);
    a.prm = make_params<T>(c->prob);
    a.X = X;
    a.W = W;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.seed_ptr = reinterpret_cast<const unsigned long long*>(c->seed_dev);
    a.queue = c->queue.as<unsigned long long>();
    a.park = c->park;
    a.chunk = (uint32_t)c->chunk;
    a.cnt = c->counters.as<dwos::Counters>();
    a.tot = c->totals.as<dwos::Counters>();
    a.rec_u = c->rec_u.as<T>();
    a.rec_prim = c->rec_prim.as<int32_t>();
    a.rec_b = c->rec_b.as<T>();
    a.rec_uoff = c->rec_uoff.as<T>();
    a.rec_steps = nullptr;
    a.cv_run = nullptr;
    a.cv_qthresh = 1u << 24;
    a.prim_dep = c->has_params ? c->prim_dep.as<int32_t>() : nullptr;
    return a;
}

// Attach the control-variate records to a differential launch.
template <class T>
void cv_args(dwos_ctx* c, dwos::WalkArgs<T>& a) {
    a.cv_run = c->cv_run.as<int32_t>();
    a.cv_xoff = c->cv_xoff.as<T>();
    a.cv_xbar = c->cv_xbar.as<T>();
    a.cv_g = c->cv_g.as<T>();
    a.cv_stop = c->cv_stop.as<T>();
    a.cv_y = c->cv_y.as<T>();
    a.cv_rho = c->cv_rho.as<T>();
    a.cv_d = c->cv_d.as<T>();
    a.cv_S = c->cv_S.as<T>();
    a.cv_alive = c->cv_alive.as<int32_t>();
    a.cv_qthresh = c->cv_qthresh;
}

// Network values at the recorded points, then the control-variate estimate
// of every nested mean (in place in rec_uoff).
// Once per differential call: beta from the previous call's sums (or 1 after
// attaching), sums cleared.
dwos_status cv_begin(dwos_ctx* c) {
    HIP_OK(c->cv_beta.reserve(sizeof(double)));
    HIP_OK(c->cv_stats.reserve(3 * sizeof(double)));
    hipLaunchKernelGGL(dwos::cv_beta_kernel, dim3(1), dim3(64), 0, c->stream, c->cv_beta.as<double>(),
                       c->cv_stats.as<double>(), c->cv_fresh ? 1 : 0);
    c->cv_fresh = false;
    return DWOS_OK;
}

template <class T, int D>
dwos_status cv_apply(dwos_ctx* c, int64_t walks) {
    hipStream_t s = c->stream;
    const int K = c->prob.K;
    const int32_t* run = c->cv_run.as<int32_t>();
    HIP_OK(dwos_host::mlp_eval_launch<T>(c->cv, s, c->cv_xoff.as<T>(), walks, run, 1, 0,
                                         c->cv_Noff.as<float>(), nullptr, nullptr));
    HIP_OK(dwos_host::mlp_eval_launch<T>(c->cv, s, c->cv_stop.as<T>(), walks * K, run, K, 1,
                                         c->cv_Nstop.as<float>(), nullptr, nullptr));
    HIP_OK(dwos_host::mlp_eval_launch<T>(c->cv, s, c->cv_y.as<T>(), walks * K, run, K, 1,
                                         c->cv_Ny.as<float>(), nullptr, c->cv_Ly.as<float>()));
    dwos::CvCombineArgs<T> ca{};
    ca.run = run;
    ca.prim = c->rec_prim.as<int32_t>();
    ca.pverts = c->pverts.as<int32_t>();
    ca.vparam = c->has_params ? c->vparam.as<int32_t>() : nullptr;
    ca.S = c->cv_S.as<T>();
    ca.alive = c->cv_alive.as<int32_t>();
    ca.rho = c->cv_rho.as<T>();
    ca.d = c->cv_d.as<T>();
    ca.Noff = c->cv_Noff.as<float>();
    ca.Nstop = c->cv_Nstop.as<float>();
    ca.Ny = c->cv_Ny.as<float>();
    ca.Ly = c->cv_Ly.as<float>();
    ca.uoff = c->rec_uoff.as<T>();
    ca.target = c->cv_target.as<T>();
    ca.uoff_plain = c->cv_uplain.as<T>();
    ca.beta = c->cv_beta.as<double>();
    ca.stats = c->cv_stats.as<double>();
    ca.nwalks = walks;
    ca.K = K;
    ca.sigma = T(c->prob.sigma);
    ca.kappa = T(std::sqrt(c->prob.sigma));
    ca.inv_q = T(16777216.0 / (double)c->cv_qthresh);
    hipLaunchKernelGGL((dwos::cv_combine_kernel<T, D>), dim3(blocks_for(walks, 256)), dim3(256), 0, s, ca);
    c->cv_nrec = walks;
    return DWOS_OK;
}

// Upload an instance table (skipped when identical to the last one).  The
// host copy lives in the context, so the asynchronous copy needs no sync.
template <class T>
dwos_status upload_instances(dwos_ctx* c, const dwos::Instance<T>* in, size_t n) {
    const size_t bytes = n * sizeof(dwos::Instance<T>);
    const unsigned char* src = reinterpret_cast<const unsigned char*>(in);
    if (c->inst_host.size() == bytes && std::memcmp(c->inst_host.data(), src, bytes) == 0 &&
        c->instbuf.bytes >= bytes)
        return DWOS_OK;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_OK(hipStreamIsCapturing(c->stream, &cap));
    if (cap != hipStreamCaptureStatusNone)
        return fail(DWOS_ESTATE, "instance table changed during graph capture: run the call once before capturing");
    HIP_OK(hipStreamSynchronize(c->stream));   // the previous table may still be in use
    c->inst_host.assign(src, src + bytes);
    HIP_OK(c->instbuf.reserve(bytes));
    HIP_OK(hipMemcpyAsync(c->instbuf.ptr, c->inst_host.data(), bytes, hipMemcpyHostToDevice, c->stream));
    return DWOS_OK;
}

// Per batch instance the leaf positions of its primitives, [begin, end), so
// that a first query may start from the previous call's answer for its row
// only when that primitive is the row's instance's.
dwos_status upload_prange(dwos_ctx* c) {
    const size_t n = c->instances.size();
    std::vector<int32_t> pr(2 * std::max<size_t>(1, n), 0);
    for (size_t i = 0; i < n; ++i) {
        pr[2 * i] = (int32_t)c->instances[i].np_off;
        pr[2 * i + 1] = (int32_t)(i + 1 < n ? c->instances[i + 1].np_off : (int64_t)c->hostOrder.size());
    }
    HIP_OK(upload(c->inst_prange, pr.data(), pr.size(), c->stream));
    return DWOS_OK;
}

// single-instance table for points [p0, p0 + P) of a chunk
template <class T>
dwos_status set_single_instance(dwos_ctx* c, int64_t p0, int64_t P, int32_t W) {
    dwos::Instance<T> in{};
    in.walk_begin = 0;
    in.point_begin = p0;
    in.p_counter = p0;
    in.root = 0;
    in.P = (int32_t)P;
    const double sg = c->prob.sigma;
    in.kappa = T(std::sqrt(sg));
    in.eps = T(c->prob.eps);
    in.delta = T(c->prob.delta);
    return upload_instances(c, &in, 1);
}

dwos_status begin_call(dwos_ctx* c, bool need_params) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!c->has_boundary && !c->has_imp)
        return fail(DWOS_ESTATE, "no boundary: call dwos_set_boundary (or dwos_set_implicit) first");
    if (!c->has_problem) return fail(DWOS_ESTATE, "no problem: call dwos_set_problem first");
    if (need_params && !c->has_params && !c->has_imp)
        return fail(DWOS_ESTATE, "no parameters: call dwos_set_parameters first");
    HIP_OK(hipSetDevice(c->device));
    HIP_OK(c->counters.reserve(sizeof(dwos::Counters)));
    hipLaunchKernelGGL(dwos::fill_u64_kernel, dim3(1), dim3(64), 0, c->stream,
                       c->counters.as<unsigned long long>(), (int64_t)(sizeof(dwos::Counters) / 8));
    return ensure_totals(c);
}

// Entry points of a single problem (not a batch context's instances).
dwos_status single_call(dwos_ctx* c, bool need_params) {
    if (c && !c->instances.empty())
        return fail(DWOS_ESTATE, "batch context: use dwos_batch_solve / dwos_batch_grad");
    return begin_call(c, need_params);
}

dwos_status finish_call(dwos_ctx* c, dwos_stats* st, size_t ev_from) {
    HIP_OK(hipGetLastError());
    if (!st) return DWOS_OK;
    HIP_OK(hipStreamSynchronize(c->stream));
    dwos::Counters h{};
    HIP_OK(hipMemcpy(&h, c->counters.ptr, sizeof(h), hipMemcpyDeviceToHost));
    st->walks = (int64_t)h.walks;
    st->nested_walks = (int64_t)h.nested;
    st->steps = (int64_t)h.steps;
    st->terminal = (int64_t)h.terminal;
    st->truncated = (int64_t)h.truncated;
    st->nodes = (int64_t)h.nodes;
    st->prims = (int64_t)h.prims;
    st->stack_overflow = (int64_t)h.overflow;
    st->invalid = (int64_t)h.invalid;
    double ms = 0.0;
    dwos_status s = drain_events(c, &ms, ev_from);
    st->walk_ms = ms;
    return s;
}

// ---------------------------------------------------------------------------
// the main driver: walks over chunks of points, then per-chunk reductions
// ---------------------------------------------------------------------------
enum class Op { Solve, Grad, SqLoss, Jvp, Records };

struct OpArgs {
    const double* X;
    int64_t P;
    int32_t W, B;
    uint64_t seed;
    const double* w;
    const double* uref;
    double* u_mean;
    double* u_var;
    double* grad;
    double* loss;
    double* udot;
    double* udot_var;
    // records op
    double* rec_u_out;
    int64_t* rec_steps_out;
    int32_t* rec_prim_out;
    double* rec_uoff_out;
    double* rec_udot_out;
    int32_t mode;
    // control-variate record export (oracle layout)
    double* cv_walk_out;
    double* cv_nested_out;
};

template <class T>
__global__ void copy_records_kernel(const T* u, const int32_t* prim, const T* uoff, int64_t n, int64_t off,
                                    double* uo, int32_t* po, double* uoffo, int diff) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uo[off + i] = double(u[i]);
    if (po) po[off + i] = diff ? (prim[i] >= 0 ? (prim[i] >> 1) : -1) : -1;
    if (uoffo) uoffo[off + i] = diff ? double(uoff[i]) : 0.0;
}

__global__ void copy_steps_kernel(const int64_t* s, int64_t n, int64_t off, int64_t* o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[off + i] = s[i];
}

template <class T, int D>
dwos_status run_op(dwos_ctx* c, Op op, const OpArgs& o, dwos_stats* st) {
    const bool diff = op != Op::Solve && !(op == Op::Records && o.mode == 0);
    const int64_t P = o.P;
    const int32_t W = o.W;
    hipStream_t s = c->stream;
    if (c->has_ref && diff && c->cv)
        return fail(DWOS_ESTATE, "the control variate is not supported with a reflecting boundary");
    const bool bvc = diff && c->prob.dudn == 1;
    if (bvc && (c->cv || c->has_ref))
        return fail(DWOS_ESTATE, "the gradient normal-derivative estimator takes neither a control variate "
                                 "nor a reflecting boundary");
    if (c->start_n > 0 && c->start_n != P)
        return fail(DWOS_EINVAL, "start segments were set for " + std::to_string(c->start_n) +
                                     " points, the call has " + std::to_string(P));
    const int64_t chunk_pts = std::max<int64_t>(1, kMaxWalksPerChunk / W);
    const int64_t max_walks = std::min<int64_t>(P, chunk_pts) * W;
    dwos_status rc = ensure_records<T>(c, std::max<int64_t>(1, max_walks), diff, op == Op::Records);
    if (rc) return rc;
    const size_t ev_from = c->pending.size();
    const bool needA = op == Op::Grad || op == Op::SqLoss;
    if (needA) {
        HIP_OK(c->accA.reserve(c->nv * D * sizeof(double)));
        HIP_OK(c->accB.reserve(c->nv * sizeof(double)));
        hipLaunchKernelGGL(dwos::fill_f64_kernel, dim3(blocks_for(c->nv * D, 256)), dim3(256), 0, s,
                           c->accA.as<double>(), c->nv * D);
        hipLaunchKernelGGL(dwos::fill_f64_kernel, dim3(blocks_for(c->nv, 256)), dim3(256), 0, s,
                           c->accB.as<double>(), c->nv);
    }
    const dwos::Params<T> prm = make_params<T>(c->prob);
    const dwos::Scene<T> scene = make_scene<T>(c);
    if (diff && c->cv) {
        rc = cv_begin(c);
        if (rc) return rc;
    }
    for (int64_t p0 = 0; p0 < P; p0 += chunk_pts) {
        const int64_t Pc = std::min(chunk_pts, P - p0);
        const int64_t walks = Pc * W;
        rc = set_single_instance<T>(c, p0, Pc, W);
        if (rc) return rc;
        dwos::WalkArgs<T> a = base_args<T>(c, o.X, W, o.seed);
        a.inst = c->instbuf.as<dwos::Instance<T>>();
        a.n_inst = 1;
        a.total = walks;
        a.wid_offset = 0;
        // every walk of a point starts with the same closest-point query,
        // started from the primitive the previous query of that row found
        // (any primitive of the scene only bounds the search: the answer is
        // the same; callers solve at the same points again and again)
        const void* fl_old = c->first_leaf.ptr;
        HIP_OK(c->first_leaf.reserve(Pc * sizeof(int32_t)));
        if (c->first_leaf.ptr != fl_old) c->first_warm = false;
        HIP_OK(c->first_d2.reserve(Pc * sizeof(T)));
        hipLaunchKernelGGL((dwos::first_query_kernel<T, D>), dim3(blocks_for(Pc, 64)), dim3(64), 0, s, scene,
                           c->instbuf.as<dwos::Instance<T>>(), 1, o.X + p0 * D, p0, Pc, nullptr,
                           c->first_warm ? c->first_leaf.as<int32_t>() : nullptr, c->first_leaf.as<int32_t>(),
                           c->first_d2.as<T>());
        c->first_warm = true;
        a.first_leaf = c->first_leaf.as<int32_t>();
        a.first_d2 = c->first_d2.as<T>();
        a.x_base = p0;
        a.rec_steps = op == Op::Records ? c->rec_steps.as<int64_t>() : nullptr;
        // 3D meshes: hand the points out in a spatially coherent order (the
        // walks in flight then share the BVH's cache lines); only scheduling
        // changes, every walk and record is the same
        a.perm = nullptr;
        if (D == 3 && Pc >= 1024) {
            HIP_OK(c->order_cell.reserve(Pc * sizeof(int32_t)));
            HIP_OK(c->order_perm.reserve(Pc * sizeof(int32_t)));
            HIP_OK(c->order_hist.reserve(dwos::kOrderCells * sizeof(uint32_t)));
            hipLaunchKernelGGL(dwos::fill_u64_kernel, dim3(blocks_for(dwos::kOrderCells / 2, 64)), dim3(64), 0, s,
                               c->order_hist.as<unsigned long long>(), (int64_t)(dwos::kOrderCells / 2));
            hipLaunchKernelGGL((dwos::order_cell_kernel<T, D>), dim3(blocks_for(Pc, 256)), dim3(256), 0, s,
                               c->nodes.as<T>(), o.X + p0 * D, Pc, c->order_cell.as<int32_t>(),
                               c->order_hist.as<uint32_t>());
            hipLaunchKernelGGL(dwos::order_scan_kernel, dim3(1), dim3(1024), 0, s, c->order_hist.as<uint32_t>());
            hipLaunchKernelGGL(dwos::order_scatter_kernel, dim3(blocks_for(Pc, 256)), dim3(256), 0, s,
                               c->order_cell.as<int32_t>(), Pc, c->order_hist.as<uint32_t>(),
                               c->order_perm.as<int32_t>());
            a.perm = c->order_perm.as<int32_t>();
        }
        const bool use_cv = diff && c->cv != nullptr;
        if (use_cv) cv_args<T>(c, a);
        const bool robin_w = diff && c->has_ref && c->robin;
        if (robin_w) {
            HIP_OK(c->rec_w.reserve(std::max<int64_t>(1, max_walks) * sizeof(T)));
            a.rec_w = c->rec_w.as<T>();
        }
        // walk ids within a chunk restart at 0; the instance's p_counter = p0
        // keeps the Philox point word absolute
        if constexpr (D == 2) {
            if (c->has_ref) rc = diff ? launch_wost<T, 1>(c, a) : launch_wost<T, 0>(c, a);
            else if (bvc) rc = launch_walks<T, D, 2>(c, a);
            else rc = diff ? launch_walks<T, D, 1>(c, a) : launch_walks<T, D, 0>(c, a);
        } else {
            if (c->has_ref) rc = diff ? launch_wost3<T, 1>(c, a) : launch_wost3<T, 0>(c, a);
            else if (bvc) rc = launch_walks<T, D, 2>(c, a);
            else rc = diff ? launch_walks<T, D, 1>(c, a) : launch_walks<T, D, 0>(c, a);
        }
        if (rc) return rc;
        if (use_cv) {
            rc = cv_apply<T, D>(c, walks);
            if (rc) return rc;
            if (o.cv_walk_out)
                hipLaunchKernelGGL((dwos::cv_export_kernel<T, D>), dim3(blocks_for(walks, 256)), dim3(256), 0, s,
                                   c->cv_run.as<int32_t>(), c->cv_xoff.as<T>(), c->cv_uplain.as<T>(),
                                   c->rec_uoff.as<T>(), c->cv_target.as<T>(), c->rec_u.as<T>(),
                                   c->rec_prim.as<int32_t>(), c->cv_S.as<T>(), c->cv_alive.as<int32_t>(),
                                   c->cv_stop.as<T>(),
                                   c->cv_y.as<T>(), c->cv_rho.as<T>(), c->cv_d.as<T>(), walks, c->prob.K,
                                   p0 * W, o.cv_walk_out, o.cv_nested_out);
        }
        // per-point statistics
        if (o.u_mean) {
            hipLaunchKernelGGL(dwos::point_stats_kernel<T>, dim3(blocks_for(Pc, 4)), dim3(256), 0, s,
                               c->rec_u.as<T>(), Pc, W, o.u_mean + p0, o.u_var ? o.u_var + p0 : nullptr);
        }
        if (needA) {
            dwos::AccArgs<T> aa{};
            aa.s = scene;
            aa.prm = prm;
            aa.delta = T(c->prob.delta);
            aa.rec_u = c->rec_u.as<T>();
            aa.rec_prim = c->rec_prim.as<int32_t>();
            aa.rec_b = c->rec_b.as<T>();
            aa.rec_uoff = c->rec_uoff.as<T>();
            aa.rec_w = robin_w ? c->rec_w.as<T>() : nullptr;
            aa.nwalks = walks;
            aa.p_offset = p0;
            aa.W = W;
            aa.B = o.B;
            aa.mode = op == Op::Grad ? 0 : 1;
            aa.w = o.w;
            aa.uref = o.uref;
            aa.bc_pid = c->has_bc_params ? c->bc_pid.as<int32_t>() : nullptr;
            aa.prim_dep = c->prim_dep.as<int32_t>();
            aa.vparam = c->vparam.as<int32_t>();
            aa.A = c->accA.as<double>();
            aa.Bacc = c->accB.as<double>();
            hipLaunchKernelGGL((dwos::accumulate_kernel<T, D>), dim3(blocks_for(walks, 256)), dim3(256), 0, s, aa);
        }
        if (op == Op::Jvp || (op == Op::Records && diff && o.rec_udot_out)) {
            dwos::JvpArgs<T> ja{};
            ja.s = scene;
            ja.prm = prm;
            ja.delta = T(c->prob.delta);
            ja.J = make_csr(c);
            ja.rec_prim = c->rec_prim.as<int32_t>();
            ja.rec_b = c->rec_b.as<T>();
            ja.rec_uoff = c->rec_uoff.as<T>();
            ja.rec_w = robin_w ? c->rec_w.as<T>() : nullptr;
            ja.P = Pc;
            ja.p_offset = p0;
            ja.W = W;
            ja.udot = op == Op::Jvp ? o.udot : nullptr;
            ja.udot_var = op == Op::Jvp ? o.udot_var : nullptr;
            ja.walk_udot = op == Op::Records ? o.rec_udot_out + p0 * W * c->N : nullptr;
            dim3 grid((unsigned)Pc, (unsigned)((c->N + 63) / 64));
            hipLaunchKernelGGL((dwos::jvp_kernel<T, D>), grid, dim3(64), 0, s, ja);
        }
        if (op == Op::Records) {
            hipLaunchKernelGGL(copy_records_kernel<T>, dim3(blocks_for(walks, 256)), dim3(256), 0, s,
                               c->rec_u.as<T>(), diff ? c->rec_prim.as<int32_t>() : nullptr,
                               diff ? c->rec_uoff.as<T>() : nullptr, walks, p0 * W, o.rec_u_out,
                               o.rec_prim_out, o.rec_uoff_out, diff ? 1 : 0);
            if (o.rec_steps_out)
                hipLaunchKernelGGL(copy_steps_kernel, dim3(blocks_for(walks, 256)), dim3(256), 0, s,
                                   c->rec_steps.as<int64_t>(), walks, p0 * W, o.rec_steps_out);
        }
    }
    if (needA) {
        hipLaunchKernelGGL(dwos::spmv_kernel<D>, dim3(blocks_for(c->N, 4)), dim3(256), 0, s, make_csr(c),
                           c->accA.as<double>(), c->accB.as<double>(), o.grad);
    }
    if (op == Op::SqLoss && o.loss) {
        hipLaunchKernelGGL(dwos::sqloss_kernel, dim3(1), dim3(256), 0, s, o.u_mean, o.uref, P, o.loss);
    }
    return finish_call(c, st, ev_from);
}

// ---------------------------------------------------------------------------
// allocation-free solve: every workspace in the device's `scratch` array
// ---------------------------------------------------------------------------
template <class T>
__global__ void set_instance_kernel(dwos::Instance<T>* dst, dwos::Instance<T> v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = v;
}

// Layout of the scratch array for a solve of P points x W walks: work-queue
// counter, this call's and the cumulative walk counters, the instance, then
// 256-byte aligned per-point first queries and per-walk values.
struct NoAllocLayout {
    size_t queue = 0, cnt = 64, tot = 256, inst = 512, head = 1024;
    size_t leaf, d2, rec, end;
    NoAllocLayout(int64_t P, int32_t W, size_t el) {
        auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
        leaf = head;
        d2 = leaf + up((size_t)P * sizeof(int32_t));
        rec = d2 + up((size_t)P * el);
        end = rec + up((size_t)P * (size_t)W * el);
    }
};

template <class T, int D>
dwos_status run_solve_noalloc(dwos_ctx* c, const double* X, int64_t P, int32_t W, uint64_t seed, double* u_mean,
                              double* u_var, unsigned char* base) {
    static_assert(sizeof(dwos::Counters) <= 192 && sizeof(dwos::Instance<T>) <= 512, "scratch header layout");
    hipStream_t s = c->stream;
    const NoAllocLayout L(P, W, sizeof(T));
    // clear the header (queue, counters, instance slot) with a fill kernel
    hipLaunchKernelGGL(dwos::fill_u64_kernel, dim3(blocks_for((int64_t)(L.head / 8), 64)), dim3(64), 0, s,
                       reinterpret_cast<unsigned long long*>(base), (int64_t)(L.head / 8));
    dwos::Instance<T> in{};
    in.walk_begin = 0;
    in.point_begin = 0;
    in.p_counter = 0;
    in.root = 0;
    in.P = (int32_t)P;
    in.kappa = T(std::sqrt(c->prob.sigma));
    in.eps = T(c->prob.eps);
    in.delta = T(c->prob.delta);
    auto* inst = reinterpret_cast<dwos::Instance<T>*>(base + L.inst);
    hipLaunchKernelGGL(set_instance_kernel<T>, dim3(1), dim3(64), 0, s, inst, in);
    const dwos::Scene<T> scene = make_scene<T>(c);
    auto* leaf = reinterpret_cast<int32_t*>(base + L.leaf);
    auto* d2 = reinterpret_cast<T*>(base + L.d2);
    hipLaunchKernelGGL((dwos::first_query_kernel<T, D>), dim3(blocks_for(P, 64)), dim3(64), 0, s, scene, inst, 1, X,
                       (int64_t)0, P, nullptr, nullptr, leaf, d2);
    dwos::WalkArgs<T> a = base_args<T>(c, X, W, seed);
    a.inst = inst;
    a.n_inst = 1;
    a.total = P * (int64_t)W;
    a.wid_offset = 0;
    a.queue = reinterpret_cast<unsigned long long*>(base + L.queue);
    a.cnt = reinterpret_cast<dwos::Counters*>(base + L.cnt);
    a.rec_u = reinterpret_cast<T*>(base + L.rec);
    a.rec_prim = nullptr;
    a.rec_b = nullptr;
    a.rec_uoff = nullptr;
    a.rec_steps = nullptr;
    a.first_leaf = leaf;
    a.first_d2 = d2;
    a.x_base = 0;
    dwos_status rc = launch_walks<T, D, 0>(c, a, reinterpret_cast<dwos::Counters*>(base + L.tot), false);
    if (rc) return rc;
    hipLaunchKernelGGL(dwos::point_stats_kernel<T>, dim3(blocks_for(P, 4)), dim3(256), 0, s, a.rec_u, P, W, u_mean,
                       u_var);
    HIP_OK(hipGetLastError());
    return DWOS_OK;
}

// Launch the persistent implicit-boundary walk kernel (2D).
template <class T, int MODE>
dwos_status launch_imp(dwos_ctx* c, dwos::WalkArgs<T>& a) {
    hipStream_t s = c->stream;
    a.tot = c->totals.as<dwos::Counters>() + MODE;
    hipLaunchKernelGGL(dwos::fill_u64_kernel, dim3(1), dim3(64), 0, s, a.queue, (int64_t)1);
    constexpr int block = dwos::kBlock;
    auto kern = dwos::implicit_kernel<T, MODE>;
    const size_t lds = (size_t)std::max<int64_t>(c->imp_n, dwos::kImpRegs) * 3 * sizeof(T);
    int per = 0;
    HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, lds));
    per = std::max(1, per);
    const int64_t need = (a.total + block - 1) / block;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)per * c->cu_count));
    dwos::ImpArgs<T> im{};
    im.mono = c->imp_mono.as<T>();
    im.n = (int32_t)c->imp_n;
    im.c = T(c->imp_c);
    im.xbar = c->imp_xbar.as<T>();
    im.s = c->imp_s.as<T>();
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_OK(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, a, im);
        HIP_OK(hipGetLastError());
        return DWOS_OK;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    HIP_OK(hipEventRecord(e0, s));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, a, im);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(e1, s));
    c->pending.push_back({e0, e1, MODE});
    if (c->pending.size() > 4096) {
        dwos_status st = drain_events(c, nullptr, c->pending.size());
        if (st) return st;
    }
    return DWOS_OK;
}

// The driver for an implicit boundary: the same chunking, records and
// per-point statistics as run_op; the parameters are the 3n monopole
// coordinates (a_n, p_n), so forward and reverse mode reduce the per-walk
// terminal data (xbar, s) with imp_jvp_kernel and imp_grad_kernel.
template <class T>
dwos_status run_imp(dwos_ctx* c, Op op, const OpArgs& o, dwos_stats* st) {
    const bool diff = op != Op::Solve && !(op == Op::Records && o.mode == 0);
    const int64_t P = o.P;
    const int32_t W = o.W;
    hipStream_t s = c->stream;
    if (c->cv) return fail(DWOS_ESTATE, "the control variate is not supported on an implicit boundary");
    if (diff && c->prob.dudn != 0)
        return fail(DWOS_ESTATE, "the gradient normal-derivative estimator is not available on an implicit boundary");
    if (c->prob.bc[0].kind != 0)
        return fail(DWOS_ESTATE, "an implicit boundary takes restricted (quadratic) boundary data of label 0");
    const int64_t chunk_pts = std::max<int64_t>(1, kMaxWalksPerChunk / W);
    const int64_t max_walks = std::max<int64_t>(1, std::min<int64_t>(P, chunk_pts) * W);
    dwos_status rc = ensure_records<T>(c, max_walks, diff, op == Op::Records);
    if (rc) return rc;
    const bool needA = op == Op::Grad || op == Op::SqLoss;
    if (diff) {
        HIP_OK(c->imp_xbar.reserve(max_walks * 2 * sizeof(T)));
        HIP_OK(c->imp_s.reserve(max_walks * sizeof(T)));
    }
    if (needA) {
        HIP_OK(c->imp_coef.reserve(max_walks * sizeof(double)));
        hipLaunchKernelGGL(dwos::fill_f64_kernel, dim3(blocks_for(c->N, 256)), dim3(256), 0, s, o.grad, c->N);
    }
    const size_t ev_from = c->pending.size();
    const int32_t n = (int32_t)c->imp_n;
    for (int64_t p0 = 0; p0 < P; p0 += chunk_pts) {
        const int64_t Pc = std::min(chunk_pts, P - p0);
        const int64_t walks = Pc * W;
        rc = set_single_instance<T>(c, p0, Pc, W);
        if (rc) return rc;
        dwos::WalkArgs<T> a = base_args<T>(c, o.X, W, o.seed);
        a.inst = c->instbuf.as<dwos::Instance<T>>();
        a.n_inst = 1;
        a.total = walks;
        a.wid_offset = 0;
        a.x_base = p0;
        a.rec_steps = op == Op::Records ? c->rec_steps.as<int64_t>() : nullptr;
        rc = diff ? launch_imp<T, 1>(c, a) : launch_imp<T, 0>(c, a);
        if (rc) return rc;
        if (o.u_mean) {
            hipLaunchKernelGGL(dwos::point_stats_kernel<T>, dim3(blocks_for(Pc, 4)), dim3(256), 0, s,
                               c->rec_u.as<T>(), Pc, W, o.u_mean + p0, o.u_var ? o.u_var + p0 : nullptr);
        }
        if (needA) {
            hipLaunchKernelGGL(dwos::imp_coef_kernel<T>, dim3(blocks_for(walks, 256)), dim3(256), 0, s,
                               c->rec_u.as<T>(), c->rec_prim.as<int32_t>(), walks, W,
                               op == Op::SqLoss ? o.B : 1, op == Op::Grad ? 0 : 1, p0, o.w, o.uref,
                               c->imp_coef.as<double>());
            hipLaunchKernelGGL(dwos::imp_grad_kernel<T>, dim3(blocks_for(walks, dwos::kImpTile)), dim3(256), 0, s,
                               c->imp_xbar.as<T>(), c->imp_s.as<T>(), c->imp_coef.as<double>(), walks,
                               c->imp_mono.as<T>(), n, o.grad);
        }
        if (op == Op::Jvp || (op == Op::Records && diff && o.rec_udot_out)) {
            hipLaunchKernelGGL(dwos::imp_jvp_kernel<T>, dim3((unsigned)Pc), dim3(64), 0, s, c->rec_prim.as<int32_t>(),
                               c->imp_xbar.as<T>(), c->imp_s.as<T>(), c->imp_mono.as<T>(), n, Pc, W, p0,
                               op == Op::Jvp ? o.udot : nullptr, op == Op::Jvp ? o.udot_var : nullptr,
                               op == Op::Records ? o.rec_udot_out + p0 * W * c->N : nullptr);
        }
        if (op == Op::Records) {
            hipLaunchKernelGGL(copy_records_kernel<T>, dim3(blocks_for(walks, 256)), dim3(256), 0, s,
                               c->rec_u.as<T>(), diff ? c->rec_prim.as<int32_t>() : nullptr,
                               diff ? c->rec_uoff.as<T>() : nullptr, walks, p0 * W, o.rec_u_out,
                               o.rec_prim_out, o.rec_uoff_out, diff ? 1 : 0);
            if (o.rec_steps_out)
                hipLaunchKernelGGL(copy_steps_kernel, dim3(blocks_for(walks, 256)), dim3(256), 0, s,
                                   c->rec_steps.as<int64_t>(), walks, p0 * W, o.rec_steps_out);
        }
    }
    if (op == Op::SqLoss && o.loss) {
        hipLaunchKernelGGL(dwos::sqloss_kernel, dim3(1), dim3(256), 0, s, o.u_mean, o.uref, P, o.loss);
    }
    return finish_call(c, st, ev_from);
}

// Adjoint formulation (Appendix B): one lane per (sample, walk) writes the
// terminal record and its two weights, the mode-2 scatter and the SpMV give
// grad.
template <class T, int D>
dwos_status run_adjoint(dwos_ctx* c, const int32_t* code, const double* bary, const double* wq, int64_t S,
                        const dwos_quad* uref, int32_t W, uint64_t seed, double* grad, double* lam, double* uoff,
                        dwos_stats* st) {
    hipStream_t s = c->stream;
    const int64_t walks = S * W;
    const size_t ev_from = c->pending.size();
    dwos_status rc = ensure_records<T>(c, std::max<int64_t>(1, walks), true, false);
    if (rc) return rc;
    HIP_OK(c->adj_w.reserve(std::max<int64_t>(1, walks) * sizeof(double)));
    HIP_OK(c->adj_e.reserve(std::max<int64_t>(1, walks) * sizeof(double)));
    HIP_OK(c->accA.reserve(c->nv * D * sizeof(double)));
    HIP_OK(c->accB.reserve(c->nv * sizeof(double)));
    hipLaunchKernelGGL(dwos::fill_f64_kernel, dim3(blocks_for(c->nv * D, 256)), dim3(256), 0, s,
                       c->accA.as<double>(), c->nv * D);
    hipLaunchKernelGGL(dwos::fill_f64_kernel, dim3(blocks_for(c->nv, 256)), dim3(256), 0, s,
                       c->accB.as<double>(), c->nv);
    if (walks > 0) {
        dwos::AdjArgs<T> a{};
        a.s = make_scene<T>(c);
        a.s.n_stage_nodes = 0;
        a.s.stage_prims = 0;
        a.prm = make_params<T>(c->prob);
        a.kappa = T(std::sqrt(c->prob.sigma));
        a.eps = T(c->prob.eps);
        a.delta = T(c->prob.delta);
        a.code = code;
        a.bary = bary;
        a.wq = wq;
        a.S = S;
        a.W = W;
        a.ref[0] = uref->c;
        for (int i = 0; i < 3; ++i) a.ref[1 + i] = uref->b[i];
        for (int i = 0; i < 9; ++i) a.ref[4 + i] = uref->A[i];
        a.key0 = (uint32_t)seed;
        a.key1 = (uint32_t)(seed >> 32);
        a.prim_dep = c->prim_dep.as<int32_t>();
        a.rec_prim = c->rec_prim.as<int32_t>();
        a.rec_b = c->rec_b.as<T>();
        a.rec_uoff = c->rec_uoff.as<T>();
        a.rec_w = c->adj_w.as<double>();
        a.rec_e = c->adj_e.as<double>();
        a.out_lam = lam;
        a.out_uoff = uoff;
        a.cnt = c->counters.as<dwos::Counters>();
        a.tot = c->totals.as<dwos::Counters>() + 2;
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        HIP_OK(hipStreamIsCapturing(s, &cap));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (cap == hipStreamCaptureStatusNone) {
            HIP_OK(hipEventCreate(&e0));
            HIP_OK(hipEventCreate(&e1));
            HIP_OK(hipEventRecord(e0, s));
        }
        hipLaunchKernelGGL((dwos::adjoint_kernel<T, D>), dim3(blocks_for(walks, 256)), dim3(256), 0, s, a);
        HIP_OK(hipGetLastError());
        if (cap == hipStreamCaptureStatusNone) {
            HIP_OK(hipEventRecord(e1, s));
            c->pending.push_back({e0, e1, 2});
        }
        dwos::AccArgs<T> aa{};
        aa.s = a.s;
        aa.prm = a.prm;
        aa.delta = a.delta;
        aa.rec_prim = c->rec_prim.as<int32_t>();
        aa.rec_b = c->rec_b.as<T>();
        aa.rec_uoff = c->rec_uoff.as<T>();
        aa.nwalks = walks;
        aa.p_offset = 0;
        aa.W = W;
        aa.B = 1;
        aa.mode = 2;
        aa.w = c->adj_w.as<double>();
        aa.e = c->adj_e.as<double>();
        aa.bc_pid = c->has_bc_params ? c->bc_pid.as<int32_t>() : nullptr;
        aa.prim_dep = c->prim_dep.as<int32_t>();
        aa.vparam = c->vparam.as<int32_t>();
        aa.A = c->accA.as<double>();
        aa.Bacc = c->accB.as<double>();
        hipLaunchKernelGGL((dwos::accumulate_kernel<T, D>), dim3(blocks_for(walks, 256)), dim3(256), 0, s, aa);
    }
    hipLaunchKernelGGL(dwos::spmv_kernel<D>, dim3(blocks_for(c->N, 4)), dim3(256), 0, s, make_csr(c),
                       c->accA.as<double>(), c->accB.as<double>(), grad);
    return finish_call(c, st, ev_from);
}

dwos_status dispatch(dwos_ctx* c, Op op, const OpArgs& o, dwos_stats* st) {
    if (c->has_imp) return c->prec == DWOS_FP32 ? run_imp<float>(c, op, o, st) : run_imp<double>(c, op, o, st);
    if (c->prec == DWOS_FP32) {
        return c->D == 2 ? run_op<float, 2>(c, op, o, st) : run_op<float, 3>(c, op, o, st);
    }
    return c->D == 2 ? run_op<double, 2>(c, op, o, st) : run_op<double, 3>(c, op, o, st);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* dwos_last_error(void) { return dwos_host::g_last_error.c_str(); }

dwos_status dwos_create(int32_t dim, int32_t precision, void* stream, dwos_ctx** out) {
    if (!out) return fail(DWOS_EINVAL, "dwos_create: out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(DWOS_EINVAL, "dwos_create: dim must be 2 or 3");
    if (precision != DWOS_FP32 && precision != DWOS_FP64) return fail(DWOS_EINVAL, "dwos_create: bad precision");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return fail(DWOS_EDEVICE, "dwos_create: no HIP device");
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(DWOS_EDEVICE, std::string("dwos_create: device is ") + prop.gcnArchName + ", library built for gfx950");
    auto* c = new (std::nothrow) dwos_ctx();
    if (!c) return fail(DWOS_ENOMEM, "dwos_create: out of host memory");
    c->D = dim;
    c->prec = precision;
    c->variant = dim == 3 ? 1 : 0;
    c->stream = static_cast<hipStream_t>(stream);
    c->device = dev;
    c->cu_count = prop.multiProcessorCount;
    int smem = 0;
    if (hipDeviceGetAttribute(&smem, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) smem = 65536;
    c->max_smem = (size_t)smem;
    if (dwos_status rs = resolve_scratch(dev)) {
        delete c;
        return rs;
    }
    *out = c;
    return DWOS_OK;
}

dwos_status dwos_destroy(dwos_ctx* c) {
    if (!c) return DWOS_OK;
    (void)hipStreamSynchronize(c->stream);
    for (auto& pr : c->pending) { (void)hipEventDestroy(pr.e0); (void)hipEventDestroy(pr.e1); }
    delete c;
    return DWOS_OK;
}

dwos_status dwos_set_boundary(dwos_ctx* c, const double* V, int64_t nv, const int32_t* prims, int64_t np,
                              const int32_t* label, const double* gvert) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    const int D = c->D;
    if (!c->instances.empty()) return fail(DWOS_ESTATE, "set_boundary: context is a batch context");
    if (c->has_imp) return fail(DWOS_ESTATE, "set_boundary: context has an implicit boundary");
    dwos_status rc = check_geometry(D, V, nv, prims, np, label, DWOS_MAX_LABELS);
    if (rc) return rc;
    HIP_OK(hipSetDevice(c->device));
    dwos::HostBVH bvh = dwos::build_bvh(V, prims, np, D);
    if (bvh.max_depth >= dwos::kMaxDepth) return fail(DWOS_EINVAL, "set_boundary: BVH too deep");
    dwos::reorder_bfs(bvh);
    std::vector<double> Vv(V, V + nv * D);
    std::vector<int32_t> Pv(prims, prims + np * D);
    std::vector<int32_t> Lv(np, 0);
    if (label) Lv.assign(label, label + np);
    std::vector<double> Gv(nv, 0.0);
    if (gvert) Gv.assign(gvert, gvert + nv);
    rc = c->prec == DWOS_FP32 ? upload_geometry<float>(c, Vv, Pv, Lv, Gv, bvh.nodes, bvh.order)
                              : upload_geometry<double>(c, Vv, Pv, Lv, Gv, bvh.nodes, bvh.order);
    if (rc) return rc;
    c->has_boundary = true;
    c->has_params = false;   // Jacobian rows refer to the previous vertices
    return DWOS_OK;
}

dwos_status dwos_update_vertices(dwos_ctx* c, const double* Vdev) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!c->has_boundary) return fail(DWOS_ESTATE, "update_vertices: no boundary");
    if (!c->instances.empty()) return fail(DWOS_ESTATE, "update_vertices: not supported on batch contexts");
    if (!Vdev) return fail(DWOS_EINVAL, "update_vertices: NULL vertices");
    HIP_OK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int D = c->D;
    auto run = [&](auto tag) -> dwos_status {
        using T = decltype(tag);
        if (D == 2) {
            hipLaunchKernelGGL((dwos::pack_vertices_kernel<T, 2>), dim3(blocks_for(c->nv * 2, 256)), dim3(256), 0, s,
                               Vdev, c->nv, c->verts.as<T>());
            hipLaunchKernelGGL((dwos::pack_prims_kernel<T, 2>), dim3(blocks_for(c->np, 256)), dim3(256), 0, s,
                               c->verts.as<T>(), c->pverts.as<int32_t>(), c->orig.as<int32_t>(), c->np, c->prims.as<T>());
            hipLaunchKernelGGL((dwos::refit_nodes_kernel<T, 2>), dim3(blocks_for(c->n_nodes, 4)), dim3(256), 0, s,
                               c->nodes.as<T>(), c->prims.as<T>(), c->node_ranges.as<int32_t>(), c->n_nodes);
        } else {
            hipLaunchKernelGGL((dwos::pack_vertices_kernel<T, 3>), dim3(blocks_for(c->nv * 3, 256)), dim3(256), 0, s,
                               Vdev, c->nv, c->verts.as<T>());
            hipLaunchKernelGGL((dwos::pack_prims_kernel<T, 3>), dim3(blocks_for(c->np, 256)), dim3(256), 0, s,
                               c->verts.as<T>(), c->pverts.as<int32_t>(), c->orig.as<int32_t>(), c->np, c->prims.as<T>());
            hipLaunchKernelGGL((dwos::refit_nodes_kernel<T, 3>), dim3(blocks_for(c->n_nodes, 4)), dim3(256), 0, s,
                               c->nodes.as<T>(), c->prims.as<T>(), c->node_ranges.as<int32_t>(), c->n_nodes);
        }
        HIP_OK(hipGetLastError());
        return DWOS_OK;
    };
    return c->prec == DWOS_FP32 ? run(float{}) : run(double{});
}

dwos_status dwos_apply_parameters(dwos_ctx* c, const double* Vb, const double* pi) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!c->has_boundary || !c->has_params) return fail(DWOS_ESTATE, "apply_parameters: need boundary and parameters");
    if (!Vb || !pi) return fail(DWOS_EINVAL, "apply_parameters: NULL argument");
    HIP_OK(hipSetDevice(c->device));
    HIP_OK(c->vtmp.reserve(c->nv * c->D * sizeof(double)));
    if (c->D == 2)
        hipLaunchKernelGGL(dwos::apply_params_kernel<2>, dim3(blocks_for(c->nv, 256)), dim3(256), 0, c->stream, Vb,
                           c->rowptr.as<int64_t>(), c->pid.as<int32_t>(), c->vel.as<double>(), pi, c->nv,
                           c->vtmp.as<double>());
    else
        hipLaunchKernelGGL(dwos::apply_params_kernel<3>, dim3(blocks_for(c->nv, 256)), dim3(256), 0, c->stream, Vb,
                           c->rowptr.as<int64_t>(), c->pid.as<int32_t>(), c->vel.as<double>(), pi, c->nv,
                           c->vtmp.as<double>());
    HIP_OK(hipGetLastError());
    return dwos_update_vertices(c, c->vtmp.as<double>());
}

dwos_status dwos_set_problem(dwos_ctx* c, const dwos_problem* p) {
    if (!c || !p) return fail(DWOS_EINVAL, "set_problem: NULL argument");
    if (!(p->sigma >= 0) || !std::isfinite(p->sigma)) return fail(DWOS_EINVAL, "set_problem: sigma must be finite and >= 0");
    if (!(p->eps > 0) || !std::isfinite(p->eps)) return fail(DWOS_EINVAL, "set_problem: eps must be > 0");
    if (!(p->delta > 0) || !std::isfinite(p->delta)) return fail(DWOS_EINVAL, "set_problem: delta must be > 0");
    if (p->K < 1 || p->K > 255) return fail(DWOS_EINVAL, "set_problem: K must be in 1..255");
    if (p->kmax < 1) return fail(DWOS_EINVAL, "set_problem: kmax must be >= 1");
    if (p->rr != 0 && p->rr != 1) return fail(DWOS_EINVAL, "set_problem: rr must be 0 or 1");
    if (!p->rr && p->sigma > 0)
        return fail(DWOS_EINVAL, "set_problem: sigma > 0 needs Russian roulette (rr = 1): the walks do not carry "
                                 "the product of the attenuation factors");
    if (p->n_gauss < 0 || p->n_gauss > DWOS_MAX_GAUSS) return fail(DWOS_EINVAL, "set_problem: n_gauss out of range");
    if (p->n_labels < 1 || p->n_labels > DWOS_MAX_LABELS) return fail(DWOS_EINVAL, "set_problem: n_labels out of range");
    if (p->dudn != 0 && p->dudn != 1) return fail(DWOS_EINVAL, "set_problem: dudn must be 0 or 1");
    if (p->dudn == 1 && (p->sigma != 0 || p->src_c0 != 0 || p->n_gauss != 0))
        return fail(DWOS_EINVAL, "set_problem: the gradient normal-derivative estimator (dudn = 1) is for the "
                                 "Laplace equation (sigma = 0, no source)");
    if (!std::isfinite(p->src_c0)) return fail(DWOS_EINVAL, "set_problem: non-finite source");
    for (int i = 0; i < p->n_gauss; ++i) {
        for (int k = 0; k < 5; ++k)
            if (!std::isfinite(p->gauss[i][k])) return fail(DWOS_EINVAL, "set_problem: non-finite gaussian");
        if (!(p->gauss[i][4] > 0)) return fail(DWOS_EINVAL, "set_problem: gaussian width must be > 0");
    }
    for (int l = 0; l < p->n_labels; ++l) {
        if (p->bc[l].kind != 0 && p->bc[l].kind != 1) return fail(DWOS_EINVAL, "set_problem: bad boundary-data kind");
        if (!std::isfinite(p->bc[l].c)) return fail(DWOS_EINVAL, "set_problem: non-finite boundary data");
        for (int i = 0; i < 3; ++i) if (!std::isfinite(p->bc[l].b[i])) return fail(DWOS_EINVAL, "set_problem: non-finite boundary data");
        for (int i = 0; i < 9; ++i) if (!std::isfinite(p->bc[l].A[i])) return fail(DWOS_EINVAL, "set_problem: non-finite boundary data");
    }
    c->prob = *p;
    c->has_problem = true;
    return DWOS_OK;
}

}  // extern "C"

namespace {

// The parameter Jacobian of the context's (possibly combined batch) vertex
// array: validation, parameter-sorted rows, the transpose, mapped-value
// parameters and the per-primitive dependence flags.
dwos_status set_parameters_impl(dwos_ctx* c, int64_t N, const int64_t* rowptr, const int32_t* pid,
                                const double* vel, const int32_t* bc_pid) {
    if (N < 1 || N > INT32_MAX || !rowptr) return fail(DWOS_EINVAL, "set_parameters: bad N or NULL rowptr");
    const int D = c->D;
    const int64_t nv = c->nv;
    if (rowptr[0] != 0) return fail(DWOS_EINVAL, "set_parameters: rowptr[0] must be 0");
    for (int64_t i = 0; i < nv; ++i)
        if (rowptr[i + 1] < rowptr[i]) return fail(DWOS_EINVAL, "set_parameters: rowptr not monotone");
    const int64_t nnz = rowptr[nv];
    if (nnz > 0 && (!pid || !vel)) return fail(DWOS_EINVAL, "set_parameters: NULL pid/vel");
    // rows sorted by parameter id (binary search in forward mode)
    std::vector<int64_t> rp(rowptr, rowptr + nv + 1);
    std::vector<int32_t> pv(nnz);
    std::vector<double> vv(nnz * D);
    for (int64_t i = 0; i < nv; ++i) {
        std::vector<int64_t> idx;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (pid[e] < 0 || pid[e] >= N) return fail(DWOS_EINVAL, "set_parameters: pid out of range");
            for (int cc = 0; cc < D; ++cc)
                if (!std::isfinite(vel[e * D + cc])) return fail(DWOS_EINVAL, "set_parameters: non-finite velocity");
            idx.push_back(e);
        }
        std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return pid[a] < pid[b]; });
        for (size_t q = 0; q < idx.size(); ++q) {
            const int64_t e = rowptr[i] + (int64_t)q;
            if (q > 0 && pid[idx[q]] == pid[idx[q - 1]]) return fail(DWOS_EINVAL, "set_parameters: duplicate (vertex, parameter)");
            pv[e] = pid[idx[q]];
            for (int cc = 0; cc < D; ++cc) vv[e * D + cc] = vel[idx[q] * D + cc];
        }
    }
    // transpose: parameter-major
    std::vector<int64_t> cp(N + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) cp[pv[e] + 1]++;
    for (int64_t j = 0; j < N; ++j) cp[j + 1] += cp[j];
    std::vector<int32_t> cvt(nnz);
    std::vector<double> cvl(nnz * D);
    std::vector<int64_t> fillp(cp.begin(), cp.end() - 1);
    for (int64_t i = 0; i < nv; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int64_t q = fillp[pv[e]]++;
            cvt[q] = (int32_t)i;
            for (int cc = 0; cc < D; ++cc) cvl[q * D + cc] = vv[e * D + cc];
        }
    // mapped boundary values as parameters
    std::vector<int32_t> bcp(nv, -1);
    std::vector<int64_t> bp(N + 1, 0);
    std::vector<int32_t> bvt;
    bool any_bc = false;
    if (bc_pid) {
        for (int64_t i = 0; i < nv; ++i) {
            if (bc_pid[i] < -1 || bc_pid[i] >= N) return fail(DWOS_EINVAL, "set_parameters: bc_pid out of range");
            bcp[i] = bc_pid[i];
            if (bc_pid[i] >= 0) { bp[bc_pid[i] + 1]++; any_bc = true; }
        }
        for (int64_t j = 0; j < N; ++j) bp[j + 1] += bp[j];
        bvt.assign(bp[N], 0);
        std::vector<int64_t> f(bp.begin(), bp.end() - 1);
        for (int64_t i = 0; i < nv; ++i) if (bcp[i] >= 0) bvt[f[bcp[i]]++] = (int32_t)i;
    }
    HIP_OK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    HIP_OK(upload(c->rowptr, rp.data(), rp.size(), s));
    HIP_OK(upload(c->pid, pv.data(), std::max<size_t>(1, pv.size()) * (pv.empty() ? 0 : 1), s));
    HIP_OK(c->pid.reserve(4));
    HIP_OK(upload(c->vel, vv.data(), vv.size(), s));
    HIP_OK(c->vel.reserve(8));
    HIP_OK(upload(c->colptr, cp.data(), cp.size(), s));
    HIP_OK(upload(c->cvert, cvt.data(), cvt.size(), s));
    HIP_OK(c->cvert.reserve(4));
    HIP_OK(upload(c->cvel, cvl.data(), cvl.size(), s));
    HIP_OK(c->cvel.reserve(8));
    c->has_bc_params = any_bc;
    if (any_bc) {
        HIP_OK(upload(c->bc_pid, bcp.data(), bcp.size(), s));
        HIP_OK(upload(c->bcptr, bp.data(), bp.size(), s));
        HIP_OK(upload(c->bcvert, bvt.data(), bvt.size(), s));
    }
    // vertices that move or carry a parameter value: terminal points on
    // their primitives are the ones whose nested walks enter the gradient
    std::vector<int32_t> vpar(nv, 0);
    for (int64_t i = 0; i < nv; ++i) vpar[i] = (rp[i + 1] > rp[i] || bcp[i] >= 0) ? 1 : 0;
    HIP_OK(upload(c->vparam, vpar.data(), vpar.size(), s));
    HIP_OK(c->prim_dep.reserve(c->np * sizeof(int32_t)));
    hipLaunchKernelGGL(dwos::prim_dep_kernel, dim3(blocks_for(c->np, 256)), dim3(256), 0, s,
                       c->pverts.as<int32_t>(), c->vparam.as<int32_t>(), c->np, D, c->prim_dep.as<int32_t>());
    HIP_OK(hipGetLastError());
    c->N = N;
    c->has_params = true;
    return DWOS_OK;
}

}  // namespace

extern "C" {

dwos_status dwos_set_parameters(dwos_ctx* c, int64_t N, const int64_t* rowptr, const int32_t* pid,
                                const double* vel, const int32_t* bc_pid) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!c->has_boundary) return fail(DWOS_ESTATE, "set_parameters: no boundary");
    if (!c->instances.empty()) return fail(DWOS_ESTATE, "set_parameters: not supported on batch contexts");
    return set_parameters_impl(c, N, rowptr, pid, vel, bc_pid);
}

static dwos_status check_points(const double* X, int64_t P, int32_t W) {
    if (P < 0) return fail(DWOS_EINVAL, "P must be >= 0");
    if (W < 1) return fail(DWOS_EINVAL, "W must be >= 1");
    if (P > 0 && !X) return fail(DWOS_EINVAL, "NULL points");
    if (P > INT32_MAX) return fail(DWOS_EINVAL, "too many points");
    return DWOS_OK;
}

dwos_status dwos_solve(dwos_ctx* c, const double* X, int64_t P, int32_t W, uint64_t seed, double* u_mean,
                       double* u_var, dwos_stats* stats) {
    dwos_status rc = single_call(c, false);
    if (rc) return rc;
    if ((rc = check_points(X, P, W))) return rc;
    if (P > 0 && !u_mean) return fail(DWOS_EINVAL, "solve: NULL u_mean");
    if (P == 0) return finish_call(c, stats, c->pending.size());
    OpArgs o{};
    o.X = X; o.P = P; o.W = W; o.seed = seed; o.u_mean = u_mean; o.u_var = u_var;
    return dispatch(c, Op::Solve, o, stats);
}

dwos_status dwos_solve_noalloc(dwos_ctx* c, const double* X, int64_t P, int32_t W, uint64_t seed, double* u_mean,
                               double* u_var) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!c->instances.empty()) return fail(DWOS_ESTATE, "solve_noalloc: batch context");
    if (!c->has_boundary) return fail(DWOS_ESTATE, "solve_noalloc: no mesh boundary: call dwos_set_boundary first");
    if (c->has_ref || c->has_imp)
        return fail(DWOS_ESTATE, "solve_noalloc: reflecting or implicit boundaries are not supported");
    if (!c->has_problem) return fail(DWOS_ESTATE, "solve_noalloc: no problem: call dwos_set_problem first");
    if (P < 0 || W < 1) return fail(DWOS_EINVAL, "solve_noalloc: need P >= 0 and W >= 1");
    if (P > 0 && (!X || !u_mean)) return fail(DWOS_EINVAL, "solve_noalloc: NULL points or output");
    const size_t el = c->prec == DWOS_FP32 ? sizeof(float) : sizeof(double);
    if (P > (int64_t(1) << 26) || (double)P * (double)W > (double)kScratchBytes)
        return fail(DWOS_EINVAL, "solve_noalloc: P x W too large for the fixed workspace");
    const NoAllocLayout L(P, W, el);
    if (L.end > kScratchBytes)
        return fail(DWOS_EINVAL, "solve_noalloc: P x W needs " + std::to_string(L.end) + " bytes of workspace, more than the " +
                                     std::to_string(kScratchBytes) + " bytes of the fixed array");
    HIP_OK(hipSetDevice(c->device));
    auto* base = static_cast<unsigned char*>(scratch_ptr(c->device));
    if (!base) return fail(DWOS_ESTATE, "solve_noalloc: workspace address not resolved for this device");
    if (P == 0) return DWOS_OK;
    if (c->prec == DWOS_FP32)
        return c->D == 2 ? run_solve_noalloc<float, 2>(c, X, P, W, seed, u_mean, u_var, base)
                         : run_solve_noalloc<float, 3>(c, X, P, W, seed, u_mean, u_var, base);
    return c->D == 2 ? run_solve_noalloc<double, 2>(c, X, P, W, seed, u_mean, u_var, base)
                     : run_solve_noalloc<double, 3>(c, X, P, W, seed, u_mean, u_var, base);
}

dwos_status dwos_grad(dwos_ctx* c, const double* X, int64_t P, const double* w, int32_t W, uint64_t seed,
                      double* grad, double* u_mean, dwos_stats* stats) {
    dwos_status rc = single_call(c, true);
    if (rc) return rc;
    if ((rc = check_points(X, P, W))) return rc;
    if (!grad || (P > 0 && !w)) return fail(DWOS_EINVAL, "grad: NULL grad or w");
    OpArgs o{};
    o.X = X; o.P = P; o.W = W; o.seed = seed; o.w = w; o.grad = grad; o.u_mean = u_mean;
    return dispatch(c, Op::Grad, o, stats);
}

dwos_status dwos_grad_sqloss(dwos_ctx* c, const double* X, int64_t P, const double* u_ref, int32_t W, int32_t B,
                             uint64_t seed, double* loss, double* grad, double* u_mean, dwos_stats* stats) {
    dwos_status rc = single_call(c, true);
    if (rc) return rc;
    if ((rc = check_points(X, P, W))) return rc;
    if (B < 2 || W % B != 0) return fail(DWOS_EINVAL, "grad_sqloss: need B >= 2 and W % B == 0");
    if (!grad || (P > 0 && !u_ref)) return fail(DWOS_EINVAL, "grad_sqloss: NULL grad or u_ref");
    if (loss && P > 0 && !u_mean) return fail(DWOS_EINVAL, "grad_sqloss: loss needs u_mean");
    OpArgs o{};
    o.X = X; o.P = P; o.W = W; o.B = B; o.seed = seed; o.uref = u_ref; o.loss = loss; o.grad = grad;
    o.u_mean = u_mean;
    return dispatch(c, Op::SqLoss, o, stats);
}

dwos_status dwos_jvp(dwos_ctx* c, const double* X, int64_t P, int32_t W, uint64_t seed, double* udot,
                     double* udot_var, double* u_mean, dwos_stats* stats) {
    dwos_status rc = single_call(c, true);
    if (rc) return rc;
    if ((rc = check_points(X, P, W))) return rc;
    if (P > 0 && !udot) return fail(DWOS_EINVAL, "jvp: NULL udot");
    if (P * c->N > (int64_t(1) << 31)) return fail(DWOS_ENOMEM, "jvp: P*N too large");
    OpArgs o{};
    o.X = X; o.P = P; o.W = W; o.seed = seed; o.udot = udot; o.udot_var = udot_var; o.u_mean = u_mean;
    return dispatch(c, Op::Jvp, o, stats);
}

dwos_status dwos_walk_records(dwos_ctx* c, const double* X, int64_t P, int32_t W, uint64_t seed, int32_t mode,
                              double* u, int64_t* steps, int32_t* prim, double* uoff, double* udot) {
    dwos_status rc = single_call(c, mode == 1 && udot != nullptr);
    if (rc) return rc;
    if ((rc = check_points(X, P, W))) return rc;
    if (mode != 0 && mode != 1) return fail(DWOS_EINVAL, "walk_records: mode must be 0 or 1");
    if (P > 0 && !u) return fail(DWOS_EINVAL, "walk_records: NULL u");
    OpArgs o{};
    o.X = X; o.P = P; o.W = W; o.seed = seed; o.mode = mode;
    o.rec_u_out = u; o.rec_steps_out = steps; o.rec_prim_out = prim; o.rec_uoff_out = uoff; o.rec_udot_out = udot;
    return dispatch(c, Op::Records, o, nullptr);
}

dwos_status dwos_cv_attach(dwos_ctx* c, dwos_mlp* m, double q) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (m) {
        if (!(q > 0.0 && q <= 1.0)) return fail(DWOS_EINVAL, "cv_attach: q must lie in (0, 1]");
        if (m->dim != c->D) return fail(DWOS_EINVAL, "cv_attach: network dimension differs from the context");
        if (m->device != c->device) return fail(DWOS_EINVAL, "cv_attach: network on another device");
        double t = std::round(q * 16777216.0);
        if (t < 1.0) t = 1.0;
        c->cv_qthresh = (uint32_t)t;
    } else {
        c->cv_qthresh = 1u << 24;
    }
    c->cv = m;
    c->cv_nrec = 0;
    c->cv_fresh = true;
    return DWOS_OK;
}

dwos_status dwos_cv_beta(dwos_ctx* c, double* beta) {
    if (!c || !beta) return fail(DWOS_EINVAL, "cv_beta: NULL argument");
    if (!c->cv) return fail(DWOS_ESTATE, "cv_beta: no network attached");
    if (c->cv_fresh || !c->cv_beta.ptr) { *beta = 1.0; return DWOS_OK; }
    HIP_OK(hipSetDevice(c->device));
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemcpy(beta, c->cv_beta.ptr, sizeof(double), hipMemcpyDeviceToHost));
    return DWOS_OK;
}

dwos_status dwos_cv_train(dwos_ctx* c, int32_t steps, int32_t batch, float lr, uint64_t seed, float* loss) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!c->cv) return fail(DWOS_ESTATE, "cv_train: no network attached");
    if (c->cv_nrec <= 0) return fail(DWOS_ESTATE, "cv_train: no differential walks recorded since attaching");
    if (steps < 0 || batch < 1 || !(lr > 0.f)) return fail(DWOS_EINVAL, "cv_train: bad steps, batch or lr");
    HIP_OK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int D = c->D, K = c->prob.K;
    const int64_t b = batch, rows = 2 * b + 2 * b * K, nval = 2 * b + b * K;
    HIP_OK(c->cv_bx.reserve((size_t)rows * D * sizeof(float)));
    HIP_OK(c->cv_bN.reserve((size_t)rows * sizeof(float)));
    HIP_OK(c->cv_bL.reserve((size_t)b * K * sizeof(float)));
    HIP_OK(c->cv_bNbar.reserve((size_t)rows * sizeof(float)));
    HIP_OK(c->cv_bLbar.reserve((size_t)rows * sizeof(float)));
    HIP_OK(c->cv_bs.reserve((size_t)(2 * b + 2 * b * K) * sizeof(float)));
    HIP_OK(c->cv_bvalid.reserve((size_t)b * sizeof(int32_t)));
    float* su = c->cv_bs.as<float>();
    float* sg = su + b;
    float* sw = sg + b;
    float* salive = sw + b * K;
    float* X = c->cv_bx.as<float>();
    float* N = c->cv_bN.as<float>();
    for (int32_t it = 0; it < steps; ++it) {
        auto sample = [&](auto tag) {
            using T = decltype(tag);
            auto kern = D == 2 ? dwos::cv_sample_kernel<T, 2> : dwos::cv_sample_kernel<T, 3>;
            hipLaunchKernelGGL(kern, dim3(blocks_for(b, 256)), dim3(256), 0, s, c->cv_run.as<int32_t>(),
                               c->rec_prim.as<int32_t>(), c->pverts.as<int32_t>(),
                               c->has_params ? c->vparam.as<int32_t>() : nullptr, c->cv_xoff.as<T>(), c->cv_xbar.as<T>(), c->cv_g.as<T>(), c->cv_uplain.as<T>(),
                               c->cv_S.as<T>(), c->cv_alive.as<int32_t>(), c->cv_stop.as<T>(), c->cv_y.as<T>(),
                               c->cv_rho.as<T>(),
                               c->cv_d.as<T>(), c->cv_nrec, batch, K, (uint32_t)it, (uint32_t)seed,
                               (uint32_t)(seed >> 32), T(std::sqrt(c->prob.sigma)), X, su, sg, sw, salive,
                               c->cv_bvalid.as<int32_t>());
        };
        if (c->prec == DWOS_FP32) sample(float{}); else sample(double{});
        HIP_OK(hipGetLastError());
        HIP_OK(dwos_host::mlp_eval_launch<float>(c->cv, s, X, nval, nullptr, 1, 0, N, nullptr, nullptr));
        HIP_OK(dwos_host::mlp_eval_launch<float>(c->cv, s, X + nval * D, b * K, nullptr, 1, 0, N + nval,
                                                 nullptr, c->cv_bL.as<float>()));
        float* lo = (it + 1 == steps) ? loss : nullptr;
        if (lo) hipLaunchKernelGGL(dwos::fill_f32_kernel, dim3(1), dim3(64), 0, s, lo, (int64_t)1);
        hipLaunchKernelGGL(dwos::cv_adjoint_kernel, dim3(blocks_for(b, 256)), dim3(256), 0, s, N,
                           c->cv_bL.as<float>(), su, sg, sw, salive, c->cv_bvalid.as<int32_t>(), batch, K,
                           (float)c->prob.sigma, 1.0f, c->cv_bNbar.as<float>(), c->cv_bLbar.as<float>(), lo);
        HIP_OK(hipGetLastError());
        HIP_OK(dwos_host::mlp_vjp_launch(c->cv, s, X, c->cv_bNbar.as<float>(), c->cv_bLbar.as<float>(), rows));
        HIP_OK(dwos_host::mlp_adam_launch(c->cv, s, lr, 0.9f, 0.999f, 1e-8f));
    }
    return DWOS_OK;
}

dwos_status dwos_cv_walk_records(dwos_ctx* c, const double* X, int64_t P, int32_t W, uint64_t seed,
                                 double* walk, double* nested) {
    dwos_status rc = single_call(c, false);
    if (rc) return rc;
    if ((rc = check_points(X, P, W))) return rc;
    if (!c->cv) return fail(DWOS_ESTATE, "cv_walk_records: no network attached");
    if (P > 0 && (!walk || !nested)) return fail(DWOS_EINVAL, "cv_walk_records: NULL output");
    HIP_OK(c->rec_u.reserve(1));
    OpArgs o{};
    o.X = X; o.P = P; o.W = W; o.seed = seed; o.mode = 1;
    o.cv_walk_out = walk;
    o.cv_nested_out = nested;
    // the plain per-walk arrays are not exported: keep them in the context
    HIP_OK(c->export_u.reserve(std::max<int64_t>(1, P * W) * sizeof(double)));
    o.rec_u_out = c->export_u.as<double>();
    return dispatch(c, Op::Records, o, nullptr);
}

dwos_status dwos_closest(dwos_ctx* c, const double* X, int64_t P, double* out) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!c->has_boundary) return fail(DWOS_ESTATE, "closest: no boundary");
    if (!c->instances.empty()) return fail(DWOS_ESTATE, "closest: batch context");
    if (P < 0 || (P > 0 && (!X || !out))) return fail(DWOS_EINVAL, "closest: bad arguments");
    if (P == 0) return DWOS_OK;
    HIP_OK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    auto run = [&](auto tag) {
        using T = decltype(tag);
        if (c->D == 2)
            hipLaunchKernelGGL((dwos::closest_kernel<T, 2>), dim3(blocks_for(P, 64)), dim3(64), 0, s,
                               make_scene<T>(c), 0, X, P, out);
        else
            hipLaunchKernelGGL((dwos::closest_kernel<T, 3>), dim3(blocks_for(P, 64)), dim3(64), 0, s,
                               make_scene<T>(c), 0, X, P, out);
    };
    if (c->prec == DWOS_FP32) run(float{}); else run(double{});
    HIP_OK(hipGetLastError());
    return DWOS_OK;
}

dwos_status dwos_eval_ball_kernels(dwos_ctx* c, const double* r, const double* R, int64_t n, double sigma,
                                   double* GB, double* alpha) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (n < 0 || (n > 0 && (!r || !R || !GB || !alpha)) || !(sigma >= 0))
        return fail(DWOS_EINVAL, "eval_ball_kernels: bad arguments");
    if (n == 0) return DWOS_OK;
    HIP_OK(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const double kappa = std::sqrt(sigma);
    auto run = [&](auto tag) {
        using T = decltype(tag);
        if (c->D == 2)
            hipLaunchKernelGGL((dwos::ball_kernel_eval<T, 2>), dim3(blocks_for(n, 256)), dim3(256), 0, s, r, R, n,
                               T(kappa), GB, alpha);
        else
            hipLaunchKernelGGL((dwos::ball_kernel_eval<T, 3>), dim3(blocks_for(n, 256)), dim3(256), 0, s, r, R, n,
                               T(kappa), GB, alpha);
    };
    if (c->prec == DWOS_FP32) run(float{}); else run(double{});
    HIP_OK(hipGetLastError());
    return DWOS_OK;
}

dwos_status dwos_set_reflecting(dwos_ctx* c, const double* V, int64_t nv, const int32_t* segs, int64_t ns) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (ns == 0) {   // back to a Dirichlet-only problem
        c->has_ref = false;
        c->ref_n = 0;
        return DWOS_OK;
    }
    if (c->robin && ns > 65536)
        return fail(DWOS_EINVAL, "set_reflecting: a Robin condition allows at most 65536 reflecting primitives");
    if (!c->instances.empty()) return fail(DWOS_ESTATE, "set_reflecting: context is a batch context");
    if (c->has_imp) return fail(DWOS_ESTATE, "set_reflecting: context has an implicit boundary");
    dwos_status rc = check_geometry(c->D, V, nv, segs, ns, nullptr, 1);
    if (rc) return fail(rc, "set_reflecting: " + dwos_host::g_last_error.substr(std::min<size_t>(14, dwos_host::g_last_error.size())));
    if (c->D == 3) {
        HIP_OK(hipSetDevice(c->device));
        dwos::HostBVH tb = dwos::build_bvh(V, segs, ns, 3);
        if (tb.max_depth >= dwos::kMaxDepth) return fail(DWOS_EINVAL, "set_reflecting: BVH too deep");
        dwos::reorder_bfs(tb);
        rc = c->prec == DWOS_FP32 ? upload_reflecting3<float>(c, V, segs, ns, tb)
                                  : upload_reflecting3<double>(c, V, segs, ns, tb);
        if (rc) return rc;
        c->has_ref = true;
        return DWOS_OK;
    }
    std::vector<std::vector<int32_t>> inc(nv);
    for (int64_t i = 0; i < ns; ++i)
        for (int e = 0; e < 2; ++e) inc[segs[2 * i + e]].push_back((int32_t)i);
    HIP_OK(hipSetDevice(c->device));
    dwos::HostBVH bvh = dwos::build_bvh(V, segs, ns, 2);
    if (bvh.max_depth >= dwos::kMaxDepth) return fail(DWOS_EINVAL, "set_reflecting: BVH too deep");
    dwos::reorder_bfs(bvh);
    rc = c->prec == DWOS_FP32 ? upload_reflecting<float>(c, V, segs, ns, inc, bvh)
                              : upload_reflecting<double>(c, V, segs, ns, inc, bvh);
    if (rc) return rc;
    c->has_ref = true;
    return DWOS_OK;
}

dwos_status dwos_set_robin(dwos_ctx* c, double mu, const dwos_bc* h) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!(mu >= 0) || !std::isfinite(mu)) return fail(DWOS_EINVAL, "set_robin: mu must be finite and >= 0");
    double hq[13] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (h) {
        if (h->kind != 0) return fail(DWOS_EINVAL, "set_robin: the Robin data must be a restricted field (kind 0)");
        hq[0] = h->c;
        for (int i = 0; i < 3; ++i) hq[1 + i] = h->b[i];
        // A: 3 x 3 row major, the top-left D x D block used
        for (int i = 0; i < 9; ++i) hq[4 + i] = h->A[i];
        for (double v : hq)
            if (!std::isfinite(v)) return fail(DWOS_EINVAL, "set_robin: non-finite Robin data");
    }
    const bool on = mu > 0 || h != nullptr;
    if (on && !c->has_ref) return fail(DWOS_ESTATE, "set_robin: no reflecting boundary");
    if (on && c->ref_n > 65536)
        return fail(DWOS_EINVAL, "set_robin: a Robin condition allows at most 65536 reflecting primitives");
    c->robin = on;
    c->robin_mu = mu;
    for (int i = 0; i < 13; ++i) c->robin_hq[i] = hq[i];
    return DWOS_OK;
}

dwos_status dwos_set_start_segments(dwos_ctx* c, const int32_t* seg, int64_t P) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!seg || P == 0) {
        c->start_n = 0;
        return DWOS_OK;
    }
    if (P < 0) return fail(DWOS_EINVAL, "set_start_segments: negative count");
    if (!c->has_ref) return fail(DWOS_ESTATE, "set_start_segments: no reflecting boundary");
    for (int64_t p = 0; p < P; ++p)
        if (seg[p] < -1 || seg[p] >= c->ref_n)
            return fail(DWOS_EINVAL, "set_start_segments: segment index out of range at point " + std::to_string(p));
    HIP_OK(hipSetDevice(c->device));
    HIP_OK(upload(c->start_seg, seg, (size_t)P, c->stream));
    c->start_n = P;
    return DWOS_OK;
}

dwos_status dwos_reflect_query(dwos_ctx* c, const double* X, const double* dir, const double* cap,
                               const int32_t* on, const double* nin, int64_t n, double* out) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!c->has_ref) return fail(DWOS_ESTATE, "reflect_query: no reflecting boundary");
    if (n < 0 || (n > 0 && (!X || !dir || !cap || !on || !nin || !out)))
        return fail(DWOS_EINVAL, "reflect_query: bad arguments");
    if (n == 0) return DWOS_OK;
    HIP_OK(hipSetDevice(c->device));
    auto run = [&](auto tag) {
        using T = decltype(tag);
        if (c->D == 3)
            hipLaunchKernelGGL(dwos::ref3_query_kernel<T>, dim3(blocks_for(n, 64)), dim3(64), 0, c->stream,
                               make_ref3<T>(c), X, dir, cap, on, nin, n, out);
        else
            hipLaunchKernelGGL(dwos::ref_query_kernel<T>, dim3(blocks_for(n, 64)), dim3(64), 0, c->stream,
                               make_ref<T>(c), X, dir, cap, on, nin, n, out);
    };
    if (c->prec == DWOS_FP32) run(float{}); else run(double{});
    HIP_OK(hipGetLastError());
    return DWOS_OK;
}

dwos_status dwos_eval_reflect_weight(dwos_ctx* c, const double* r, const double* R, int64_t n, double sigma,
                                     double* w) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (n < 0 || (n > 0 && (!r || !R || !w)) || !(sigma >= 0))
        return fail(DWOS_EINVAL, "eval_reflect_weight: bad arguments");
    if (n == 0) return DWOS_OK;
    HIP_OK(hipSetDevice(c->device));
    const double kappa = std::sqrt(sigma);
    auto run = [&](auto tag) {
        using T = decltype(tag);
        if (c->D == 2)
            hipLaunchKernelGGL((dwos::reflect_weight_eval<T, 2>), dim3(blocks_for(n, 256)), dim3(256), 0, c->stream,
                               r, R, n, T(kappa), w);
        else
            hipLaunchKernelGGL((dwos::reflect_weight_eval<T, 3>), dim3(blocks_for(n, 256)), dim3(256), 0, c->stream,
                               r, R, n, T(kappa), w);
    };
    if (c->prec == DWOS_FP32) run(float{}); else run(double{});
    HIP_OK(hipGetLastError());
    return DWOS_OK;
}

dwos_status dwos_set_implicit(dwos_ctx* c, const double* mono, int64_t n, double cconst) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (n == 0) {   // back to no boundary
        c->has_imp = false;
        c->imp_n = 0;
        c->N = 0;
        return DWOS_OK;
    }
    if (c->D != 2) return fail(DWOS_EINVAL, "set_implicit: implicit boundaries are supported in 2D only");
    if (n < 0 || n > dwos::kMaxMono) return fail(DWOS_EINVAL, "set_implicit: n must be in 0..1024");
    if (!mono) return fail(DWOS_EINVAL, "set_implicit: NULL monopoles");
    if (!(cconst < 0) || !std::isfinite(cconst)) return fail(DWOS_EINVAL, "set_implicit: c must be finite and < 0");
    for (int64_t i = 0; i < n; ++i) {
        if (!(mono[3 * i] > 0) || !std::isfinite(mono[3 * i]))
            return fail(DWOS_EINVAL, "set_implicit: scale a_" + std::to_string(i) + " must be finite and > 0");
        if (!std::isfinite(mono[3 * i + 1]) || !std::isfinite(mono[3 * i + 2]))
            return fail(DWOS_EINVAL, "set_implicit: non-finite position of monopole " + std::to_string(i));
    }
    if (c->has_boundary) return fail(DWOS_ESTATE, "set_implicit: context has a mesh boundary");
    if (c->has_ref) return fail(DWOS_ESTATE, "set_implicit: context has a reflecting boundary");
    if (c->cv) return fail(DWOS_ESTATE, "set_implicit: a control variate is attached");
    if (!c->instances.empty()) return fail(DWOS_ESTATE, "set_implicit: context is a batch context");
    HIP_OK(hipSetDevice(c->device));
    if (c->prec == DWOS_FP32) {
        std::vector<float> h(mono, mono + 3 * n);
        HIP_OK(upload(c->imp_mono, h.data(), h.size(), c->stream));
    } else {
        HIP_OK(upload(c->imp_mono, mono, (size_t)(3 * n), c->stream));
    }
    c->has_imp = true;
    c->imp_n = n;
    c->imp_c = cconst;
    c->N = 3 * n;
    return DWOS_OK;
}

dwos_status dwos_implicit_band_grad(dwos_ctx* c, const double* X, int64_t P, const double* coef, double eps_band,
                                    double* grad, int32_t* region) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!c->has_imp) return fail(DWOS_ESTATE, "implicit_band_grad: no implicit boundary");
    if (P < 0 || (P > 0 && (!X || !coef)) || !grad) return fail(DWOS_EINVAL, "implicit_band_grad: bad arguments");
    if (!(eps_band > 0) || !std::isfinite(eps_band)) return fail(DWOS_EINVAL, "implicit_band_grad: eps_band must be > 0");
    if (P == 0) return DWOS_OK;
    HIP_OK(hipSetDevice(c->device));
    auto run = [&](auto tag) -> dwos_status {
        using T = decltype(tag);
        HIP_OK(c->imp_bx.reserve(P * 2 * sizeof(T)));
        HIP_OK(c->imp_bs.reserve(P * sizeof(T)));
        HIP_OK(c->imp_coef.reserve(P * sizeof(double)));
        hipLaunchKernelGGL(dwos::imp_band_kernel<T>, dim3(blocks_for(P, 256)), dim3(256), 0, c->stream, X, P, coef,
                           c->imp_mono.as<T>(), (int32_t)c->imp_n, T(c->imp_c), T(eps_band), c->imp_bx.as<T>(),
                           c->imp_bs.as<T>(), c->imp_coef.as<double>(), region);
        hipLaunchKernelGGL(dwos::imp_grad_kernel<T>, dim3(blocks_for(P, dwos::kImpTile)), dim3(256), 0, c->stream,
                           c->imp_bx.as<T>(), c->imp_bs.as<T>(), c->imp_coef.as<double>(), P, c->imp_mono.as<T>(),
                           (int32_t)c->imp_n, grad);
        return DWOS_OK;
    };
    dwos_status rc = c->prec == DWOS_FP32 ? run(float{}) : run(double{});
    if (rc) return rc;
    HIP_OK(hipGetLastError());
    return DWOS_OK;
}

dwos_status dwos_scene_info(dwos_ctx* c, int64_t* info) {
    if (!c || !info) return fail(DWOS_EINVAL, "scene_info: NULL argument");
    if (!c->has_boundary) return fail(DWOS_ESTATE, "scene_info: no mesh boundary");
    const size_t el = c->prec == DWOS_FP32 ? sizeof(float) : sizeof(double);
    const int64_t nb = dwos::node_scalars(c->D) * (int64_t)el, pb = dwos::prim_scalars(c->D) * (int64_t)el;
    int64_t stage_nodes = 0, stage_prims = 0, lds = 0;
    if (c->prec == DWOS_FP32) {
        const dwos::Scene<float> sc = make_scene<float>(c);
        stage_nodes = sc.n_stage_nodes;
        stage_prims = sc.stage_prims;
        lds = (int64_t)stage_bytes<float>(sc, c->D);
    }
    info[0] = c->n_nodes;
    info[1] = c->n_nodes * nb;
    info[2] = c->np * pb;
    info[3] = stage_nodes;
    info[4] = stage_prims;
    info[5] = c->np;
    info[6] = c->nv;
    info[7] = lds;
    return DWOS_OK;
}

dwos_status dwos_set_variant(dwos_ctx* c, int32_t variant) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (variant != 0 && variant != 1) return fail(DWOS_EINVAL, "set_variant: variant must be 0 or 1");
    c->variant = variant;
    return DWOS_OK;
}

dwos_status dwos_set_tuning(dwos_ctx* c, const dwos_tuning* t) {
    if (!c || !t) return fail(DWOS_EINVAL, "set_tuning: NULL argument");
    if (t->variant != 0 && t->variant != 1) return fail(DWOS_EINVAL, "set_tuning: variant must be 0 or 1");
    if (t->park < 1 || t->park > 64) return fail(DWOS_EINVAL, "set_tuning: park must be in 1..64");
    if (t->tail < 0 || t->tail > 63) return fail(DWOS_EINVAL, "set_tuning: tail must be in 0..63");
    if (t->chunk < 64 || t->chunk > 65536 || t->chunk % 64 != 0)
        return fail(DWOS_EINVAL, "set_tuning: chunk must be a multiple of 64 in 64..65536");
    if (t->stage_nodes < -1) return fail(DWOS_EINVAL, "set_tuning: stage_nodes must be -1 or >= 0");
    c->variant = t->variant;
    c->park = t->park;
    c->tail = t->tail;
    c->chunk = t->chunk;
    c->stage_cap = t->stage_nodes;
    return DWOS_OK;
}

dwos_status dwos_get_tuning(dwos_ctx* c, dwos_tuning* t) {
    if (!c || !t) return fail(DWOS_EINVAL, "get_tuning: NULL argument");
    t->variant = c->variant;
    t->park = c->park;
    t->tail = c->tail;
    t->chunk = c->chunk;
    t->stage_nodes = c->stage_cap;
    return DWOS_OK;
}

}  // extern "C"

namespace {

// Process-wide autotuner results, keyed by device, dimension, precision,
// batch or single scene and the scene's size in half-octaves of primitives.
struct TuneKey {
    int device, D, prec, batch, bucket, grad;
    bool operator<(const TuneKey& o) const {
        return std::tie(device, D, prec, batch, bucket, grad) <
               std::tie(o.device, o.D, o.prec, o.batch, o.bucket, o.grad);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, dwos_tuning> g_tune_cache;

TuneKey tune_key(const dwos_ctx* c, bool grad) {
    const int64_t np = c->instances.empty() ? c->np : (int64_t)c->hostOrder.size();
    const int bucket = np > 0 ? (int)std::floor(2.0 * std::log2((double)np)) : 0;
    return {c->device, c->D, c->prec, c->instances.empty() ? 0 : 1, bucket, grad ? 1 : 0};
}

}  // namespace

extern "C" {

dwos_status dwos_autotune(dwos_ctx* c, const double* X, const int64_t* P, int32_t W, uint64_t seed, int32_t flags,
                          dwos_tuning* chosen, double* ms) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (!P || W < 1 || !X) return fail(DWOS_EINVAL, "autotune: need points, point counts and W >= 1");
    if (flags & ~(DWOS_TUNE_CACHE | DWOS_TUNE_GRAD)) return fail(DWOS_EINVAL, "autotune: unknown flags");
    const bool batch = !c->instances.empty();
    const bool with_grad = (flags & DWOS_TUNE_GRAD) != 0;
    if (!batch && !c->has_boundary) return fail(DWOS_ESTATE, "autotune: no mesh boundary");
    if (!c->has_problem) return fail(DWOS_ESTATE, "autotune: no problem: call dwos_set_problem first");
    // the timed call: a forward solve of the whole batch, or of a prefix of
    // the points with about 2^22 walks
    int64_t pts = 0;
    if (batch) {
        for (size_t i = 0; i < c->instances.size(); ++i) {
            if (P[i] < 0 || P[i] > INT32_MAX) return fail(DWOS_EINVAL, "autotune: bad point count");
            pts += P[i];
        }
    } else {
        if (P[0] <= 0) return fail(DWOS_EINVAL, "autotune: need points");
        pts = std::min<int64_t>(P[0], std::max<int64_t>(64, ((int64_t)1 << 22) / W));
    }
    if (pts <= 0) return fail(DWOS_EINVAL, "autotune: need points");
    int64_t Ntot = 0;
    if (with_grad) {
        if (batch) {
            for (const auto& bp : c->batch_params) Ntot += bp.N;
        } else if (c->has_params) {
            Ntot = c->N;
        }
        if (Ntot < 1) return fail(DWOS_ESTATE, "autotune: DWOS_TUNE_GRAD needs parameters");
    }
    dwos_tuning cur{};
    dwos_get_tuning(c, &cur);
    const TuneKey key = tune_key(c, with_grad);
    if (flags & DWOS_TUNE_CACHE) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            dwos_status rc = dwos_set_tuning(c, &it->second);
            if (rc) return rc;
            if (chosen) *chosen = it->second;
            if (ms) { ms[0] = -1.0; ms[1] = -1.0; }
            return DWOS_OK;
        }
    }
    DevBuf mean, wone, gout;
    HIP_OK(mean.reserve(pts * sizeof(double)));
    if (with_grad) {
        const std::vector<double> ones((size_t)pts, 1.0);
        HIP_OK(upload(wone, ones.data(), ones.size(), c->stream));
        HIP_OK(gout.reserve(Ntot * sizeof(double)));
    }
    std::vector<int64_t> Pb(P, P + (batch ? c->instances.size() : 1));
    if (!batch) Pb[0] = pts;
    // the timed call: a forward solve, and with DWOS_TUNE_GRAD a reverse-mode
    // call with unit weights on the same points; *ms (if given) gets the sum
    // of their walk-kernel times
    auto run = [&](uint64_t sd, double* ms_out) -> dwos_status {
        dwos_stats st{}, st2{};
        dwos_stats* ps = ms_out ? &st : nullptr;
        dwos_status r = batch ? dwos_batch_solve(c, X, Pb.data(), W, sd, mean.as<double>(), nullptr, ps)
                              : dwos_solve(c, X, pts, W, sd, mean.as<double>(), nullptr, ps);
        if (r) return r;
        if (with_grad) {
            dwos_stats* ps2 = ms_out ? &st2 : nullptr;
            r = batch ? dwos_batch_grad(c, X, Pb.data(), wone.as<double>(), W, sd + 1, gout.as<double>(), nullptr, ps2)
                      : dwos_grad(c, X, pts, wone.as<double>(), W, sd + 1, gout.as<double>(), nullptr, ps2);
            if (r) return r;
        }
        if (ms_out) *ms_out = st.walk_ms + st2.walk_ms;
        return DWOS_OK;
    };
    // every candidate runs the same walks (same seed); the better of two
    // timings of the walk kernel(s) scores it
    auto score = [&](const dwos_tuning& t, double& out) -> dwos_status {
        dwos_status rc = dwos_set_tuning(c, &t);
        if (rc) return rc;
        double best = 0.0;
        for (int r = 0; r < 2; ++r) {
            double ms_r = 0.0;
            rc = run(seed, &ms_r);
            if (rc) return rc;
            if (r == 0 || ms_r < best) best = ms_r;
        }
        out = best;
        return DWOS_OK;
    };
    dwos_status rc = run(seed, nullptr);   // warm-up: workspaces, uploads
    double t_best = 0.0;
    if (!rc) rc = score(cur, t_best);
    const double t_start = t_best;
    dwos_tuning best = cur;
    // coordinate descent, one pass; a change must win by more than 1%
    auto try_dim = [&](int32_t dwos_tuning::*field, std::initializer_list<int32_t> vals) -> dwos_status {
        const int32_t keep = best.*field;
        for (int32_t v : vals) {
            if (v == keep) continue;
            dwos_tuning t = best;
            t.*field = v;
            double tv = 0.0;
            dwos_status r2 = score(t, tv);
            if (r2) return r2;
            if (tv < 0.99 * t_best) { t_best = tv; best = t; }
        }
        return DWOS_OK;
    };
    if (!rc && c->prec == DWOS_FP32) rc = try_dim(&dwos_tuning::variant, {0, 1});
    if (!rc) rc = try_dim(&dwos_tuning::park, {16, 24, 32, 40});
    if (!rc) rc = try_dim(&dwos_tuning::tail, {0, 4, 8, 16});
    if (!rc) rc = try_dim(&dwos_tuning::chunk, {64, 128, 256, 512});
    if (!rc && c->prec == DWOS_FP32 && best.variant == 0 && !batch) {
        const int32_t staged = c->prec == DWOS_FP32 ? make_scene<float>(c).n_stage_nodes : 0;
        if (staged > 4) rc = try_dim(&dwos_tuning::stage_nodes, {-1, staged / 2, staged / 4, 0});
    }
    if (rc) {
        dwos_set_tuning(c, &cur);
        return rc;
    }
    dwos_set_tuning(c, &best);
    HIP_OK(hipStreamSynchronize(c->stream));
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = best;
    }
    if (chosen) *chosen = best;
    if (ms) { ms[0] = t_start; ms[1] = t_best; }
    return DWOS_OK;
}

dwos_status dwos_set_seed_buffer(dwos_ctx* c, const uint64_t* seed_dev) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    c->seed_dev = seed_dev;
    return DWOS_OK;
}

dwos_status dwos_adjoint_grad(dwos_ctx* c, const int32_t* code, const double* bary, const double* wq, int64_t S,
                              const dwos_quad* uref, int32_t W, uint64_t seed, double* grad, double* rec_lambda,
                              double* rec_uoff, dwos_stats* stats) {
    dwos_status rc = single_call(c, true);
    if (rc) return rc;
    if (c->has_imp) return fail(DWOS_ESTATE, "adjoint_grad: needs a mesh boundary, not an implicit one");
    if (c->has_ref) return fail(DWOS_ESTATE, "adjoint_grad: reflecting boundaries are not supported");
    if (c->cv) return fail(DWOS_ESTATE, "adjoint_grad: detach the control variate first");
    if (c->prob.dudn != 0) return fail(DWOS_ESTATE, "adjoint_grad: needs the backward-difference du/dn (dudn = 0)");
    if (S < 0 || W < 1) return fail(DWOS_EINVAL, "adjoint_grad: need S >= 0 and W >= 1");
    if (!grad || !uref || (S > 0 && (!code || !bary || !wq)))
        return fail(DWOS_EINVAL, "adjoint_grad: NULL argument");
    if (S > INT32_MAX || S * (int64_t)W > (int64_t(1) << 30))
        return fail(DWOS_EINVAL, "adjoint_grad: more than 2^30 walks");
    if (S > 0) {   // every code must name a primitive
        std::vector<int32_t> h((size_t)S);
        HIP_OK(hipMemcpyAsync(h.data(), code, S * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < S; ++i)
            if (h[i] < 0 || (int64_t)(h[i] >> 1) >= c->np)
                return fail(DWOS_EINVAL, "adjoint_grad: code " + std::to_string(i) + " names no primitive");
    }
    if (c->prec == DWOS_FP32)
        return c->D == 2 ? run_adjoint<float, 2>(c, code, bary, wq, S, uref, W, seed, grad, rec_lambda, rec_uoff, stats)
                         : run_adjoint<float, 3>(c, code, bary, wq, S, uref, W, seed, grad, rec_lambda, rec_uoff, stats);
    return c->D == 2 ? run_adjoint<double, 2>(c, code, bary, wq, S, uref, W, seed, grad, rec_lambda, rec_uoff, stats)
                     : run_adjoint<double, 3>(c, code, bary, wq, S, uref, W, seed, grad, rec_lambda, rec_uoff, stats);
}

dwos_status dwos_walk_timing(dwos_ctx* c, int32_t kind, int32_t reset, double* walk_ms, int64_t* launches,
                             dwos_stats* totals) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (kind < 0 || kind > 2) return fail(DWOS_EINVAL, "walk_timing: kind must be 0, 1 or 2");
    HIP_OK(hipSetDevice(c->device));
    dwos_status rc = drain_events(c, nullptr, 0);
    if (rc) return rc;
    if (walk_ms) *walk_ms = c->timed_ms[kind];
    if (launches) *launches = c->timed_launches[kind];
    if ((rc = ensure_totals(c))) return rc;
    HIP_OK(hipStreamSynchronize(c->stream));
    dwos::Counters h{};
    HIP_OK(hipMemcpy(&h, c->totals.as<dwos::Counters>() + kind, sizeof(h), hipMemcpyDeviceToHost));
    if (totals) {
        totals->walks = (int64_t)h.walks;
        totals->nested_walks = (int64_t)h.nested;
        totals->steps = (int64_t)h.steps;
        totals->terminal = (int64_t)h.terminal;
        totals->truncated = (int64_t)h.truncated;
        totals->nodes = (int64_t)h.nodes;
        totals->prims = (int64_t)h.prims;
        totals->stack_overflow = (int64_t)h.overflow;
        totals->invalid = (int64_t)h.invalid;
        totals->walk_ms = c->timed_ms[kind];
    }
    if (reset) {
        c->timed_ms[kind] = 0.0;
        c->timed_launches[kind] = 0;
        hipLaunchKernelGGL(dwos::fill_u64_kernel, dim3(1), dim3(64), 0, c->stream,
                           reinterpret_cast<unsigned long long*>(c->totals.as<dwos::Counters>() + kind),
                           (int64_t)(sizeof(dwos::Counters) / 8));
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    return DWOS_OK;
}

dwos_status dwos_batch_add_instance(dwos_ctx* c, const double* V, int64_t nv, const int32_t* prims, int64_t np,
                                    const int32_t* label, double sigma, double eps, double delta, int32_t* index) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (c->has_ref) return fail(DWOS_ESTATE, "batch_add_instance: context has a reflecting boundary");
    if (c->has_imp) return fail(DWOS_ESTATE, "batch_add_instance: context has an implicit boundary");
    const int D = c->D;
    dwos_status rc = check_geometry(D, V, nv, prims, np, label, DWOS_MAX_LABELS);
    if (rc) return rc;
    if (!(sigma >= 0) || !std::isfinite(sigma) || !(eps > 0) || !(delta > 0) || !std::isfinite(eps) ||
        !std::isfinite(delta))
        return fail(DWOS_EINVAL, "batch_add_instance: need sigma >= 0, eps > 0, delta > 0");
    if (c->has_boundary && c->instances.empty())
        return fail(DWOS_ESTATE, "batch_add_instance: context already holds a single boundary");
    if (c->instances.size() >= 65535) return fail(DWOS_EINVAL, "batch_add_instance: too many instances");
    const int64_t nv_off = (int64_t)c->hostV.size() / D, np_off = (int64_t)c->hostOrder.size();
    if (nv_off + nv > INT32_MAX || (np_off + np) > (int64_t(1) << 27))
        return fail(DWOS_EINVAL, "batch_add_instance: batch too large");
    dwos::HostBVH bvh = dwos::build_bvh(V, prims, np, D);
    if (bvh.max_depth >= dwos::kMaxDepth) return fail(DWOS_EINVAL, "batch_add_instance: BVH too deep");
    dwos::reorder_bfs(bvh);
    const int32_t node_off = (int32_t)c->hostNodes.size();
    for (auto nd : bvh.nodes) {
        for (int k = 0; k < 2; ++k) {
            if (nd.child[k] >= 0) {
                nd.child[k] += node_off;
            } else {
                const int32_t v = -1 - nd.child[k];
                nd.child[k] = dwos::leaf_ref((v >> 3) + (int32_t)np_off, (v & 7) + 1);
            }
            nd.range[k][0] += (int32_t)np_off;
            nd.range[k][1] += (int32_t)np_off;
        }
        c->hostNodes.push_back(nd);
    }
    for (int64_t i = 0; i < np; ++i) c->hostOrder.push_back(bvh.order[i] + (int32_t)np_off);
    for (int64_t i = 0; i < np * D; ++i) c->hostP.push_back(prims[i] + (int32_t)nv_off);
    for (int64_t i = 0; i < np; ++i) c->hostL.push_back(label ? label[i] : 0);
    c->hostV.insert(c->hostV.end(), V, V + nv * D);
    c->hostG.resize(c->hostV.size() / D, 0.0);
    c->instances.push_back({node_off, nv_off, np_off, sigma, eps, delta});
    c->batch_params.emplace_back();
    c->batch_params_dirty = true;
    c->batch_dirty = true;
    c->has_params = false;
    if (index) *index = (int32_t)c->instances.size() - 1;
    return DWOS_OK;
}

}  // extern "C"

namespace {

// A screened instance (sigma > 0) needs Russian roulette: the walks do not
// carry the product of the attenuation factors (Sec. 3.3).  The problem's rr
// flag is shared by every instance of a batch, while sigma is per instance.
dwos_status check_batch_roulette(const dwos_ctx* c, const char* who) {
    if (c->prob.rr) return DWOS_OK;
    for (size_t i = 0; i < c->instances.size(); ++i)
        if (c->instances[i].sigma > 0)
            return fail(DWOS_EINVAL, std::string(who) + ": instance " + std::to_string(i) +
                                         " has sigma > 0, which needs Russian roulette (rr = 1)");
    return DWOS_OK;
}

template <class T, int D>
dwos_status run_batch(dwos_ctx* c, const double* X, const int64_t* P, int32_t W, uint64_t seed, double* u_mean,
                      double* u_var, dwos_stats* st) {
    hipStream_t s = c->stream;
    const int n = (int)c->instances.size();
    std::vector<dwos::Instance<T>> tab(n);
    int64_t walks = 0, pts = 0;
    for (int i = 0; i < n; ++i) {
        tab[i].walk_begin = walks;
        tab[i].point_begin = pts;
        tab[i].p_counter = 0;
        tab[i].root = c->instances[i].root;
        tab[i].P = (int32_t)P[i];
        tab[i].kappa = T(std::sqrt(c->instances[i].sigma));
        tab[i].eps = T(c->instances[i].eps);
        tab[i].delta = T(c->instances[i].delta);
        walks += P[i] * W;
        pts += P[i];
    }
    if (walks > (int64_t(1) << 28)) return fail(DWOS_ENOMEM, "batch_solve: more than 2^28 walks in one batch");
    dwos_status rc = ensure_records<T>(c, std::max<int64_t>(1, walks), false, false);
    if (rc) return rc;
    rc = upload_instances<T>(c, tab.data(), tab.size());
    if (rc) return rc;
    const size_t ev_from = c->pending.size();
    const dwos::Scene<T> scene = make_scene<T>(c);
    HIP_OK(c->first_leaf.reserve(std::max<int64_t>(1, pts) * sizeof(int32_t)));
    HIP_OK(c->first_d2.reserve(std::max<int64_t>(1, pts) * sizeof(T)));
    c->first_warm = false;   // batch leaves are positions in the instances' trees
    hipLaunchKernelGGL((dwos::first_query_kernel<T, D>), dim3(blocks_for(pts, 64)), dim3(64), 0, s, scene,
                       c->instbuf.as<dwos::Instance<T>>(), n, X, (int64_t)0, pts, c->inst_prange.as<int32_t>(),
                       c->first_leaf.as<int32_t>(), c->first_leaf.as<int32_t>(), c->first_d2.as<T>());
    dwos::WalkArgs<T> a = base_args<T>(c, X, W, seed);
    a.inst = c->instbuf.as<dwos::Instance<T>>();
    a.n_inst = n;
    a.total = walks;
    a.wid_offset = 0;
    a.first_leaf = c->first_leaf.as<int32_t>();
    a.first_d2 = c->first_d2.as<T>();
    a.x_base = 0;
    rc = launch_walks<T, D, 0>(c, a);
    if (rc) return rc;
    hipLaunchKernelGGL(dwos::point_stats_kernel<T>, dim3(blocks_for(pts, 4)), dim3(256), 0, s, c->rec_u.as<T>(),
                       pts, W, u_mean, u_var);
    return finish_call(c, st, ev_from);
}

// Reverse mode over every instance in one persistent launch: the
// differential walks with their instance constants, the per-vertex
// scatter over the batch's vertex array and the SpMV with the combined
// Jacobian (instance i's parameters after those of instances < i).
template <class T, int D>
dwos_status run_batch_grad(dwos_ctx* c, const double* X, const int64_t* P, const double* w, int32_t W,
                           uint64_t seed, double* grad, double* u_mean, dwos_stats* st) {
    hipStream_t s = c->stream;
    const int n = (int)c->instances.size();
    std::vector<dwos::Instance<T>> tab(n);
    int64_t walks = 0, pts = 0;
    for (int i = 0; i < n; ++i) {
        tab[i].walk_begin = walks;
        tab[i].point_begin = pts;
        tab[i].p_counter = 0;
        tab[i].root = c->instances[i].root;
        tab[i].P = (int32_t)P[i];
        tab[i].kappa = T(std::sqrt(c->instances[i].sigma));
        tab[i].eps = T(c->instances[i].eps);
        tab[i].delta = T(c->instances[i].delta);
        walks += P[i] * W;
        pts += P[i];
    }
    if (walks > (int64_t(1) << 28)) return fail(DWOS_ENOMEM, "batch_grad: more than 2^28 walks in one batch");
    dwos_status rc = ensure_records<T>(c, std::max<int64_t>(1, walks), true, false);
    if (rc) return rc;
    rc = upload_instances<T>(c, tab.data(), tab.size());
    if (rc) return rc;
    const size_t ev_from = c->pending.size();
    const dwos::Scene<T> scene = make_scene<T>(c);
    HIP_OK(c->accA.reserve(c->nv * D * sizeof(double)));
    HIP_OK(c->accB.reserve(c->nv * sizeof(double)));
    hipLaunchKernelGGL(dwos::fill_f64_kernel, dim3(blocks_for(c->nv * D, 256)), dim3(256), 0, s,
                       c->accA.as<double>(), c->nv * D);
    hipLaunchKernelGGL(dwos::fill_f64_kernel, dim3(blocks_for(c->nv, 256)), dim3(256), 0, s,
                       c->accB.as<double>(), c->nv);
    if (pts > 0) {
        HIP_OK(c->first_leaf.reserve(pts * sizeof(int32_t)));
        HIP_OK(c->first_d2.reserve(pts * sizeof(T)));
        c->first_warm = false;   // batch leaves are positions in the instances' trees
        hipLaunchKernelGGL((dwos::first_query_kernel<T, D>), dim3(blocks_for(pts, 64)), dim3(64), 0, s, scene,
                           c->instbuf.as<dwos::Instance<T>>(), n, X, (int64_t)0, pts,
                           c->inst_prange.as<int32_t>(), c->first_leaf.as<int32_t>(), c->first_leaf.as<int32_t>(),
                           c->first_d2.as<T>());
        dwos::WalkArgs<T> a = base_args<T>(c, X, W, seed);
        a.inst = c->instbuf.as<dwos::Instance<T>>();
        a.n_inst = n;
        a.total = walks;
        a.wid_offset = 0;
        a.first_leaf = c->first_leaf.as<int32_t>();
        a.first_d2 = c->first_d2.as<T>();
        a.x_base = 0;
        rc = launch_walks<T, D, 1>(c, a);
        if (rc) return rc;
        if (u_mean)
            hipLaunchKernelGGL(dwos::point_stats_kernel<T>, dim3(blocks_for(pts, 4)), dim3(256), 0, s,
                               c->rec_u.as<T>(), pts, W, u_mean, nullptr);
        dwos::AccArgs<T> aa{};
        aa.s = scene;
        aa.prm = make_params<T>(c->prob);
        aa.delta = T(c->instances[0].delta);   // one delta for the batch (checked by the caller)
        aa.rec_u = c->rec_u.as<T>();
        aa.rec_prim = c->rec_prim.as<int32_t>();
        aa.rec_b = c->rec_b.as<T>();
        aa.rec_uoff = c->rec_uoff.as<T>();
        aa.nwalks = walks;
        aa.p_offset = 0;
        aa.W = W;
        aa.B = 1;
        aa.mode = 0;
        aa.w = w;
        aa.uref = nullptr;
        aa.bc_pid = nullptr;
        aa.prim_dep = c->prim_dep.as<int32_t>();
        aa.vparam = c->vparam.as<int32_t>();
        aa.A = c->accA.as<double>();
        aa.Bacc = c->accB.as<double>();
        hipLaunchKernelGGL((dwos::accumulate_kernel<T, D>), dim3(blocks_for(walks, 256)), dim3(256), 0, s, aa);
    }
    hipLaunchKernelGGL(dwos::spmv_kernel<D>, dim3(blocks_for(c->N, 4)), dim3(256), 0, s, make_csr(c),
                       c->accA.as<double>(), c->accB.as<double>(), grad);
    return finish_call(c, st, ev_from);
}

}  // namespace

extern "C" {

dwos_status dwos_batch_set_parameters(dwos_ctx* c, int32_t index, int64_t N, const int64_t* rowptr,
                                     const int32_t* pid, const double* vel) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (index < 0 || index >= (int32_t)c->instances.size())
        return fail(DWOS_EINVAL, "batch_set_parameters: no instance " + std::to_string(index));
    const int D = c->D;
    const int64_t nv0 = c->instances[index].nv_off;
    const int64_t nv1 = index + 1 < (int32_t)c->instances.size() ? c->instances[index + 1].nv_off
                                                                 : (int64_t)c->hostV.size() / D;
    const int64_t nv = nv1 - nv0;
    if (N < 0 || N > INT32_MAX) return fail(DWOS_EINVAL, "batch_set_parameters: bad N");
    dwos_ctx::BatchParams bp;
    bp.N = N;
    if (N > 0) {
        if (!rowptr) return fail(DWOS_EINVAL, "batch_set_parameters: NULL rowptr");
        if (rowptr[0] != 0) return fail(DWOS_EINVAL, "batch_set_parameters: rowptr[0] must be 0");
        for (int64_t i = 0; i < nv; ++i)
            if (rowptr[i + 1] < rowptr[i]) return fail(DWOS_EINVAL, "batch_set_parameters: rowptr not monotone");
        const int64_t nnz = rowptr[nv];
        if (nnz > 0 && (!pid || !vel)) return fail(DWOS_EINVAL, "batch_set_parameters: NULL pid/vel");
        for (int64_t e = 0; e < nnz; ++e) {
            if (pid[e] < 0 || pid[e] >= N) return fail(DWOS_EINVAL, "batch_set_parameters: pid out of range");
            for (int k = 0; k < D; ++k)
                if (!std::isfinite(vel[e * D + k])) return fail(DWOS_EINVAL, "batch_set_parameters: non-finite velocity");
        }
        bp.rowptr.assign(rowptr, rowptr + nv + 1);
        bp.pid.assign(pid, pid + nnz);
        bp.vel.assign(vel, vel + nnz * D);
    }
    c->batch_params[index] = std::move(bp);
    c->batch_params_dirty = true;
    return DWOS_OK;
}

dwos_status dwos_batch_grad(dwos_ctx* c, const double* X_all, const int64_t* P, const double* w, int32_t W,
                            uint64_t seed, double* grad, double* u_mean, dwos_stats* stats) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (c->instances.empty()) return fail(DWOS_ESTATE, "batch_grad: no instances");
    if (!c->has_problem) return fail(DWOS_ESTATE, "batch_grad: no problem: call dwos_set_problem first");
    if (c->cv) return fail(DWOS_ESTATE, "batch_grad: the control variate is not supported on batch contexts");
    if (c->prob.dudn != 0) return fail(DWOS_ESTATE, "batch_grad: the gradient normal-derivative estimator is not supported on batch contexts");
    if (!P || W < 1 || !grad) return fail(DWOS_EINVAL, "batch_grad: bad P, W or grad");
    if (dwos_status rr = check_batch_roulette(c, "batch_grad")) return rr;
    int64_t pts = 0, Ntot = 0;
    for (size_t i = 0; i < c->instances.size(); ++i) {
        if (P[i] < 0 || P[i] > INT32_MAX) return fail(DWOS_EINVAL, "batch_grad: bad point count");
        pts += P[i];
        Ntot += c->batch_params[i].N;
        if (c->instances[i].delta != c->instances[0].delta)
            return fail(DWOS_EINVAL, "batch_grad: every instance must have the same delta");
    }
    if (Ntot < 1) return fail(DWOS_ESTATE, "batch_grad: no parameters: call dwos_batch_set_parameters");
    if (pts > 0 && (!X_all || !w)) return fail(DWOS_EINVAL, "batch_grad: NULL points or weights");
    HIP_OK(hipSetDevice(c->device));
    if (c->batch_dirty) {
        dwos_status rc = c->prec == DWOS_FP32
            ? upload_geometry<float>(c, c->hostV, c->hostP, c->hostL, c->hostG, c->hostNodes, c->hostOrder)
            : upload_geometry<double>(c, c->hostV, c->hostP, c->hostL, c->hostG, c->hostNodes, c->hostOrder);
        if (rc) return rc;
        rc = upload_prange(c);
        if (rc) return rc;
        c->batch_dirty = false;
        c->has_boundary = true;
        c->batch_params_dirty = true;
    }
    if (c->batch_params_dirty || !c->has_params) {
        // the combined Jacobian over the batch's vertex array
        const int D = c->D;
        const int64_t nv = (int64_t)c->hostV.size() / D;
        std::vector<int64_t> rp(nv + 1, 0);
        std::vector<int32_t> pv;
        std::vector<double> vv;
        int64_t poff = 0;
        for (size_t i = 0; i < c->instances.size(); ++i) {
            const auto& bp = c->batch_params[i];
            const int64_t v0 = c->instances[i].nv_off;
            const int64_t v1 = i + 1 < c->instances.size() ? c->instances[i + 1].nv_off : nv;
            for (int64_t v = v0; v < v1; ++v) {
                const int64_t lv = v - v0;
                if (bp.N > 0)
                    for (int64_t e = bp.rowptr[lv]; e < bp.rowptr[lv + 1]; ++e) {
                        pv.push_back((int32_t)(bp.pid[e] + poff));
                        for (int k = 0; k < D; ++k) vv.push_back(bp.vel[e * D + k]);
                    }
                rp[v + 1] = (int64_t)pv.size();
            }
            poff += bp.N;
        }
        dwos_status rc = set_parameters_impl(c, Ntot, rp.data(), pv.data(), vv.data(), nullptr);
        if (rc) return rc;
        c->batch_params_dirty = false;
    }
    dwos_status rc = begin_call(c, true);
    if (rc) return rc;
    if (c->prec == DWOS_FP32)
        return c->D == 2 ? run_batch_grad<float, 2>(c, X_all, P, w, W, seed, grad, u_mean, stats)
                         : run_batch_grad<float, 3>(c, X_all, P, w, W, seed, grad, u_mean, stats);
    return c->D == 2 ? run_batch_grad<double, 2>(c, X_all, P, w, W, seed, grad, u_mean, stats)
                     : run_batch_grad<double, 3>(c, X_all, P, w, W, seed, grad, u_mean, stats);
}

dwos_status dwos_batch_solve(dwos_ctx* c, const double* X_all, const int64_t* P, int32_t W, uint64_t seed,
                             double* u_mean, double* u_var, dwos_stats* stats) {
    if (!c) return fail(DWOS_EINVAL, "NULL context");
    if (c->instances.empty()) return fail(DWOS_ESTATE, "batch_solve: no instances");
    if (!c->has_problem) return fail(DWOS_ESTATE, "batch_solve: no problem: call dwos_set_problem first");
    if (!P || W < 1) return fail(DWOS_EINVAL, "batch_solve: bad P or W");
    if (dwos_status rr = check_batch_roulette(c, "batch_solve")) return rr;
    int64_t pts = 0;
    for (size_t i = 0; i < c->instances.size(); ++i) {
        if (P[i] < 0 || P[i] > INT32_MAX) return fail(DWOS_EINVAL, "batch_solve: bad point count");
        pts += P[i];
    }
    if (pts > 0 && (!X_all || !u_mean)) return fail(DWOS_EINVAL, "batch_solve: NULL points or output");
    HIP_OK(hipSetDevice(c->device));
    if (c->batch_dirty) {
        dwos_status rc = c->prec == DWOS_FP32
            ? upload_geometry<float>(c, c->hostV, c->hostP, c->hostL, c->hostG, c->hostNodes, c->hostOrder)
            : upload_geometry<double>(c, c->hostV, c->hostP, c->hostL, c->hostG, c->hostNodes, c->hostOrder);
        if (rc) return rc;
        rc = upload_prange(c);
        if (rc) return rc;
        c->batch_dirty = false;
        c->has_boundary = true;
    }
    dwos_status rc = begin_call(c, false);
    if (rc) return rc;
    if (pts == 0) return finish_call(c, stats, c->pending.size());
    if (c->prec == DWOS_FP32)
        return c->D == 2 ? run_batch<float, 2>(c, X_all, P, W, seed, u_mean, u_var, stats)
                         : run_batch<float, 3>(c, X_all, P, W, seed, u_mean, u_var, stats);
    return c->D == 2 ? run_batch<double, 2>(c, X_all, P, W, seed, u_mean, u_var, stats)
                     : run_batch<double, 3>(c, X_all, P, W, seed, u_mean, u_var, stats);
}

}  // extern "C"
