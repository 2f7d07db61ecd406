// Host BVH builder: binned surface-area heuristic over primitive boxes.
#include "bvh.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace dwos {
namespace {

struct Box {
    double lo[3] = {std::numeric_limits<double>::infinity(), std::numeric_limits<double>::infinity(),
                    std::numeric_limits<double>::infinity()};
    double hi[3] = {-std::numeric_limits<double>::infinity(), -std::numeric_limits<double>::infinity(),
                    -std::numeric_limits<double>::infinity()};
    void grow(const Box& b, int D) {
        for (int i = 0; i < D; ++i) { lo[i] = std::min(lo[i], b.lo[i]); hi[i] = std::max(hi[i], b.hi[i]); }
    }
    void grow(const double* p, int D) {
        for (int i = 0; i < D; ++i) { lo[i] = std::min(lo[i], p[i]); hi[i] = std::max(hi[i], p[i]); }
    }
    // surface area (3D) or perimeter (2D): proportional to the probability
    // that a random query ball overlaps the box
    double area(int D) const {
        double e[3] = {0, 0, 0};
        for (int i = 0; i < D; ++i) e[i] = std::max(0.0, hi[i] - lo[i]);
        return D == 2 ? e[0] + e[1] : e[0] * e[1] + e[1] * e[2] + e[2] * e[0];
    }
};

// Best-fit normal of a point set: the eigenvector of the smallest eigenvalue
// of its covariance (2D in closed form, 3D by cyclic Jacobi rotations).
void fit_normal(const std::vector<double>& pts, int D, double n[3]) {
    const size_t m = pts.size() / 3;
    double c[3] = {0, 0, 0};
    for (size_t i = 0; i < m; ++i) for (int k = 0; k < 3; ++k) c[k] += pts[3 * i + k];
    for (int k = 0; k < 3; ++k) c[k] /= std::max<size_t>(1, m);
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (size_t i = 0; i < m; ++i)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A[a][b] += (pts[3 * i + a] - c[a]) * (pts[3 * i + b] - c[b]);
    n[0] = n[1] = n[2] = 0;
    if (D == 2) {
        const double th = 0.5 * std::atan2(2 * A[0][1], A[0][0] - A[1][1]);  // major axis
        n[0] = -std::sin(th);
        n[1] = std::cos(th);
        return;
    }
    double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = std::fabs(A[0][1]) + std::fabs(A[0][2]) + std::fabs(A[1][2]);
        if (off < 1e-300) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (std::fabs(A[p][q]) < 1e-300) continue;
                const double th = 0.5 * std::atan2(2 * A[p][q], A[q][q] - A[p][p]);
                const double cs = std::cos(th), sn = std::sin(th);
                for (int k = 0; k < 3; ++k) {   // A <- A J
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = cs * akp - sn * akq;
                    A[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; ++k) {   // A <- J^T A
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cs * apk - sn * aqk;
                    A[q][k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = cs * vkp - sn * vkq;
                    V[k][q] = sn * vkp + cs * vkq;
                }
            }
    }
    int j = 0;
    for (int k = 1; k < 3; ++k) if (A[k][k] < A[j][j]) j = k;
    const double L = std::sqrt(V[0][j] * V[0][j] + V[1][j] * V[1][j] + V[2][j] * V[2][j]);
    for (int k = 0; k < 3; ++k) n[k] = V[k][j] / (L > 0 ? L : 1.0);
}

struct Builder {
    int D;
    int LM = 8;                  // largest leaf
    const double* V = nullptr;
    const int32_t* P = nullptr;
    std::vector<Box> pbox;
    std::vector<double> cen;     // np x 3 centroids
    std::vector<int32_t> idx;    // permutation being partitioned
    HostBVH out;

    Box range_box(int b, int e) const {
        Box bx;
        for (int i = b; i < e; ++i) bx.grow(pbox[idx[i]], D);
        return bx;
    }

    // returns the child reference of the subtree over idx[b, e)
    int32_t build(int b, int e, int depth) {
        const int n = e - b;
        if (n <= LM) return leaf_ref(b, n);
        // room left below this node: a subtree of n prims needs
        // ceil(log2(n / LM)) further levels when split at the median
        const int levels_needed = (int)std::ceil(std::log2((double)n / LM));
        const bool force_median = depth + 1 + levels_needed >= kMaxDepth - 2;

        Box cb;
        for (int i = b; i < e; ++i) cb.grow(&cen[3 * (size_t)idx[i]], D);
        int axis = 0;
        double ext = cb.hi[0] - cb.lo[0];
        for (int a = 1; a < D; ++a)
            if (cb.hi[a] - cb.lo[a] > ext) { ext = cb.hi[a] - cb.lo[a]; axis = a; }

        int mid = -1;
        if (!force_median && ext > 0) {
            constexpr int NB = 32;
            Box bb[NB];
            int bc[NB] = {0};
            const double scale = NB / ext;
            auto bin_of = [&](int i) {
                int k = (int)((cen[3 * (size_t)idx[i] + axis] - cb.lo[axis]) * scale);
                return std::min(NB - 1, std::max(0, k));
            };
            for (int i = b; i < e; ++i) { int k = bin_of(i); bc[k]++; bb[k].grow(pbox[idx[i]], D); }
            double left_a[NB], right_a[NB];
            int left_n[NB], right_n[NB];
            Box acc; int cnt = 0;
            for (int k = 0; k < NB; ++k) { acc.grow(bb[k], D); cnt += bc[k]; left_a[k] = acc.area(D); left_n[k] = cnt; }
            acc = Box(); cnt = 0;
            for (int k = NB - 1; k >= 0; --k) { acc.grow(bb[k], D); cnt += bc[k]; right_a[k] = acc.area(D); right_n[k] = cnt; }
            double best = std::numeric_limits<double>::infinity();
            int bestk = -1;
            for (int k = 0; k < NB - 1; ++k) {
                if (left_n[k] == 0 || right_n[k + 1] == 0) continue;
                double c = left_a[k] * left_n[k] + right_a[k + 1] * right_n[k + 1];
                if (c < best) { best = c; bestk = k; }
            }
            if (bestk >= 0) {
                auto it = std::partition(idx.begin() + b, idx.begin() + e,
                                         [&](int32_t p) {
                                             int k = (int)((cen[3 * (size_t)p + axis] - cb.lo[axis]) * scale);
                                             k = std::min(NB - 1, std::max(0, k));
                                             return k <= bestk;
                                         });
                mid = (int)(it - idx.begin());
                // keep the depth guarantee: neither side may need more levels
                // than remain
                int lmax = std::max(mid - b, e - mid);
                int need = (int)std::ceil(std::log2(std::max(1.0, (double)lmax / LM)));
                if (depth + 1 + need >= kMaxDepth - 2) mid = -1;
            }
        }
        if (mid <= b || mid >= e) {
            mid = b + n / 2;
            std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e,
                             [&](int32_t p, int32_t q) {
                                 double a = cen[3 * (size_t)p + axis], c = cen[3 * (size_t)q + axis];
                                 return a < c || (a == c && p < q);
                             });
        }
        const int32_t me = (int32_t)out.nodes.size();
        out.nodes.push_back(HostNode{});
        out.nodes[me].depth = depth;
        out.max_depth = std::max(out.max_depth, depth);
        Box l = range_box(b, mid), r = range_box(mid, e);
        int32_t c0 = build(b, mid, depth + 1);
        int32_t c1 = build(mid, e, depth + 1);
        HostNode& nd = out.nodes[me];
        for (int i = 0; i < 3; ++i) {
            nd.lo[0][i] = i < D ? l.lo[i] : 0; nd.hi[0][i] = i < D ? l.hi[i] : 0;
            nd.lo[1][i] = i < D ? r.lo[i] : 0; nd.hi[1][i] = i < D ? r.hi[i] : 0;
        }
        nd.child[0] = c0;
        nd.child[1] = c1;
        set_slab(nd, 0, b, mid);
        set_slab(nd, 1, mid, e);
        return me;
    }

    // slab of the primitives idx[b, e): fitted normal, exact enclosure
    void set_slab(HostNode& nd, int c, int b, int e) {
        nd.range[c][0] = b;
        nd.range[c][1] = e;
        std::vector<double> pts;
        pts.reserve(3 * D * (size_t)(e - b));
        for (int i = b; i < e; ++i)
            for (int k = 0; k < D; ++k) {
                const double* v = V + (size_t)P[(size_t)idx[i] * D + k] * D;
                pts.push_back(v[0]); pts.push_back(v[1]); pts.push_back(D == 3 ? v[2] : 0.0);
            }
        double n[3];
        fit_normal(pts, D, n);
        double lo = std::numeric_limits<double>::infinity(), hi = -lo;
        for (size_t i = 0; i < pts.size() / 3; ++i) {
            const double pr = n[0] * pts[3 * i] + n[1] * pts[3 * i + 1] + n[2] * pts[3 * i + 2];
            lo = std::min(lo, pr); hi = std::max(hi, pr);
        }
        for (int k = 0; k < 3; ++k) nd.n[c][k] = n[k];
        nd.o[c] = 0.5 * (lo + hi);
        nd.t[c] = 0.5 * (hi - lo);
    }
};

}  // namespace

HostBVH build_bvh(const double* V, const int32_t* prims, int64_t np, int D) {
    Builder B;
    B.D = D;
    B.LM = leaf_max(D);
    B.V = V;
    B.P = prims;
    B.pbox.resize(np);
    B.cen.assign(3 * (size_t)np, 0.0);
    B.idx.resize(np);
    for (int64_t p = 0; p < np; ++p) {
        Box bx;
        for (int k = 0; k < D; ++k) bx.grow(V + (size_t)prims[p * D + k] * D, D);
        B.pbox[p] = bx;
        for (int i = 0; i < D; ++i) B.cen[3 * p + i] = 0.5 * (bx.lo[i] + bx.hi[i]);
        B.idx[p] = (int32_t)p;
    }
    B.out.nodes.reserve(np);
    if (np <= leaf_max(D)) {
        // a single leaf under a root pair node whose second child is empty
        HostNode nd{};
        Box bx = B.range_box(0, (int)np);
        for (int i = 0; i < 3; ++i) {
            nd.lo[0][i] = i < D ? bx.lo[i] : 0; nd.hi[0][i] = i < D ? bx.hi[i] : 0;
            nd.lo[1][i] = 1e300; nd.hi[1][i] = -1e300;
        }
        nd.child[0] = leaf_ref(0, (int)np);
        nd.child[1] = leaf_ref(0, 1);
        nd.depth = 0;
        B.set_slab(nd, 0, 0, (int)np);
        // the second child is empty: an inverted box and a slab nothing is near
        nd.n[1][0] = 1; nd.n[1][1] = 0; nd.n[1][2] = 0;
        nd.o[1] = 0; nd.t[1] = -1e300;
        nd.range[1][0] = 0; nd.range[1][1] = 0;
        B.out.nodes.push_back(nd);
    } else {
        B.build(0, (int)np, 0);
    }
    B.out.order = B.idx;
    B.out.leaf_of.assign(np, 0);
    for (int64_t i = 0; i < np; ++i) B.out.leaf_of[B.out.order[i]] = (int32_t)i;
    return std::move(B.out);
}

void reorder_bfs(HostBVH& bvh) {
    const size_t n = bvh.nodes.size();
    std::vector<int32_t> order;
    order.reserve(n);
    order.push_back(0);
    for (size_t h = 0; h < order.size(); ++h)
        for (int c = 0; c < 2; ++c)
            if (bvh.nodes[order[h]].child[c] >= 0) order.push_back(bvh.nodes[order[h]].child[c]);
    std::vector<int32_t> newid(n, -1);
    for (size_t i = 0; i < order.size(); ++i) newid[order[i]] = (int32_t)i;
    std::vector<HostNode> out(order.size());
    for (size_t i = 0; i < order.size(); ++i) {
        out[i] = bvh.nodes[order[i]];
        for (int c = 0; c < 2; ++c)
            if (out[i].child[c] >= 0) out[i].child[c] = newid[out[i].child[c]];
    }
    bvh.nodes.swap(out);
}

}  // namespace dwos
