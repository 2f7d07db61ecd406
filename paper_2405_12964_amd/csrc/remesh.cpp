// Isotropic remeshing of a boundary (host code): the periodic remeshing of
// the paper's shape-optimisation loop (Sec. 7.2, "Gradient
// preconditioning", which cites Botsch and Kobbelt's remeshing approach).
// For a target edge length L each iteration
//   1. splits every edge longer than 4L/3 at its midpoint,
//   2. collapses every edge shorter than 4L/5 into its midpoint unless that
//      would create an edge longer than 4L/3, change the topology (the link
//      condition) or flip a triangle,
//   3. (3D) flips edges that bring the four vertices' valences nearer 6,
//   4. moves every free vertex towards the centroid of its neighbours within
//      its tangent plane (line in 2D),
//   5. projects the moved vertices back onto the input surface.
// Fixed vertices (and, in 3D, vertices on a border edge) neither move nor
// disappear; an edge between two of them is neither split nor collapsed.
// 2D meshes are polylines (segments), 3D meshes triangles; orientation is
// preserved.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <limits>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/dwos.h"
#include "host_common.hpp"

using dwos_host::fail;

struct dwos_mesh {
    int dim = 0;
    std::vector<double> V;       // nv x dim
    std::vector<int32_t> P;      // np x dim
    std::vector<int64_t> src;    // nv: input vertex index, -1 for a new vertex
};

namespace {

using V3 = std::array<double, 3>;

V3 sub(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
V3 add(const V3& a, const V3& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
V3 mul(const V3& a, double s) { return {a[0] * s, a[1] * s, a[2] * s}; }
double dot(const V3& a, const V3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
V3 cross(const V3& a, const V3& b) {
    return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
double norm(const V3& a) { return std::sqrt(dot(a, a)); }

uint64_t ekey(int a, int b) {
    if (a > b) std::swap(a, b);
    return (uint64_t)(uint32_t)a << 32 | (uint32_t)b;
}

// closest point on a triangle (Ericson, Real-Time Collision Detection, 5.1.5)
V3 closest_on_tri(const V3& p, const V3& a, const V3& b, const V3& c) {
    const V3 ab = sub(b, a), ac = sub(c, a), ap = sub(p, a);
    const double d1 = dot(ab, ap), d2 = dot(ac, ap);
    if (d1 <= 0 && d2 <= 0) return a;
    const V3 bp = sub(p, b);
    const double d3 = dot(ab, bp), d4 = dot(ac, bp);
    if (d3 >= 0 && d4 <= d3) return b;
    const double vc = d1 * d4 - d3 * d2;
    if (vc <= 0 && d1 >= 0 && d3 <= 0) return add(a, mul(ab, d1 / (d1 - d3)));
    const V3 cp = sub(p, c);
    const double d5 = dot(ab, cp), d6 = dot(ac, cp);
    if (d6 >= 0 && d5 <= d6) return c;
    const double vb = d5 * d2 - d1 * d6;
    if (vb <= 0 && d2 >= 0 && d6 <= 0) return add(a, mul(ac, d2 / (d2 - d6)));
    const double va = d3 * d6 - d5 * d4;
    if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0)
        return add(b, mul(sub(c, b), (d4 - d3) / ((d4 - d3) + (d5 - d6))));
    const double den = 1.0 / (va + vb + vc);
    return add(a, add(mul(ab, vb * den), mul(ac, vc * den)));
}

V3 closest_on_seg(const V3& p, const V3& a, const V3& b) {
    const V3 ab = sub(b, a);
    const double l2 = dot(ab, ab);
    double t = l2 > 0 ? dot(sub(p, a), ab) / l2 : 0.0;
    t = std::min(1.0, std::max(0.0, t));
    return add(a, mul(ab, t));
}

// The input surface with a uniform grid over its primitives' boxes, for
// projecting moved vertices back onto it.
struct Surface {
    int D;
    std::vector<V3> V;
    std::vector<std::array<int, 3>> P;
    V3 lo{}, cell{};
    int n[3] = {1, 1, 1};
    std::vector<std::vector<int>> bins;

    Surface(int D_, const std::vector<V3>& V_, const std::vector<std::array<int, 3>>& P_, double h)
        : D(D_), V(V_), P(P_) {
        V3 hi{-1e300, -1e300, -1e300};
        lo = {1e300, 1e300, 1e300};
        for (const V3& v : V)
            for (int i = 0; i < D; ++i) { lo[i] = std::min(lo[i], v[i]); hi[i] = std::max(hi[i], v[i]); }
        // at most ~2^20 cells: coarser than h for a large extent
        double vol = 1;
        for (int i = 0; i < D; ++i) vol *= std::max(hi[i] - lo[i], 1e-12);
        h = std::max(h, std::pow(vol / 1048576.0, 1.0 / D));
        size_t cells = 1;
        for (int i = 0; i < 3; ++i) {
            if (i >= D) { n[i] = 1; cell[i] = 1; lo[i] = 0; continue; }
            const double ext = std::max(hi[i] - lo[i], 1e-12);
            n[i] = (int)std::min<double>(1024.0, std::max(1.0, std::ceil(ext / h)));
            cell[i] = ext / n[i] * (1 + 1e-9);
            cells *= (size_t)n[i];
        }
        bins.assign(cells, {});
        for (int f = 0; f < (int)P.size(); ++f) {
            int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
            for (int i = 0; i < D; ++i) {
                double a = 1e300, b = -1e300;
                for (int k = 0; k < D; ++k) { a = std::min(a, V[P[f][k]][i]); b = std::max(b, V[P[f][k]][i]); }
                c0[i] = clampi((int)std::floor((a - lo[i]) / cell[i]), i);
                c1[i] = clampi((int)std::floor((b - lo[i]) / cell[i]), i);
            }
            for (int z = c0[2]; z <= c1[2]; ++z)
                for (int y = c0[1]; y <= c1[1]; ++y)
                    for (int x = c0[0]; x <= c1[0]; ++x) bins[((size_t)z * n[1] + y) * n[0] + x].push_back(f);
        }
    }
    int clampi(int v, int i) const { return std::min(n[i] - 1, std::max(0, v)); }

    V3 closest_in(const V3& p, int f) const {
        if (D == 2) return closest_on_seg(p, V[P[f][0]], V[P[f][1]]);
        return closest_on_tri(p, V[P[f][0]], V[P[f][1]], V[P[f][2]]);
    }

    // nearest point of the surface: rings of cells around p until the best
    // distance is within the searched radius
    V3 project(const V3& p) const {
        int c[3] = {0, 0, 0};
        for (int i = 0; i < D; ++i) c[i] = clampi((int)std::floor((p[i] - lo[i]) / cell[i]), i);
        double best = std::numeric_limits<double>::infinity();
        V3 q = p;
        const int rmax = std::max(n[0], std::max(n[1], n[2]));
        for (int r = 0; r <= rmax; ++r) {
            for (int z = (D == 3 ? c[2] - r : 0); z <= (D == 3 ? c[2] + r : 0); ++z)
                for (int y = c[1] - r; y <= c[1] + r; ++y)
                    for (int x = c[0] - r; x <= c[0] + r; ++x) {
                        const int m = std::max(std::abs(x - c[0]), std::max(std::abs(y - c[1]), std::abs(z - c[2])));
                        if (m != r) continue;   // the ring only
                        if (x < 0 || y < 0 || z < 0 || x >= n[0] || y >= n[1] || z >= n[2]) continue;
                        for (int f : bins[((size_t)z * n[1] + y) * n[0] + x]) {
                            const V3 s = closest_in(p, f);
                            const double d = norm(sub(s, p));
                            if (d < best) { best = d; q = s; }
                        }
                    }
            // every primitive not seen yet lies outside the searched block of
            // cells, so at least `margin` away from p (p may be outside the
            // grid, where the margin is negative until the whole grid is seen)
            double margin = std::numeric_limits<double>::infinity();
            for (int i = 0; i < D; ++i) {
                const double blo = lo[i] + (c[i] - r) * cell[i], bhi = lo[i] + (c[i] + r + 1) * cell[i];
                margin = std::min(margin, std::min(p[i] - blo, bhi - p[i]));
            }
            if (best <= margin) break;
        }
        return q;
    }
};

// ---------------------------------------------------------------- 2D -------
struct Poly {
    std::vector<V3> V;
    std::vector<std::array<int, 3>> S;   // segments (a, b, unused)
    std::vector<char> fixed;
    std::vector<int64_t> src;
};

void rebuild_2d(Poly& m, std::vector<int>& next, std::vector<int>& prev) {
    next.assign(m.V.size(), -1);
    prev.assign(m.V.size(), -1);
    for (const auto& s : m.S) { next[s[0]] = s[1]; prev[s[1]] = s[0]; }
}

void remesh_2d(Poly& m, const Surface& surf, double L, int iters) {
    const double hi = 4.0 / 3.0 * L, lo = 4.0 / 5.0 * L;
    std::vector<int> next, prev;
    for (int it = 0; it < iters; ++it) {
        // 1. split long segments
        std::vector<std::array<int, 3>> S2;
        for (const auto& s : m.S) {
            const int a = s[0], b = s[1];
            const double l = norm(sub(m.V[a], m.V[b]));
            const int k = (l > hi && !(m.fixed[a] && m.fixed[b])) ? (int)std::ceil(l / L) : 1;
            int prevv = a;
            for (int j = 1; j < k; ++j) {
                m.V.push_back(add(m.V[a], mul(sub(m.V[b], m.V[a]), (double)j / k)));
                m.fixed.push_back(0);
                m.src.push_back(-1);
                const int v = (int)m.V.size() - 1;
                S2.push_back({prevv, v, 0});
                prevv = v;
            }
            S2.push_back({prevv, b, 0});
        }
        m.S.swap(S2);
        rebuild_2d(m, next, prev);
        // 2. collapse short segments (b into the midpoint, a removed)
        std::vector<char> dead(m.V.size(), 0), touched(m.V.size(), 0);
        for (const auto& s : m.S) {
            const int a = s[0], b = s[1];
            if (dead[a] || dead[b] || touched[a] || touched[b]) continue;
            if (norm(sub(m.V[a], m.V[b])) >= lo) continue;
            const int pa = prev[a], nb = next[b];
            if (pa < 0 || nb < 0 || pa == b || nb == a || pa == nb) continue;   // open ends, tiny loops
            if (m.fixed[a] && m.fixed[b]) continue;
            const V3 mid = m.fixed[a] ? m.V[a] : m.fixed[b] ? m.V[b] : mul(add(m.V[a], m.V[b]), 0.5);
            if (norm(sub(mid, m.V[pa])) > hi || norm(sub(mid, m.V[nb])) > hi) continue;
            // keep b, drop a
            m.V[b] = mid;
            if (m.fixed[a]) { m.fixed[b] = 1; m.src[b] = m.src[a]; }
            dead[a] = 1;
            next[pa] = b;
            prev[b] = pa;
            touched[pa] = touched[b] = touched[nb] = 1;
        }
        S2.clear();
        for (size_t v = 0; v < m.V.size(); ++v)
            if (!dead[v] && next[v] >= 0) S2.push_back({(int)v, next[v], 0});
        m.S.swap(S2);
        // 3. relax along the tangent and project
        rebuild_2d(m, next, prev);
        std::vector<V3> nv = m.V;
        for (size_t v = 0; v < m.V.size(); ++v) {
            if (dead[v] || m.fixed[v] || prev[v] < 0 || next[v] < 0) continue;
            const V3 q = mul(add(m.V[prev[v]], m.V[next[v]]), 0.5);
            V3 t = sub(m.V[next[v]], m.V[prev[v]]);
            const double tl = norm(t);
            if (tl == 0) continue;
            t = mul(t, 1.0 / tl);
            nv[v] = surf.project(add(m.V[v], mul(t, dot(t, sub(q, m.V[v])))));
        }
        m.V.swap(nv);
        // compact the vertex array
        std::vector<int> remap(m.V.size(), -1);
        Poly c;
        for (size_t v = 0; v < m.V.size(); ++v) {
            if (dead[v]) continue;
            remap[v] = (int)c.V.size();
            c.V.push_back(m.V[v]);
            c.fixed.push_back(m.fixed[v]);
            c.src.push_back(m.src[v]);
        }
        for (const auto& s : m.S) c.S.push_back({remap[s[0]], remap[s[1]], 0});
        m = std::move(c);
    }
}

// ---------------------------------------------------------------- 3D -------
struct Tri {
    std::vector<V3> V;
    std::vector<std::array<int, 3>> F;
    std::vector<char> fixed;
    std::vector<int64_t> src;
};

// edge -> up to two faces (third slot counts faces beyond two)
struct EdgeMap {
    std::unordered_map<uint64_t, std::array<int, 3>> m;
    void build(const Tri& t) {
        m.clear();
        m.reserve(t.F.size() * 2);
        for (int f = 0; f < (int)t.F.size(); ++f)
            for (int k = 0; k < 3; ++k) {
                auto& e = m.try_emplace(ekey(t.F[f][k], t.F[f][(k + 1) % 3]), std::array<int, 3>{-1, -1, 0}).first->second;
                if (e[0] < 0) e[0] = f;
                else if (e[1] < 0) e[1] = f;
                else e[2]++;
            }
    }
};

int third(const std::array<int, 3>& f, int a, int b) {
    for (int k = 0; k < 3; ++k) if (f[k] != a && f[k] != b) return f[k];
    return -1;
}

V3 face_normal(const Tri& t, const std::array<int, 3>& f) {
    return cross(sub(t.V[f[1]], t.V[f[0]]), sub(t.V[f[2]], t.V[f[0]]));
}

void mark_border(Tri& t) {
    EdgeMap em;
    em.build(t);
    for (const auto& kv : em.m)
        if (kv.second[1] < 0) { t.fixed[kv.first >> 32] = 1; t.fixed[kv.first & 0xffffffffu] = 1; }
}

void split_3d(Tri& t, double hi) {
    for (int pass = 0; pass < 8; ++pass) {
        EdgeMap em;
        em.build(t);
        std::vector<std::pair<double, uint64_t>> longe;
        for (const auto& kv : em.m) {
            const int a = (int)(kv.first >> 32), b = (int)(kv.first & 0xffffffffu);
            const double l = norm(sub(t.V[a], t.V[b]));
            if (l > hi && kv.second[1] >= 0 && !(t.fixed[a] && t.fixed[b])) longe.push_back({l, kv.first});
        }
        if (longe.empty()) return;
        std::sort(longe.begin(), longe.end(), [](auto& x, auto& y) { return x.first > y.first; });
        std::vector<char> ftouched(t.F.size(), 0);
        for (const auto& le : longe) {
            const auto& e = em.m[le.second];
            const int f1 = e[0], f2 = e[1];
            if (ftouched[f1] || ftouched[f2]) continue;
            const int a = (int)(le.second >> 32), b = (int)(le.second & 0xffffffffu);
            t.V.push_back(mul(add(t.V[a], t.V[b]), 0.5));
            t.fixed.push_back(0);
            t.src.push_back(-1);
            const int m = (int)t.V.size() - 1;
            for (int f : {f1, f2}) {
                std::array<int, 3> F = t.F[f];
                // rotate so that the split edge is F[0] -> F[1]
                int k = 0;
                while (!((F[k] == a && F[(k + 1) % 3] == b) || (F[k] == b && F[(k + 1) % 3] == a))) ++k;
                const int p = F[k], q = F[(k + 1) % 3], r = F[(k + 2) % 3];
                t.F[f] = {p, m, r};
                t.F.push_back({m, q, r});
                ftouched[f] = 1;
                ftouched.push_back(1);
            }
        }
    }
}

// one-ring neighbour sets and vertex -> faces
void rings(const Tri& t, std::vector<std::vector<int>>& vf) {
    vf.assign(t.V.size(), {});
    for (int f = 0; f < (int)t.F.size(); ++f)
        for (int k = 0; k < 3; ++k) vf[t.F[f][k]].push_back(f);
}

void collapse_3d(Tri& t, double lo, double hi) {
    for (int pass = 0; pass < 8; ++pass) {
        EdgeMap em;
        em.build(t);
        std::vector<std::vector<int>> vf;
        rings(t, vf);
        std::vector<std::pair<double, uint64_t>> shorte;
        for (const auto& kv : em.m) {
            const int a = (int)(kv.first >> 32), b = (int)(kv.first & 0xffffffffu);
            const double l = norm(sub(t.V[a], t.V[b]));
            if (l < lo && kv.second[1] >= 0) shorte.push_back({l, kv.first});
        }
        if (shorte.empty()) return;
        std::sort(shorte.begin(), shorte.end());
        std::vector<char> vtouched(t.V.size(), 0), fdead(t.F.size(), 0);
        int done = 0;
        for (const auto& se : shorte) {
            int a = (int)(se.second >> 32), b = (int)(se.second & 0xffffffffu);
            if (vtouched[a] || vtouched[b]) continue;
            if (t.fixed[a] && t.fixed[b]) continue;
            if (t.fixed[a]) std::swap(a, b);          // b (kept) is the fixed one if any
            const auto& e = em.m[se.second];
            const int f1 = e[0], f2 = e[1];
            const int c = third(t.F[f1], a, b), d = third(t.F[f2], a, b);
            // link condition: the common neighbours of a and b are c and d
            std::unordered_set<int> na;
            for (int f : vf[a]) for (int k = 0; k < 3; ++k) if (t.F[f][k] != a) na.insert(t.F[f][k]);
            int common = 0;
            std::unordered_set<int> nb;
            for (int f : vf[b]) for (int k = 0; k < 3; ++k) if (t.F[f][k] != b) nb.insert(t.F[f][k]);
            for (int v : nb) if (na.count(v)) ++common;
            if (common != 2 || c == d) continue;
            const V3 mid = t.fixed[b] ? t.V[b] : mul(add(t.V[a], t.V[b]), 0.5);
            bool ok = true;
            for (int v : na) if (v != b && norm(sub(t.V[v], mid)) > hi) { ok = false; break; }
            for (int v : nb) if (ok && v != a && norm(sub(t.V[v], mid)) > hi) { ok = false; break; }
            if (!ok) continue;
            // no surviving face may flip or degenerate
            for (int w : {a, b}) {
                for (int f : vf[w]) {
                    if (f == f1 || f == f2 || !ok) continue;
                    std::array<int, 3> F = t.F[f];
                    const V3 n0 = face_normal(t, F);
                    for (int k = 0; k < 3; ++k) if (F[k] == a) F[k] = b;
                    const V3 saved = t.V[b];
                    t.V[b] = mid;
                    const V3 n1 = face_normal(t, F);
                    t.V[b] = saved;
                    if (dot(n0, n1) <= 1e-3 * dot(n0, n0)) ok = false;
                }
            }
            if (!ok) continue;
            t.V[b] = mid;
            for (int f : vf[a]) for (int k = 0; k < 3; ++k) if (t.F[f][k] == a) t.F[f][k] = b;
            fdead[f1] = fdead[f2] = 1;
            for (int v : na) vtouched[v] = 1;
            for (int v : nb) vtouched[v] = 1;
            vtouched[a] = vtouched[b] = 1;
            ++done;
        }
        std::vector<std::array<int, 3>> F2;
        for (size_t f = 0; f < t.F.size(); ++f) if (!fdead[f]) F2.push_back(t.F[f]);
        t.F.swap(F2);
        if (!done) return;
    }
}

void flip_3d(Tri& t) {
    for (int pass = 0; pass < 4; ++pass) {
        EdgeMap em;
        em.build(t);
        std::vector<int> val(t.V.size(), 0);
        for (const auto& kv : em.m) { val[kv.first >> 32]++; val[kv.first & 0xffffffffu]++; }
        std::vector<char> ftouched(t.F.size(), 0);
        std::unordered_set<uint64_t> created;   // edges made by this pass's flips
        int done = 0;
        for (const auto& kv : em.m) {
            const int f1 = kv.second[0], f2 = kv.second[1];
            if (f2 < 0 || ftouched[f1] || ftouched[f2]) continue;
            const int a = (int)(kv.first >> 32), b = (int)(kv.first & 0xffffffffu);
            const int c = third(t.F[f1], a, b), d = third(t.F[f2], a, b);
            if (c == d || em.m.count(ekey(c, d)) || created.count(ekey(c, d))) continue;
            if (val[a] <= 3 || val[b] <= 3) continue;
            auto dev = [](int x) { return (x - 6) * (x - 6); };
            const int before = dev(val[a]) + dev(val[b]) + dev(val[c]) + dev(val[d]);
            const int after = dev(val[a] - 1) + dev(val[b] - 1) + dev(val[c] + 1) + dev(val[d] + 1);
            if (after >= before) continue;
            // orient: f1 holds the directed edge p -> q, its third vertex r;
            // f2 holds q -> p with third s; new faces (s, q, r) and (r, p, s)
            std::array<int, 3> F = t.F[f1];
            int k = 0;
            while (!((F[k] == a || F[k] == b) && (F[(k + 1) % 3] == a || F[(k + 1) % 3] == b))) ++k;
            const int p = F[k], q = F[(k + 1) % 3], r = F[(k + 2) % 3];
            const int s = third(t.F[f2], a, b);
            const std::array<int, 3> g1{s, q, r}, g2{r, p, s};
            const V3 n0 = add(face_normal(t, t.F[f1]), face_normal(t, t.F[f2]));
            const V3 m1 = face_normal(t, g1), m2 = face_normal(t, g2);
            if (dot(n0, m1) <= 1e-3 * norm(n0) * norm(m1) || dot(n0, m2) <= 1e-3 * norm(n0) * norm(m2)) continue;
            t.F[f1] = g1;
            t.F[f2] = g2;
            created.insert(ekey(c, d));
            val[a]--; val[b]--; val[c]++; val[d]++;
            ftouched[f1] = ftouched[f2] = 1;
            ++done;
        }
        if (!done) return;
    }
}

void relax_3d(Tri& t, const Surface& surf) {
    std::vector<std::vector<int>> vf;
    rings(t, vf);
    std::vector<V3> nv = t.V;
    for (size_t v = 0; v < t.V.size(); ++v) {
        if (t.fixed[v] || vf[v].empty()) continue;
        V3 q{0, 0, 0}, n{0, 0, 0};
        std::unordered_set<int> nb;
        for (int f : vf[v]) {
            n = add(n, face_normal(t, t.F[f]));
            for (int k = 0; k < 3; ++k) if (t.F[f][k] != (int)v) nb.insert(t.F[f][k]);
        }
        for (int w : nb) q = add(q, t.V[w]);
        q = mul(q, 1.0 / nb.size());
        const double nl = norm(n);
        if (nl == 0) continue;
        n = mul(n, 1.0 / nl);
        const V3 dlt = sub(q, t.V[v]);
        nv[v] = surf.project(add(t.V[v], sub(dlt, mul(n, dot(n, dlt)))));
    }
    t.V.swap(nv);
}

void compact_3d(Tri& t) {
    std::vector<int> used(t.V.size(), -1);
    Tri c;
    for (auto& f : t.F)
        for (int k = 0; k < 3; ++k)
            if (used[f[k]] < 0) {
                used[f[k]] = (int)c.V.size();
                c.V.push_back(t.V[f[k]]);
                c.fixed.push_back(t.fixed[f[k]]);
                c.src.push_back(t.src[f[k]]);
            }
    for (auto& f : t.F) c.F.push_back({used[f[0]], used[f[1]], used[f[2]]});
    t = std::move(c);
}

}  // namespace

extern "C" {

dwos_status dwos_remesh(int32_t dim, const double* V, int64_t nv, const int32_t* prims, int64_t np,
                        const int32_t* fixed, double target, int32_t iters, dwos_mesh** out) {
    if (!out) return fail(DWOS_EINVAL, "remesh: NULL out");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(DWOS_EINVAL, "remesh: dim must be 2 or 3");
    if (nv <= 0 || np <= 0 || !V || !prims || nv > INT32_MAX / 4 || np > INT32_MAX / 8)
        return fail(DWOS_EINVAL, "remesh: empty or oversized mesh");
    if (!(target > 0) || !std::isfinite(target)) return fail(DWOS_EINVAL, "remesh: target length must be > 0");
    if (iters < 0 || iters > 100) return fail(DWOS_EINVAL, "remesh: iters must be in 0..100");
    for (int64_t i = 0; i < nv * dim; ++i)
        if (!std::isfinite(V[i])) return fail(DWOS_EINVAL, "remesh: non-finite vertex");
    for (int64_t i = 0; i < np * dim; ++i)
        if (prims[i] < 0 || prims[i] >= nv) return fail(DWOS_EINVAL, "remesh: vertex index out of range");
    std::vector<V3> Vv(nv, V3{0, 0, 0});
    for (int64_t i = 0; i < nv; ++i) for (int c = 0; c < dim; ++c) Vv[i][c] = V[i * dim + c];
    std::vector<std::array<int, 3>> Pv(np, std::array<int, 3>{0, 0, 0});
    for (int64_t f = 0; f < np; ++f) {
        for (int c = 0; c < dim; ++c) Pv[f][c] = prims[f * dim + c];
        for (int c = 0; c < dim; ++c)
            for (int e = c + 1; e < dim; ++e)
                if (Pv[f][c] == Pv[f][e]) return fail(DWOS_EINVAL, "remesh: degenerate primitive " + std::to_string(f));
    }
    const Surface surf(dim, Vv, Pv, 2 * target);
    auto* m = new dwos_mesh;
    m->dim = dim;
    if (dim == 2) {
        std::vector<int> deg_out(nv, 0), deg_in(nv, 0);
        for (const auto& s : Pv) { deg_out[s[0]]++; deg_in[s[1]]++; }
        for (int64_t i = 0; i < nv; ++i)
            if (deg_out[i] > 1 || deg_in[i] > 1) {
                delete m;
                return fail(DWOS_EINVAL, "remesh: 2D vertices must have at most one segment in and one out");
            }
        Poly p;
        p.V = Vv;
        p.S = Pv;
        p.fixed.assign(nv, 0);
        p.src.resize(nv);
        for (int64_t i = 0; i < nv; ++i) { p.src[i] = i; if (fixed && fixed[i]) p.fixed[i] = 1; }
        for (int64_t i = 0; i < nv; ++i) if (deg_in[i] == 0 || deg_out[i] == 0) p.fixed[i] = 1;   // open ends
        remesh_2d(p, surf, target, iters);
        for (const V3& v : p.V) for (int c = 0; c < 2; ++c) m->V.push_back(v[c]);
        for (const auto& s : p.S) { m->P.push_back(s[0]); m->P.push_back(s[1]); }
        m->src = p.src;
    } else {
        Tri t;
        t.V = Vv;
        t.F = Pv;
        t.fixed.assign(nv, 0);
        t.src.resize(nv);
        for (int64_t i = 0; i < nv; ++i) { t.src[i] = i; if (fixed && fixed[i]) t.fixed[i] = 1; }
        EdgeMap em;
        em.build(t);
        for (const auto& kv : em.m)
            if (kv.second[2] > 0) {
                delete m;
                return fail(DWOS_EINVAL, "remesh: non-manifold edge (more than two triangles)");
            }
        mark_border(t);
        const double hi = 4.0 / 3.0 * target, lo = 4.0 / 5.0 * target;
        for (int it = 0; it < iters; ++it) {
            split_3d(t, hi);
            collapse_3d(t, lo, hi);
            compact_3d(t);
            flip_3d(t);
            relax_3d(t, surf);
        }
        compact_3d(t);
        for (const V3& v : t.V) for (int c = 0; c < 3; ++c) m->V.push_back(v[c]);
        for (const auto& f : t.F) for (int c = 0; c < 3; ++c) m->P.push_back(f[c]);
        m->src = t.src;
    }
    *out = m;
    return DWOS_OK;
}

dwos_status dwos_mesh_size(const dwos_mesh* m, int64_t* nv, int64_t* np) {
    if (!m || !nv || !np) return fail(DWOS_EINVAL, "mesh_size: NULL argument");
    *nv = (int64_t)m->V.size() / m->dim;
    *np = (int64_t)m->P.size() / m->dim;
    return DWOS_OK;
}

dwos_status dwos_mesh_get(const dwos_mesh* m, double* V, int32_t* prims, int64_t* src) {
    if (!m) return fail(DWOS_EINVAL, "mesh_get: NULL mesh");
    if (V) std::copy(m->V.begin(), m->V.end(), V);
    if (prims) std::copy(m->P.begin(), m->P.end(), prims);
    if (src) std::copy(m->src.begin(), m->src.end(), src);
    return DWOS_OK;
}

void dwos_mesh_destroy(dwos_mesh* m) { delete m; }

}  // extern "C"
