// FP64 CPU oracle for differential walk on spheres.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
// baseline leg of the benchmark may load this library.  It shares no code,
// header, table or constant generator with the GPU library: everything here
// is written out plainly from the paper (Miller, Sawhney, Crane, Gkioulekas,
// "Differential Walk on Spheres", ACM TOG 43(6), 2024).
//
// What it computes, in the paper's order:
//   * WoS for the screened Poisson Dirichlet problem (Sec. 3.3, eq. (wos),
//     Algorithm 1) with Russian roulette (Sec. 3.3, "Russian roulette").
//   * Differential WoS (Sec. 5.1, eq. (wos_deriv), Algorithm 2) with the
//     backward-difference normal derivative (eq. (dudn_fd_estimate)) or,
//     as the paper's ablation, the offset-point gradient estimator of
//     eq. (dudn_mc_estimate), the
//     joint solution estimate from the same walk (Sec. 5.1, observation 2)
//     and K nested forward walks per differential walk (Table 1).
//   * Differential boundary data for restricted fields
//     (eq. (boundary_deriv_restricted)) and for mapped data
//     (eq. (boundary_deriv_mapped), Appendix A).
//   * Reverse-mode accumulation with the U-statistic product estimator
//     (Sec. 5.3, eq. (ustatistics)).
//   * The adjoint formulation of the shape derivative (Appendix B), the
//     paper's rejected alternative, as an ablation: an adjoint walk whose
//     source is a whole forward walk at every step, on boundary samples.
// Closest points are found by brute force over every primitive, ties going to
// the lowest primitive index.  Random numbers come from Philox4x32-10
// (Salmon, Moraes, Dror, Shaw, SC'11), written here from its definition.
//
// Readings where the paper is silent (each listed in the design notes):
//   * PDE sign: -Lap u + sigma u = f, so the Green's-function source term
//     enters with a plus sign as in eq. (wos).
//   * G and P of the ball (cited by the paper to the walk-on-stars paper):
//     Q(R) = P/p^dB = 1/I0(kR) (2D), kR/sinh(kR) (3D), 1 for sigma = 0;
//     G(r;R) = [K0(kr) - K0(kR) I0(kr)/I0(kR)]/(2 pi) (2D),
//              sinh(k(R-r))/(4 pi r sinh(kR)) (3D); k = sqrt(sigma).
//   * Shell test d < eps; Russian roulette stops iff alpha < U, U in [0,1).
//   * Normal at the closest point: geometric normal of the closest primitive,
//     flipped so that n.(xbar - x') >= 0 (points out of the domain), x' the
//     walk's previous position (inside by at least eps; the terminal
//     position itself can lie within rounding of the boundary, where the
//     side is undecided), or the start point for a walk that starts in the
//     shell.  The
//     closest primitive is the lowest-index one among those whose squared
//     distance is within a relative 1e-12 of the minimum.
//   * Walk-length cap kmax: the kmax-th query is treated as terminal.
//   * Mapped data: udot = gdot_ref - grad_G g . V - V_n du/dn (Appendix A
//     with tangential components of the velocity kept explicitly).
//
//   * Mixed Dirichlet / zero-flux problems (Sec. 3.4, Sec. 4.4): walk on
//     stars, restated from the walk-on-stars papers the paper cites; see
//     "Walk on stars" below for the steps and the readings taken.
//
// Extension (not in the paper, which lists variance reduction and caches that
// estimate u without a walk as future work in Sec. 8 and Appendix B): a
// learned control variate for the nested walks, see "Control variate" below.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>
#include <algorithm>
#include <array>

extern "C" {

struct oracle_scene {
    int32_t dim;
    int32_t nv;
    const double* V;         // nv*dim vertex positions
    int32_t np;
    const int32_t* prims;    // np*dim vertex indices
    const int32_t* label;    // np labels (NULL: all 0)
    double sigma, eps, delta;
    int32_t K, kmax, rr;
    double src_c0;
    int32_t n_gauss;
    const double* gauss;     // n_gauss*(dim+2): amplitude, centre[dim], width
    int32_t n_labels;
    const int32_t* bc_kind;  // n_labels: 0 restricted quadratic field, 1 mapped
    const double* bc_quad;   // n_labels*(1+dim+dim*dim): c, b, A (row major)
    const double* gvert;     // nv values for mapped labels
    int32_t N;               // number of parameters
    const int64_t* rowptr;   // nv+1 CSR of dv_i/dpi_j by vertex
    const int32_t* pid;      // nnz parameter ids
    const double* vel;       // nnz*dim velocities dv_i/dpi_j
    const int32_t* bc_pid;   // nv parameter id of the mapped value, -1 none (NULL: none)
    // Reflecting (Neumann or Robin) part of the boundary: segments (2D) or
    // triangles (3D) over their own vertex array, fixed (independent of the
    // parameters).  n_ns = 0: a Dirichlet-only problem, solved by walk on
    // spheres.
    int32_t n_nv;
    const double* NV;        // n_nv*dim
    int32_t n_ns;
    const int32_t* nsegs;    // n_ns*dim vertex indices into NV
    // per query point: the reflecting primitive the point lies on, with the
    // domain on the side of its left normal (2D: to the left of the segment
    // from its first to its second vertex; 3D: the side that
    // (b - a) x (c - a) points to, a, b, c its vertices), or -1 for an
    // interior point (NULL: all interior)
    const int32_t* start_seg;
    // Implicit Dirichlet boundary (2D, Sec. 7.4): the zero set of
    // h(x) = mono_c + sum_n a_n / |x - p_n|, rows (a_n, p_n) of mono, with
    // the domain {h > 0}; n_mono = 0: the explicit boundary above.  The
    // parameters are (a_n, p_n) per monopole (N = 3 n_mono); the boundary
    // data is label 0's restricted field.
    int32_t n_mono;
    const double* mono;      // n_mono*3
    double mono_c;
    // Normal-derivative estimator of the differential walks: 0 the backward
    // difference of eq. (dudn_fd_estimate), 1 the offset-point gradient
    // estimator of eq. (dudn_mc_estimate) (Laplace only: sigma = 0, no
    // source, no reflecting or implicit boundary).
    int32_t dudn;
    // Robin condition on the reflecting boundary (eq. (mixed_bvp)):
    // du/dn - robin_mu u = h with n the normal into the domain, robin_mu >= 0
    // constant and the Robin data h the field c + b.x + x^T A x given by
    // robin_quad (1 + dim + dim*dim values; NULL: h = 0).  robin_mu = 0 and
    // no data: the zero-flux boundary.
    double robin_mu;
    const double* robin_quad;
};

// Learned control variate of the nested walks: network N(x) (frequencies B,
// F x dim, and parameters theta, see mlp_eval) and the probability q in (0, 1]
// of running the nested walks at a differential terminal.
struct oracle_cv {
    int32_t F;
    const double* B;
    const double* theta;
    double q;
};

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10.  Each round multiplies counter words 0 and 2 by two fixed
// constants, keeps the high and low halves, and mixes in the key; the key is
// advanced by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
void philox4x32_10(const uint32_t in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c[4] = {in[0], in[1], in[2], in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

// 24-bit uniform in [0, 1 - 2^-24]
double u24(uint32_t w) { return (double)(w >> 8) * 0x1p-24; }
// 24-bit uniform in (0, 1] (used for radii so that r > 0)
double u24pos(uint32_t w) { return (double)((w >> 8) + 1u) * 0x1p-24; }

// Identity of one walk's random stream: key = seed; counter =
// (step k, walk m, point p, purpose | nested index << 8 | instance << 16).
// purpose bit 1: nested walk; bit 2: second draw of a step (3D source-point
// direction; 2D takes it from the first draw's second word).
struct Stream {
    uint32_t key[2];
    uint32_t m, p, tag;
    void draw(uint32_t k, uint32_t extra, uint32_t out[4]) const {
        uint32_t ctr[4] = {k, m, p, tag | extra};
        philox4x32_10(ctr, key, out);
    }
};

// ---------------------------------------------------------------------------
// Geometry (Sec. 3.3.1 notation: closest point xbar, distance d)
// ---------------------------------------------------------------------------
struct Hit {
    double d2 = INFINITY;
    int prim = -1;
    double bary[3] = {0, 0, 0};
    double xbar[3] = {0, 0, 0};
};

double dot(const double* a, const double* b, int D) {
    double s = 0; for (int i = 0; i < D; ++i) s += a[i] * b[i]; return s;
}

void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// closest point on segment a-b to x; returns t in [0,1] with point a + t(b-a)
double seg_param(const double* x, const double* a, const double* b, int D) {
    double ab[3], ax[3];
    for (int i = 0; i < D; ++i) { ab[i] = b[i] - a[i]; ax[i] = x[i] - a[i]; }
    double L2 = dot(ab, ab, D);
    if (L2 <= 0) return 0.0;
    double t = dot(ax, ab, D) / L2;
    return std::min(1.0, std::max(0.0, t));
}

// Closest point on a triangle: if the orthogonal projection onto the plane
// falls inside (all barycentrics >= 0) that is the answer; otherwise the
// closest point lies on one of the three edges.
void tri_closest(const double* x, const double* a, const double* b, const double* c,
                 double bary[3], double q[3]) {
    double e1[3], e2[3], ax[3];
    for (int i = 0; i < 3; ++i) { e1[i] = b[i] - a[i]; e2[i] = c[i] - a[i]; ax[i] = x[i] - a[i]; }
    double d11 = dot(e1, e1, 3), d12 = dot(e1, e2, 3), d22 = dot(e2, e2, 3);
    double r1 = dot(ax, e1, 3), r2 = dot(ax, e2, 3);
    double det = d11 * d22 - d12 * d12;
    if (det > 0) {
        double s = (d22 * r1 - d12 * r2) / det;
        double t = (d11 * r2 - d12 * r1) / det;
        if (s >= 0 && t >= 0 && s + t <= 1) {
            bary[0] = 1 - s - t; bary[1] = s; bary[2] = t;
            for (int i = 0; i < 3; ++i) q[i] = a[i] + s * e1[i] + t * e2[i];
            return;
        }
    }
    const double* P[3] = {a, b, c};
    double best = INFINITY;
    for (int e = 0; e < 3; ++e) {
        const double* u = P[e];
        const double* v = P[(e + 1) % 3];
        double t = seg_param(x, u, v, 3);
        double pt[3], dd = 0;
        for (int i = 0; i < 3; ++i) { pt[i] = u[i] + t * (v[i] - u[i]); dd += (x[i] - pt[i]) * (x[i] - pt[i]); }
        if (dd < best) {
            best = dd;
            double bb[3] = {0, 0, 0};
            bb[e] = 1 - t; bb[(e + 1) % 3] = t;
            for (int i = 0; i < 3; ++i) { bary[i] = bb[i]; q[i] = pt[i]; }
        }
    }
}

struct Scene {
    const oracle_scene& s;
    int D;
    std::vector<std::vector<int>> ninc;   // 2D: reflecting segments incident to each vertex
    // 3D: the edges of the reflecting triangles, each with its incident
    // triangles (in increasing index order)
    struct Edge { int a, b; std::vector<int> f; };
    std::vector<Edge> edges;
    explicit Scene(const oracle_scene& sc) : s(sc), D(sc.dim) {
        if (sc.n_ns > 0 && D == 2) {
            ninc.assign(sc.n_nv, {});
            for (int i = 0; i < sc.n_ns; ++i)
                for (int k = 0; k < 2; ++k) ninc[sc.nsegs[2 * i + k]].push_back(i);
        }
        if (sc.n_ns > 0 && D == 3) {
            std::vector<std::array<int, 3>> e;   // (low vertex, high vertex, triangle)
            for (int i = 0; i < sc.n_ns; ++i)
                for (int k = 0; k < 3; ++k) {
                    const int u = sc.nsegs[3 * i + k], v = sc.nsegs[3 * i + (k + 1) % 3];
                    e.push_back({std::min(u, v), std::max(u, v), i});
                }
            std::sort(e.begin(), e.end());
            for (size_t j = 0; j < e.size(); ++j) {
                if (j == 0 || e[j][0] != e[j - 1][0] || e[j][1] != e[j - 1][1])
                    edges.push_back({e[j][0], e[j][1], {}});
                edges.back().f.push_back(e[j][2]);
            }
        }
    }
    const double* vert(int i) const { return s.V + (size_t)i * D; }
    int pv(int prim, int k) const { return s.prims[(size_t)prim * D + k]; }
    int lab(int prim) const { return s.label ? s.label[prim] : 0; }

    // DistanceToBoundary (Algorithm 1): brute force over all primitives.
    Hit closest(const double* x) const {
        Hit h;
        for (int p = 0; p < s.np; ++p) {
            double bary[3] = {0, 0, 0}, q[3] = {0, 0, 0};
            if (D == 2) {
                const double* a = vert(pv(p, 0));
                const double* b = vert(pv(p, 1));
                double t = seg_param(x, a, b, 2);
                bary[0] = 1 - t; bary[1] = t;
                for (int i = 0; i < 2; ++i) q[i] = a[i] + t * (b[i] - a[i]);
            } else {
                tri_closest(x, vert(pv(p, 0)), vert(pv(p, 1)), vert(pv(p, 2)), bary, q);
            }
            double d2 = 0;
            for (int i = 0; i < D; ++i) d2 += (x[i] - q[i]) * (x[i] - q[i]);
            // distances within a relative 1e-12 of each other are ties (two
            // primitives sharing an edge or vertex compute the same distance
            // with different rounding); a tie keeps the lowest index
            if (d2 < h.d2 * (1.0 - 1e-12)) {
                h.d2 = d2; h.prim = p;
                for (int i = 0; i < 3; ++i) { h.bary[i] = bary[i]; h.xbar[i] = q[i]; }
            }
        }
        return h;
    }

    // BoundaryNormal (Algorithm 2): geometric normal of the primitive,
    // oriented so that it points from the reference position x (inside the
    // domain) towards xbar, i.e. out of the domain.
    void normal(const Hit& h, const double* x, double n[3]) const {
        if (D == 2) {
            const double* a = vert(pv(h.prim, 0));
            const double* b = vert(pv(h.prim, 1));
            double tx = b[0] - a[0], ty = b[1] - a[1];
            double L = std::sqrt(tx * tx + ty * ty);
            n[0] = ty / L; n[1] = -tx / L; n[2] = 0;
        } else {
            const double* a = vert(pv(h.prim, 0));
            const double* b = vert(pv(h.prim, 1));
            const double* c = vert(pv(h.prim, 2));
            double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
            double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                            e1[0] * e2[1] - e1[1] * e2[0]};
            double L = std::sqrt(dot(cr, cr, 3));
            for (int i = 0; i < 3; ++i) n[i] = cr[i] / L;
        }
        double w[3] = {0, 0, 0};
        for (int i = 0; i < D; ++i) w[i] = h.xbar[i] - x[i];
        if (dot(n, w, D) < 0) for (int i = 0; i < 3; ++i) n[i] = -n[i];
    }

    // ----- boundary data g, its spatial gradient, and its surface gradient --
    bool mapped(int prim) const { return s.bc_kind[lab(prim)] == 1; }

    // Does the boundary at this primitive depend on a parameter (a vertex with
    // a velocity row or a parameterised value)?  Scenes without parameters
    // count as dependent everywhere.
    bool depends(int prim) const {
        if (s.N <= 0 || !s.rowptr) return true;
        for (int k = 0; k < D; ++k) {
            const int vi = pv(prim, k);
            if (s.rowptr[vi + 1] > s.rowptr[vi]) return true;
            if (s.bc_pid && s.bc_pid[vi] >= 0) return true;
        }
        return false;
    }

    double g(const Hit& h) const {
        int L = lab(h.prim);
        if (s.bc_kind[L] == 1) {
            double v = 0;
            for (int k = 0; k < D; ++k) v += h.bary[k] * s.gvert[pv(h.prim, k)];
            return v;
        }
        const double* q = s.bc_quad + (size_t)L * (1 + D + D * D);
        double v = q[0];
        for (int i = 0; i < D; ++i) v += q[1 + i] * h.xbar[i];
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) v += h.xbar[i] * q[1 + D + i * D + j] * h.xbar[j];
        return v;
    }

    // gradient of the restricted field: b + (A + A^T) x
    void grad_field(const Hit& h, double gr[3]) const {
        int L = lab(h.prim);
        const double* q = s.bc_quad + (size_t)L * (1 + D + D * D);
        for (int i = 0; i < 3; ++i) gr[i] = 0;
        for (int i = 0; i < D; ++i) {
            gr[i] = q[1 + i];
            for (int j = 0; j < D; ++j)
                gr[i] += (q[1 + D + i * D + j] + q[1 + D + j * D + i]) * h.xbar[j];
        }
    }

    // surface gradient of the linearly interpolated vertex values on a primitive
    void grad_surface(const Hit& h, double gr[3]) const {
        for (int i = 0; i < 3; ++i) gr[i] = 0;
        const double* a = vert(pv(h.prim, 0));
        const double* b = vert(pv(h.prim, 1));
        double ga = s.gvert[pv(h.prim, 0)], gb = s.gvert[pv(h.prim, 1)];
        if (D == 2) {
            double t[2] = {b[0] - a[0], b[1] - a[1]};
            double L2 = t[0] * t[0] + t[1] * t[1];
            for (int i = 0; i < 2; ++i) gr[i] = (gb - ga) * t[i] / L2;
        } else {
            const double* c = vert(pv(h.prim, 2));
            double gc = s.gvert[pv(h.prim, 2)];
            double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
            double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            // gradient lies in the plane: gr = alpha e1 + beta e2 with
            // gr.e1 = gb - ga, gr.e2 = gc - ga
            double d11 = dot(e1, e1, 3), d12 = dot(e1, e2, 3), d22 = dot(e2, e2, 3);
            double det = d11 * d22 - d12 * d12;
            double r1 = gb - ga, r2 = gc - ga;
            double al = (d22 * r1 - d12 * r2) / det;
            double be = (d11 * r2 - d12 * r1) / det;
            for (int i = 0; i < 3; ++i) gr[i] = al * e1[i] + be * e2[i];
        }
    }

    // source f(y)
    double f(const double* y) const {
        double v = s.src_c0;
        for (int i = 0; i < s.n_gauss; ++i) {
            const double* r = s.gauss + (size_t)i * (D + 2);
            double d2 = 0;
            for (int k = 0; k < D; ++k) d2 += (y[k] - r[1 + k]) * (y[k] - r[1 + k]);
            v += r[0] * std::exp(-d2 / (2 * r[1 + D] * r[1 + D]));
        }
        return v;
    }
    bool has_source() const { return s.src_c0 != 0.0 || s.n_gauss > 0; }

    // ----- implicit boundary (harmonic monopoles) ---------------------------
    bool implicit() const { return s.n_mono > 0; }

    // h and its gradient at x
    double hval(const double* x, double gr[2]) const {
        double h = s.mono_c;
        gr[0] = gr[1] = 0;
        for (int n = 0; n < s.n_mono; ++n) {
            const double* m = s.mono + 3 * n;
            const double dx = x[0] - m[1], dy = x[1] - m[2];
            const double r = std::sqrt(dx * dx + dy * dy);
            h += m[0] / r;
            const double q = m[0] / (r * r * r);
            gr[0] -= q * dx;
            gr[1] -= q * dy;
        }
        return h;
    }

    // Radius of a disk around x (h(x) > 0) on which h > 0, from Harnack's
    // inequality: 1/|y - p| is harmonic in 3D, so f = h - c > 0 (all a_n > 0)
    // is a positive harmonic function on the 3D ball of radius R = distance
    // to the nearest pole, and f(y) >= f(x) R (R - r) / (R + r)^2 at distance
    // r.  h stays positive while that bound exceeds -c = A: with t = r / R,
    // A (1 + t)^2 = f (1 - t), whose root in [0, 1) is
    // t = 2 (f - A) / ((2A + f) + sqrt(f^2 + 8 A f)).  The planar disk is a
    // cross-section of the ball.
    double harnack_radius(const double* x, double h) const {
        double R = INFINITY;
        for (int n = 0; n < s.n_mono; ++n) {
            const double* m = s.mono + 3 * n;
            R = std::min(R, std::hypot(x[0] - m[1], x[1] - m[2]));
        }
        const double A = -s.mono_c, f = h - s.mono_c;
        const double t = 2 * (f - A) / ((2 * A + f) + std::sqrt(f * f + 8 * A * f));
        return t * R;
    }

    // Radius of a disk around x on which h > 0: the larger of the Harnack
    // radius above and a direct bound.  With every a_n > 0, each monopole
    // term on B(x, d) is at least a_n / (|x - p_n| + d), so h > 0 there while
    // S(d) = sum_n a_n / (|x - p_n| + d) > -c.  1/S is the parallel sum of
    // the linear functions (|x - p_n| + d) / a_n, hence increasing and
    // concave, so Newton's iterates for 1/S(d) = -1/c from d = 0 rise
    // monotonically towards the root and each is a safe radius; eight are
    // taken (one is exact for a single monopole).  The direct bound is not
    // limited by the distance to a pole, as the Harnack radius is.
    double safe_radius(const double* x, double h) const {
        const double A = -s.mono_c;
        double d = 0;
        for (int it = 0; it < 8; ++it) {
            double S = 0, T = 0;
            for (int n = 0; n < s.n_mono; ++n) {
                const double* m = s.mono + 3 * n;
                const double q = std::hypot(x[0] - m[1], x[1] - m[2]) + d;
                S += m[0] / q;
                T += m[0] / (q * q);
            }
            // (1/S)' = T / S^2:  d += (1/A - 1/S) S^2 / T
            d += (S * S / A - S) / T;
        }
        return std::max(d, harnack_radius(x, h));
    }

    // The shell of Sec. 7.4, h <= |grad h| eps (which takes in points at or
    // past the zero set), applied only where h < -c: next to a pole |grad h|
    // grows faster than h and the test would hold far from the boundary.
    bool in_shell(double h, double gn) const { return h <= gn * s.eps && h < -s.mono_c; }

    // dh/dpi_j at x for pi = (a_n, p_n) per monopole
    void hparam(const double* x, double* dh) const {
        for (int n = 0; n < s.n_mono; ++n) {
            const double* m = s.mono + 3 * n;
            const double dx = x[0] - m[1], dy = x[1] - m[2];
            const double r = std::sqrt(dx * dx + dy * dy);
            dh[3 * n] = 1 / r;
            dh[3 * n + 1] = m[0] * dx / (r * r * r);
            dh[3 * n + 2] = m[0] * dy / (r * r * r);
        }
    }

    // restricted data of label 0 and its gradient at a point
    double g_field(const double* x, double gr[3]) const {
        const int D = 2;
        const double* q = s.bc_quad;
        double v = q[0];
        for (int i = 0; i < D; ++i) v += q[1 + i] * x[i];
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) v += x[i] * q[1 + D + i * D + j] * x[j];
        gr[0] = gr[1] = gr[2] = 0;
        for (int i = 0; i < D; ++i) {
            gr[i] = q[1 + i];
            for (int j = 0; j < D; ++j) gr[i] += (q[1 + D + i * D + j] + q[1 + D + j * D + i]) * x[j];
        }
        return v;
    }

    // ----- reflecting boundary (walk on stars) ------------------------------
    bool has_neumann() const { return s.n_ns > 0; }
    const double* nvert(int i) const { return s.NV + (size_t)i * D; }
    int nsv(int seg, int k) const { return s.nsegs[(size_t)D * seg + k]; }

    // Unit left normal of a reflecting primitive (the domain side of a start
    // primitive): 2D the segment's tangent turned by +90 degrees, 3D
    // (b - a) x (c - a) normalised.
    void nleft(int seg, double n[3]) const {
        const double* a = nvert(nsv(seg, 0));
        const double* b = nvert(nsv(seg, 1));
        if (D == 2) {
            double tx = b[0] - a[0], ty = b[1] - a[1], L = std::sqrt(tx * tx + ty * ty);
            n[0] = -ty / L; n[1] = tx / L; n[2] = 0;
            return;
        }
        const double* c = nvert(nsv(seg, 2));
        const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double cr[3];
        cross3(e1, e2, cr);
        const double L = std::sqrt(dot(cr, cr, 3));
        for (int i = 0; i < 3; ++i) n[i] = cr[i] / L;
    }

    // Area of reflecting triangle i (3D).
    double tri_area(int i) const {
        const double* a = nvert(nsv(i, 0));
        const double* b = nvert(nsv(i, 1));
        const double* c = nvert(nsv(i, 2));
        const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double cr[3];
        cross3(e1, e2, cr);
        return 0.5 * std::sqrt(dot(cr, cr, 3));
    }

    // Is the edge of reflecting triangles (3D) a silhouette as seen from x?
    // The 3D form of the vertex rule below: seen from x the surface turns
    // back at the edge when both triangles at it lie on the same side of the
    // plane through x and the edge.  An edge with one triangle (a rim) or
    // more than two is always counted.  A triangle seen edge-on (x in its
    // plane) does not decide: if x lies on reflecting triangle `on` (domain
    // side `nin`), an edge of `on` is a silhouette when the other triangle
    // at it leaves to the outside of the plane of `on`; otherwise an edge
    // whose triangles are both edge-on is not a silhouette (a flat part of
    // the surface containing x), and one with a single edge-on triangle is
    // decided by the other triangle's side of the plane of `on` (x on a
    // wall) or counted (x inside, a null set of points).
    bool silhouette_edge(const Edge& e, const double* x, int on, const double* nin) const {
        if (e.f.size() != 2) return true;
        const double* p = nvert(e.a);
        const double* q = nvert(e.b);
        int w[2];
        for (int k = 0; k < 2; ++k) {
            w[k] = -1;
            for (int j = 0; j < 3; ++j) {
                const int v = nsv(e.f[k], j);
                if (v != e.a && v != e.b) w[k] = v;
            }
        }
        auto outside = [&](int v) {
            const double* pw = nvert(v);
            return nin[0] * (pw[0] - p[0]) + nin[1] * (pw[1] - p[1]) + nin[2] * (pw[2] - p[2]) < 0;
        };
        if (on >= 0 && e.f[0] == on) return outside(w[1]);
        if (on >= 0 && e.f[1] == on) return outside(w[0]);
        const double t[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
        const double r[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
        double m[3];
        cross3(t, r, m);   // normal of the plane through the edge and x
        const double lm = std::sqrt(dot(m, m, 3));
        double c[2];
        bool zero[2];
        for (int k = 0; k < 2; ++k) {
            const double* pw = nvert(w[k]);
            const double d[3] = {pw[0] - p[0], pw[1] - p[1], pw[2] - p[2]};
            c[k] = dot(m, d, 3);
            zero[k] = std::fabs(c[k]) <= 1e-10 * lm * std::sqrt(dot(d, d, 3));
        }
        if (zero[0] && zero[1]) return false;
        if (zero[0] || zero[1]) return on >= 0 ? outside(zero[0] ? w[1] : w[0]) : true;
        return (c[0] > 0) == (c[1] > 0);
    }

    // Is reflecting vertex v a silhouette point as seen from x?  Seen from x,
    // the boundary turns back at v when both edges at v leave it on the same
    // side of the line through x and v.  A vertex with one edge (an open end)
    // or more than two is always counted.  An edge seen edge-on (x on its
    // line) does not decide: if x lies on the reflecting boundary (segment
    // `on`, domain side `nin`), v is a silhouette when its other edge leaves
    // to the outside of that line; the edges at v that are the segment x lies
    // on are edge-on by construction.  Off the boundary an edge-on view counts
    // as a silhouette (a conservative choice for a null set of points).
    bool silhouette(int v, const double* x, int on, const double* nin) const {
        const std::vector<int>& e = ninc[v];
        if (e.size() != 2) return true;
        const double* pv = nvert(v);
        int nb[2];
        for (int k = 0; k < 2; ++k) nb[k] = nsv(e[k], 0) == v ? nsv(e[k], 1) : nsv(e[k], 0);
        auto outside = [&](int w) {
            const double* pw = nvert(w);
            return nin[0] * (pw[0] - pv[0]) + nin[1] * (pw[1] - pv[1]) < 0;
        };
        if (on >= 0 && e[0] == on) return outside(nb[1]);
        if (on >= 0 && e[1] == on) return outside(nb[0]);
        const double vx = pv[0] - x[0], vy = pv[1] - x[1];
        const double lv = std::sqrt(vx * vx + vy * vy);
        double c[2];
        bool zero[2];
        for (int k = 0; k < 2; ++k) {
            const double* pw = nvert(nb[k]);
            const double ex = pw[0] - pv[0], ey = pw[1] - pv[1];
            c[k] = vx * ey - vy * ex;
            zero[k] = std::fabs(c[k]) <= 1e-10 * lv * std::sqrt(ex * ex + ey * ey);
        }
        if (zero[0] && zero[1]) return false;
        if (zero[0] || zero[1]) return on >= 0 ? outside(zero[0] ? nb[1] : nb[0]) : true;
        return (c[0] > 0) == (c[1] > 0);
    }

    // Squared distance from x to its closest silhouette point, capped at cap2
    // (3D: the closest point of the silhouette edges).
    double silhouette_d2(const double* x, int on, const double* nin, double cap2) const {
        double best = cap2;
        if (D == 3) {
            for (const Edge& e : edges) {
                const double* p = nvert(e.a);
                const double* q = nvert(e.b);
                const double t = seg_param(x, p, q, 3);
                double d2 = 0;
                for (int i = 0; i < 3; ++i) {
                    const double di = p[i] + t * (q[i] - p[i]) - x[i];
                    d2 += di * di;
                }
                if (d2 < best && silhouette_edge(e, x, on, nin)) best = d2;
            }
            return best;
        }
        for (int v = 0; v < s.n_nv; ++v) {
            if (ninc[v].empty()) continue;
            const double* p = nvert(v);
            double d2 = (p[0] - x[0]) * (p[0] - x[0]) + (p[1] - x[1]) * (p[1] - x[1]);
            if (d2 < best && silhouette(v, x, on, nin)) best = d2;
        }
        return best;
    }

    // First intersection of the ray x + t dir, 0 < t < tmax, with a
    // reflecting segment other than `skip`.  Returns the segment (lowest
    // index on a tie) or -1, and its t.
    int ray(const double* x, const double* dir, double tmax, int skip, double& t_out) const {
        int hit = -1;
        double best = tmax;
        if (D == 3) {
            // Moller-Trumbore: x + t dir = a + u e1 + v e2 with u, v >= 0,
            // u + v <= 1 (a direction parallel to the triangle misses it)
            for (int i = 0; i < s.n_ns; ++i) {
                if (i == skip) continue;
                const double* a = nvert(nsv(i, 0));
                const double* b = nvert(nsv(i, 1));
                const double* c = nvert(nsv(i, 2));
                const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
                const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
                double pv[3];
                cross3(dir, e2, pv);
                const double det = dot(e1, pv, 3);
                if (det == 0.0) continue;
                const double tv[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]};
                const double u = dot(tv, pv, 3) / det;
                if (u < 0 || u > 1) continue;
                double qv[3];
                cross3(tv, e1, qv);
                const double v = dot(dir, qv, 3) / det;
                if (v < 0 || u + v > 1) continue;
                const double t = dot(e2, qv, 3) / det;
                if (t > 0 && t < best) { best = t; hit = i; }
            }
            t_out = hit >= 0 ? best : tmax;
            return hit;
        }
        for (int i = 0; i < s.n_ns; ++i) {
            if (i == skip) continue;
            const double* a = nvert(nsv(i, 0));
            const double* b = nvert(nsv(i, 1));
            const double ex = b[0] - a[0], ey = b[1] - a[1];
            const double den = dir[0] * ey - dir[1] * ex;        // cross(dir, e)
            if (den == 0.0) continue;                            // parallel
            const double ax = a[0] - x[0], ay = a[1] - x[1];
            const double t = (ax * ey - ay * ex) / den;          // cross(a - x, e) / den
            const double u = (ax * dir[1] - ay * dir[0]) / den;  // cross(a - x, dir) / den
            if (t > 0 && t < best && u >= 0 && u <= 1) { best = t; hit = i; }
        }
        t_out = hit >= 0 ? best : tmax;
        return hit;
    }

    // ----- Robin condition on the reflecting boundary -----------------------
    bool has_robin() const { return s.robin_mu > 0 || s.robin_quad != nullptr; }

    // the Robin data h at a boundary point
    double robin_h(const double* z) const {
        if (!s.robin_quad) return 0.0;
        const double* q = s.robin_quad;
        double v = q[0];
        for (int i = 0; i < D; ++i) v += q[1 + i] * z[i];
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) v += z[i] * q[1 + D + i * D + j] * z[j];
        return v;
    }

    // Parameter interval [t0, t1] of the part of reflecting segment i inside
    // the disk |z - x| < R (t along the segment from its first vertex);
    // returns its length (0: the segment misses the disk).
    double clip(int i, const double* x, double R, double& t0, double& t1) const {
        const double* a = nvert(nsv(i, 0));
        const double* b = nvert(nsv(i, 1));
        const double ex = b[0] - a[0], ey = b[1] - a[1];
        const double ax = a[0] - x[0], ay = a[1] - x[1];
        const double ee = ex * ex + ey * ey, ea = ex * ax + ey * ay;
        const double disc = ea * ea - ee * (ax * ax + ay * ay - R * R);
        if (!(disc > 0)) return 0.0;
        const double sq = std::sqrt(disc);
        t0 = std::max(0.0, (-ea - sq) / ee);
        t1 = std::min(1.0, (-ea + sq) / ee);
        if (!(t1 > t0)) return 0.0;
        return std::sqrt(ee) * (t1 - t0);
    }

    // A point z uniform by length on the reflecting boundary inside the disk
    // B(x, R), and that length L (seg = -1, L = 0 when the disk holds none).
    // The segment is chosen with probability proportional to its clipped
    // length by an exponential race -- segment i draws E_i = -ln(U_i) / l_i
    // and the smallest E_i wins -- with U_i from its own Philox counter
    // (k, m, p, tag | 8 | i << 16), so the choice does not depend on the
    // order in which segments are visited; the position along the winner's
    // clipped part is word 1 of the same draw.
    //
    // 3D: the triangles that reach into the ball B(x, R) (closest point
    // nearer than R) with their whole areas A_i; L = sum A_i and the race
    // with weights A_i picks a triangle, z is uniform on it (words 1 and 2
    // of the winner's draw: with r = sqrt(U1), z = (1 - r) a + r (1 - U2) b
    // + r U2 c).  A z outside the ball returns -1 (it adds nothing): the
    // expected value of L 1(z in B) phi(z) is the integral of phi over the
    // reflecting boundary inside the ball, as with the clipped lengths in
    // 2D.  branch (3D) gets word 3 of the winner's draw, a uniform word
    // independent of the choice, for the Robin branch of the step.
    int boundary_sample(const double* x, double R, const Stream& st, uint32_t k, uint32_t extra,
                        double& L, double z[3], uint32_t* branch = nullptr) const {
        L = 0.0;
        if (D == 3) {
            int win = -1;
            double best = INFINITY;
            uint32_t ww[4] = {0, 0, 0, 0};
            for (int i = 0; i < s.n_ns; ++i) {
                double bary[3], q[3];
                tri_closest(x, nvert(nsv(i, 0)), nvert(nsv(i, 1)), nvert(nsv(i, 2)), bary, q);
                double d2 = 0;
                for (int j = 0; j < 3; ++j) d2 += (q[j] - x[j]) * (q[j] - x[j]);
                if (!(d2 < R * R)) continue;
                const double A = tri_area(i);
                L += A;
                uint32_t w[4];
                st.draw(k, extra | 8u | ((uint32_t)i << 16), w);
                const double e = -std::log(u24pos(w[0])) / A;
                if (e < best) { best = e; win = i; for (int j = 0; j < 4; ++j) ww[j] = w[j]; }
            }
            if (win < 0) return -1;
            const double* a = nvert(nsv(win, 0));
            const double* b = nvert(nsv(win, 1));
            const double* c = nvert(nsv(win, 2));
            const double r = std::sqrt(u24(ww[1])), t = u24(ww[2]);
            double d2 = 0;
            for (int j = 0; j < 3; ++j) {
                z[j] = (1 - r) * a[j] + r * (1 - t) * b[j] + r * t * c[j];
                d2 += (z[j] - x[j]) * (z[j] - x[j]);
            }
            if (branch) *branch = ww[3];
            return d2 < R * R ? win : -1;
        }
        int win = -1;
        double best = INFINITY, wt0 = 0, wt1 = 0;
        uint32_t wpos = 0;
        for (int i = 0; i < s.n_ns; ++i) {
            double t0 = 0, t1 = 0;
            const double l = clip(i, x, R, t0, t1);
            if (!(l > 0)) continue;
            L += l;
            uint32_t w[4];
            st.draw(k, extra | 8u | ((uint32_t)i << 16), w);
            const double e = -std::log(u24pos(w[0])) / l;
            if (e < best) { best = e; win = i; wt0 = t0; wt1 = t1; wpos = w[1]; }
        }
        if (win >= 0) {
            const double* a = nvert(nsv(win, 0));
            const double* b = nvert(nsv(win, 1));
            const double t = wt0 + u24(wpos) * (wt1 - wt0);
            z[0] = a[0] + t * (b[0] - a[0]);
            z[1] = a[1] + t * (b[1] - a[1]);
        }
        return win;
    }
};

// ---------------------------------------------------------------------------
// Green's function and Poisson kernel of the ball (Sec. 3.3.1)
// ---------------------------------------------------------------------------
double ball_volume(int D, double R) { return D == 2 ? M_PI * R * R : 4.0 / 3.0 * M_PI * R * R * R; }

// alpha = P(R) / p^dB(R): the recursive contribution scale of Algorithm 1.
double poisson_scale(int D, double sigma, double R) {
    if (sigma == 0.0) return 1.0;
    double k = std::sqrt(sigma);
    if (D == 2) return 1.0 / std::cyl_bessel_i(0.0, k * R);
    return k * R / std::sinh(k * R);
}

// G(r; R) of the zero-Dirichlet screened Poisson problem on the ball.
double green(int D, double sigma, double r, double R) {
    if (D == 2) {
        if (sigma == 0.0) return std::log(R / r) / (2 * M_PI);
        double k = std::sqrt(sigma);
        double I0r = std::cyl_bessel_i(0.0, k * r), I0R = std::cyl_bessel_i(0.0, k * R);
        double K0r = std::cyl_bessel_k(0.0, k * r), K0R = std::cyl_bessel_k(0.0, k * R);
        return (K0r - K0R * I0r / I0R) / (2 * M_PI);
    }
    if (sigma == 0.0) return (1.0 / r - 1.0 / R) / (4 * M_PI);
    double k = std::sqrt(sigma);
    return std::sinh(k * (R - r)) / (4 * M_PI * r * std::sinh(k * R));
}

// Mass of the Green's function over the ball, int_B G dy = (1 - Q(R))/sigma
// (R^2/(2D) at sigma = 0): the expected source integral of one step for a
// unit source.  1 - Q is summed from its power series where Q is close to 1:
//   2D: 1 - 1/I0(x) = (I0(x) - 1)/I0(x),  I0(x) - 1 = sum_{k>=1} (x^2/4)^k/(k!)^2
//   3D: 1 - x/sinh x = (sinh x - x)/sinh x,  sinh x - x = sum_{k>=1} x^(2k+1)/(2k+1)!
double green_mass(int D, double sigma, double R) {
    if (sigma == 0.0) return R * R / (2 * D);
    const double x = std::sqrt(sigma) * R;
    if (D == 2) {
        if (x < 2.0) {
            double t = 1, s = 0;
            for (int k = 1; k <= 40; ++k) { t *= (x * x / 4) / ((double)k * k); s += t; }
            return s / ((1 + s) * sigma);
        }
        return (1 - 1 / std::cyl_bessel_i(0.0, x)) / sigma;
    }
    if (x < 1.0) {
        double t = x, s = 0;
        for (int k = 1; k <= 20; ++k) { t *= x * x / ((2.0 * k) * (2.0 * k + 1)); s += t; }
        return s / (std::sinh(x) * sigma);
    }
    return (1 - x / std::sinh(x)) / sigma;
}

// Uniform directions and ball points from 24-bit uniforms.
void sphere_dir(int D, uint32_t w0, uint32_t w1, double s[3]) {
    if (D == 2) {
        double th = 2 * M_PI * u24(w0);
        s[0] = std::cos(th); s[1] = std::sin(th); s[2] = 0;
    } else {
        double z = 1 - 2 * u24(w0);
        double ph = 2 * M_PI * u24(w1);
        double rho = std::sqrt(std::max(0.0, 1 - z * z));
        s[0] = rho * std::cos(ph); s[1] = rho * std::sin(ph); s[2] = z;
    }
}

// Walk on stars (reflecting boundary): weight of a step that ends on the
// reflecting boundary at distance r < R inside the ball of radius R.  The
// boundary integral over the star-shaped region carries the Poisson kernel
// -dG/dn_z of the ball at the boundary point z; the density of z under
// uniform direction sampling is |n_z.(z - x)| / (|dS_1| r^D), so the ratio is
//   |dS_1| r^(D-1) |dG/dr|(r; R)
// with |dS_1| = 2 pi (2D) or 4 pi (3D) and G from green():
//   2D: kr [K1(kr) + K0(kR) I1(kr) / I0(kR)]
//   3D: [kr cosh(k(R - r)) + sinh(k(R - r))] / sinh(kR)
// It equals poisson_scale at r = R, tends to 1 as r -> 0, and is 1 for
// sigma = 0.  A walk at a reflecting boundary point samples the half of the
// directions that enter the domain, with twice the density, and the boundary
// integral equation there carries a factor 1/2 on the left (the solid-angle
// fraction of a smooth boundary point), so the weights are unchanged.
double neumann_weight(int D, double sigma, double r, double R) {
    if (sigma == 0.0) return 1.0;
    const double k = std::sqrt(sigma);
    if (D == 2) {
        const double a = k * r, b = k * R;
        return a * (std::cyl_bessel_k(1.0, a) +
                    std::cyl_bessel_k(0.0, b) * std::cyl_bessel_i(1.0, a) / std::cyl_bessel_i(0.0, b));
    }
    return (k * r * std::cosh(k * (R - r)) + std::sinh(k * (R - r))) / std::sinh(k * R);
}

// ---------------------------------------------------------------------------
// The control-variate network (an extension; see the file header).
//   gamma(x) = [sin(2 pi B x) (F), cos(2 pi B x) (F), x (dim), 0 ...]  (64)
//   a_1 = tanh(W_1 gamma + b_1), a_l = tanh(W_l a_{l-1} + b_l), l = 2..4 (64)
//   N(x) = w_5 . a_4 + b_5
// theta holds, for l = 1..4, W_l (64 x 64, row = output unit) then b_l (64),
// followed by w_5 (64) and b_5: 16705 values.
// ---------------------------------------------------------------------------
constexpr int kWidth = 64;
constexpr int kLayers = 4;
constexpr int kLayerSize = kWidth * kWidth + kWidth;
constexpr int kThetaSize = kLayers * kLayerSize + kWidth + 1;

struct MlpOut {
    double N = 0;
    double grad[3] = {0, 0, 0};
    double lap = 0;
};

// Input features with their spatial gradients and Laplacians.
void mlp_features(int D, int F, const double* B, const double* x, double v[kWidth],
                  double g[kWidth][3], double L[kWidth]) {
    for (int f = 0; f < kWidth; ++f) {
        v[f] = 0; L[f] = 0;
        for (int c = 0; c < 3; ++c) g[f][c] = 0;
    }
    for (int i = 0; i < F; ++i) {
        const double* b = B + (size_t)i * D;
        double th = 0, bb = 0;
        for (int c = 0; c < D; ++c) { th += 2 * M_PI * b[c] * x[c]; bb += b[c] * b[c]; }
        double sn = std::sin(th), cs = std::cos(th);
        double w2 = 4 * M_PI * M_PI * bb;
        v[i] = sn; v[F + i] = cs;
        for (int c = 0; c < D; ++c) {
            g[i][c] = 2 * M_PI * b[c] * cs;
            g[F + i][c] = -2 * M_PI * b[c] * sn;
        }
        L[i] = -w2 * sn; L[F + i] = -w2 * cs;
    }
    for (int c = 0; c < D; ++c) { v[2 * F + c] = x[c]; g[2 * F + c][c] = 1; }
}

// N, grad N and Lap N at x: the value, the dim first derivatives and the
// Laplacian are carried through every layer (chain rule; for h = tanh z,
// h' = 1 - h^2 and h'' = -2 h (1 - h^2)).
MlpOut mlp_eval(int D, int F, const double* B, const double* theta, const double* x) {
    double v[kWidth], g[kWidth][3], L[kWidth];
    mlp_features(D, F, B, x, v, g, L);
    for (int l = 0; l < kLayers; ++l) {
        const double* W = theta + (size_t)l * kLayerSize;
        const double* b = W + kWidth * kWidth;
        double nv[kWidth], ng[kWidth][3], nL[kWidth];
        for (int o = 0; o < kWidth; ++o) {
            double z = b[o], zL = 0, zg[3] = {0, 0, 0};
            for (int i = 0; i < kWidth; ++i) {
                double w = W[o * kWidth + i];
                z += w * v[i];
                zL += w * L[i];
                for (int c = 0; c < D; ++c) zg[c] += w * g[i][c];
            }
            double h = std::tanh(z), s = 1 - h * h, zz = 0;
            for (int c = 0; c < D; ++c) zz += zg[c] * zg[c];
            nv[o] = h;
            for (int c = 0; c < 3; ++c) ng[o][c] = c < D ? s * zg[c] : 0;
            nL[o] = s * zL - 2 * h * s * zz;
        }
        std::memcpy(v, nv, sizeof v); std::memcpy(g, ng, sizeof g); std::memcpy(L, nL, sizeof L);
    }
    const double* w5 = theta + (size_t)kLayers * kLayerSize;
    MlpOut out;
    out.N = w5[kWidth];
    for (int i = 0; i < kWidth; ++i) {
        out.N += w5[i] * v[i];
        out.lap += w5[i] * L[i];
        for (int c = 0; c < D; ++c) out.grad[c] += w5[i] * g[i][c];
    }
    return out;
}

// Squared-error training loss sum_i 1/2 w_i (N(x_i) - t_i)^2 and its gradient
// with respect to theta (reverse mode through the layers above).
double mlp_loss_grad(int D, int F, const double* B, const double* theta, const double* X,
                     const double* T, const double* Wt, int64_t n, double* grad) {
    double loss = 0;
    for (int64_t s = 0; s < n; ++s) {
        double a[kLayers + 1][kWidth], gdum[kWidth][3], Ldum[kWidth];
        mlp_features(D, F, B, X + s * D, a[0], gdum, Ldum);
        for (int l = 0; l < kLayers; ++l) {
            const double* W = theta + (size_t)l * kLayerSize;
            const double* b = W + kWidth * kWidth;
            for (int o = 0; o < kWidth; ++o) {
                double z = b[o];
                for (int i = 0; i < kWidth; ++i) z += W[o * kWidth + i] * a[l][i];
                a[l + 1][o] = std::tanh(z);
            }
        }
        const double* w5 = theta + (size_t)kLayers * kLayerSize;
        double N = w5[kWidth];
        for (int i = 0; i < kWidth; ++i) N += w5[i] * a[kLayers][i];
        double w = Wt ? Wt[s] : 1.0;
        double r = w * (N - T[s]);
        loss += 0.5 * w * (N - T[s]) * (N - T[s]);
        double* gw5 = grad + (size_t)kLayers * kLayerSize;
        double delta[kWidth];
        for (int i = 0; i < kWidth; ++i) {
            gw5[i] += r * a[kLayers][i];
            delta[i] = r * w5[i] * (1 - a[kLayers][i] * a[kLayers][i]);
        }
        gw5[kWidth] += r;
        for (int l = kLayers - 1; l >= 0; --l) {
            const double* W = theta + (size_t)l * kLayerSize;
            double* gW = grad + (size_t)l * kLayerSize;
            double* gb = gW + kWidth * kWidth;
            for (int o = 0; o < kWidth; ++o) {
                gb[o] += delta[o];
                for (int i = 0; i < kWidth; ++i) gW[o * kWidth + i] += delta[o] * a[l][i];
            }
            if (l == 0) break;
            double prev[kWidth];
            for (int i = 0; i < kWidth; ++i) {
                double acc = 0;
                for (int o = 0; o < kWidth; ++o) acc += W[o * kWidth + i] * delta[o];
                prev[i] = acc * (1 - a[l][i] * a[l][i]);
            }
            std::memcpy(delta, prev, sizeof delta);
        }
    }
    return loss;
}

// Vector-Jacobian product through the value and Laplacian of the network:
// grad += d/dtheta sum_i (Nbar_i N(x_i) + Lbar_i Lap N(x_i)).  The forward
// pass keeps, per layer, the pre-activation value z, its spatial gradient
// z_c and Laplacian z_L; with h = tanh z, s = 1 - h^2, Q = sum_c z_c^2 the
// layer outputs are (h, s z_c, s z_L - 2 h s Q), whose adjoints give
//   zbar_L = s abar_L
//   zbar_c = s abar_c - 4 h s z_c abar_L
//   zbar   = s abar - 2 h s sum_c z_c abar_c - (2 h s z_L + 2 s (s - 2 h^2) Q) abar_L
// and every channel goes back through W^T.
void mlp_vjp(int D, int F, const double* B, const double* theta, const double* x, double Nbar,
             double Lbar, double* grad) {
    constexpr int NC = 5;   // value, 3 gradient components, Laplacian
    double a[kLayers + 1][NC][kWidth] = {};
    double z[kLayers][NC][kWidth] = {};
    {
        double v[kWidth], g[kWidth][3], L[kWidth];
        mlp_features(D, F, B, x, v, g, L);
        for (int i = 0; i < kWidth; ++i) {
            a[0][0][i] = v[i];
            for (int c = 0; c < 3; ++c) a[0][1 + c][i] = g[i][c];
            a[0][4][i] = L[i];
        }
    }
    for (int l = 0; l < kLayers; ++l) {
        const double* W = theta + (size_t)l * kLayerSize;
        const double* b = W + kWidth * kWidth;
        for (int o = 0; o < kWidth; ++o) {
            for (int ch = 0; ch < NC; ++ch) {
                double acc = ch == 0 ? b[o] : 0.0;
                for (int i = 0; i < kWidth; ++i) acc += W[o * kWidth + i] * a[l][ch][i];
                z[l][ch][o] = acc;
            }
            double h = std::tanh(z[l][0][o]), s = 1 - h * h, Q = 0;
            for (int c = 0; c < D; ++c) Q += z[l][1 + c][o] * z[l][1 + c][o];
            a[l + 1][0][o] = h;
            for (int c = 0; c < 3; ++c) a[l + 1][1 + c][o] = c < D ? s * z[l][1 + c][o] : 0.0;
            a[l + 1][4][o] = s * z[l][4][o] - 2 * h * s * Q;
        }
    }
    const double* w5 = theta + (size_t)kLayers * kLayerSize;
    double* gw5 = grad + (size_t)kLayers * kLayerSize;
    double abar[NC][kWidth] = {};
    for (int i = 0; i < kWidth; ++i) {
        gw5[i] += Nbar * a[kLayers][0][i] + Lbar * a[kLayers][4][i];
        abar[0][i] = Nbar * w5[i];
        abar[4][i] = Lbar * w5[i];
    }
    gw5[kWidth] += Nbar;
    for (int l = kLayers - 1; l >= 0; --l) {
        const double* W = theta + (size_t)l * kLayerSize;
        double* gW = grad + (size_t)l * kLayerSize;
        double* gb = gW + kWidth * kWidth;
        double zbar[NC][kWidth] = {};
        for (int o = 0; o < kWidth; ++o) {
            double h = std::tanh(z[l][0][o]), s = 1 - h * h, Q = 0, za = 0;
            for (int c = 0; c < D; ++c) {
                Q += z[l][1 + c][o] * z[l][1 + c][o];
                za += z[l][1 + c][o] * abar[1 + c][o];
            }
            zbar[4][o] = s * abar[4][o];
            for (int c = 0; c < D; ++c) zbar[1 + c][o] = s * abar[1 + c][o] - 4 * h * s * z[l][1 + c][o] * abar[4][o];
            zbar[0][o] = s * abar[0][o] - 2 * h * s * za -
                         (2 * h * s * z[l][4][o] + 2 * s * (s - 2 * h * h) * Q) * abar[4][o];
            gb[o] += zbar[0][o];
            for (int ch = 0; ch < NC; ++ch)
                for (int i = 0; i < kWidth; ++i) gW[o * kWidth + i] += zbar[ch][o] * a[l][ch][i];
        }
        if (l == 0) break;
        for (int ch = 0; ch < NC; ++ch)
            for (int i = 0; i < kWidth; ++i) {
                double acc = 0;
                for (int o = 0; o < kWidth; ++o) acc += W[o * kWidth + i] * zbar[ch][o];
                abar[ch][i] = acc;
            }
    }
}

// ---------------------------------------------------------------------------
// Control variate of a nested walk.  For any twice differentiable N, applying
// the ball's mean-value identity for the screened operator (Sec. 3.3: the
// Poisson-kernel average of N on the sphere plus the Green's-function integral
// of -Lap N + sigma N over the ball) at every step of Algorithm 1 gives
//   N(x_0) = E[ sum over source steps j of  int_{B_j} G_j (-Lap N + sigma N)
//               + [the walk ended in the shell or at the cap] N(x_stop) ],
// with the same stopping rules (shell, roulette, cap) as the walk.  So
//   C = N(x_0) - sum_j int_{B_j} G_j (-Lap N + sigma N) - [alive] N(x_stop)
// has mean zero, and uhat + C is an estimate of u(x_0) with the same mean as
// uhat; its variance vanishes as N approaches u.  The sum over the source
// steps is estimated by one step J chosen with probability m_J / S, where
// m_j = int_{B_j} G_j is the Green's-function mass of step j's ball and S the
// walk's total (weighted reservoir sampling as the walk proceeds: step j
// replaces the choice iff U S_j < m_j with S_j the running total), and one
// uniform point y_J of B_J:
//   sum_j ~ S |B_J| G_J(|y_J - x_J|) (-Lap N + sigma N)(y_J) / m_J.
// For a residual -Lap N + sigma N that is constant along the walk the
// estimate is exact up to the ball-point weight.
// ---------------------------------------------------------------------------
struct CvTrace {
    double S = 0;          // total Green's-function mass of the source steps
    bool alive = false;    // ended in the shell or at the cap (not by roulette)
    double xstop[3] = {0, 0, 0};
    double y[3] = {0, 0, 0};
    double rho = 0, d = 0; // y = x_J + rho d dir, rho in (0, 1], d = radius of B_J
    bool any = false;      // at least one source step
};

// 24-bit threshold of the probability q: the nested walks run iff the top 24
// bits of a uniform word are below it.
uint32_t cv_threshold(double q) {
    double t = std::round(q * 16777216.0);
    if (t < 1) t = 1;
    if (t > 16777216.0) t = 16777216.0;
    return (uint32_t)t;
}

struct WalkCount { int64_t steps = 0; int64_t truncated = 0; };

// ---------------------------------------------------------------------------
// Algorithm 1: WalkOnSpheres(x, eps).  The recursion
//   u(x_k) = S_k + [continue] u(x_{k+1})
// is tail-recursive with an additive term, so it is unrolled into a loop that
// carries the running sum of source contributions.
// ---------------------------------------------------------------------------
double walk_on_spheres(const Scene& sc, const double* x0, const Stream& st, uint32_t extra,
                       WalkCount& cnt, CvTrace* tr = nullptr) {
    const int D = sc.D;
    double x[3] = {0, 0, 0};
    for (int i = 0; i < D; ++i) x[i] = x0[i];
    double acc = 0.0;
    for (uint32_t k = 0;; ++k) {
        Hit h = sc.closest(x);                          // DistanceToBoundary
        cnt.steps++;
        double d = std::sqrt(h.d2);
        bool cap = (int64_t)k + 1 >= sc.s.kmax;
        if (d < sc.s.eps || cap) {                      // in the eps-shell
            if (cap && !(d < sc.s.eps)) cnt.truncated++;
            if (tr) {
                tr->alive = true;
                for (int i = 0; i < D; ++i) tr->xstop[i] = x[i];
            }
            return acc + sc.g(h);
        }
        uint32_t w[4];
        st.draw(k, extra, w);
        if (tr) {   // reservoir choice of the source step for the control variate
            const double mj = green_mass(D, sc.s.sigma, d);
            tr->S += mj;
            tr->any = true;
            uint32_t wr[4];
            st.draw(k, extra | 4u, wr);
            if (u24(wr[0]) * tr->S < mj) {
                double dir[3];
                sphere_dir(D, wr[1], wr[2], dir);
                tr->rho = std::pow(u24pos(wr[3]), 1.0 / D);
                tr->d = d;
                for (int i = 0; i < D; ++i) tr->y[i] = x[i] + tr->rho * d * dir[i];
            }
        }
        if (sc.has_source()) {                          // source contribution
            // ball-point direction: in 2D the step's second word (the step
            // direction uses only the first), in 3D a second draw
            uint32_t wb[4] = {w[1], 0, 0, 0};
            if (D == 3) st.draw(k, extra | 2u, wb);
            double dir[3];
            sphere_dir(D, wb[0], wb[1], dir);
            double rad = d * std::pow(u24pos(w[3]), 1.0 / D);   // uniform in the ball
            double y[3] = {0, 0, 0};
            for (int i = 0; i < D; ++i) y[i] = x[i] + rad * dir[i];
            // G / p^B = G * |B|
            acc += green(D, sc.s.sigma, rad, d) * ball_volume(D, d) * sc.f(y);
        }
        double alpha = poisson_scale(D, sc.s.sigma, d); // recursive scale
        if (sc.s.rr && alpha < u24(w[2])) return acc;   // Russian roulette
        double s[3];
        sphere_dir(D, w[0], w[1], s);                   // SampleUnitSphere
        for (int i = 0; i < D; ++i) x[i] += d * s[i];
    }
}

// ---------------------------------------------------------------------------
// Walk on stars for the mixed problem of Sec. 3.4 (eq. (mixed_bvp)): the
// Dirichlet boundary and a fixed reflecting boundary with the Robin condition
// du/dn - mu u = h (n into the domain; mu = 0, h = 0: zero flux, the case of
// the paper's thermal design example).  The paper defers the estimator to
// the walk-on-stars papers (Sawhney et al. 2023; Miller et al. 2024); it is
// restated here from Green's second identity on the star-shaped region
// St = B(x, R) ∩ Omega with the ball's Green's function G (zero on the
// sphere): for x inside,
//   u(x) = int_St G f + int_{sphere part} P u
//          + int_{reflecting part in B} [P_z u - G (mu u + h)] dz,
// P = -dG/dn_out the ball's Poisson kernel (at a reflecting point z, taken
// with the domain's outward normal there).  At a point on a wall the left
// side is u(x)/2.  One step:
//   * d = distance to the Dirichlet boundary; in its eps-shell the walk
//     stops with g as in Algorithm 1.
//   * star radius R = min(d, distance to the closest silhouette point of the
//     reflecting boundary[, 1/mu]): the part of the ball visible from x is
//     then a star-shaped region bounded by the sphere and the reflecting
//     boundary, all of whose reflecting points in the ball x sees.  (1/mu
//     bounds the Robin term's mass per step, a variance choice.)
//   * direction v uniform on the circle (at a reflecting boundary point: on
//     the half that enters the domain, by reflecting the other half, which
//     doubles the density and pays the factor 2 of the wall's left side).
//   * march along v: the first reflecting boundary point at distance t < R
//     is the direction-sampled point, weight neumann_weight(t, R), else
//     x + R v with weight alpha(R) as in Algorithm 1.
//   * source: one point y = x + rho v of the ball along the same direction,
//     rho = R U^(1/D), contributing |B_R| G(rho; R) f(y) if it lies in the
//     star-shaped region (rho < t).
//   * Robin terms (mu > 0 or h != 0): z uniform by length on the reflecting
//     boundary inside the ball (length L, boundary_sample); the data term
//     adds -c L G(|z - x|; R) h(z), c = 2 on a wall (the left side's 1/2)
//     and 1 inside.  The mu term needs u(z): with probability
//     q = min(1/2, c mu L G) the walk continues at z with weight
//     -c mu L G / q, else at the direction-sampled point with its weight
//     divided by 1 - q (either choice is unbiased for any q in (0, 1)).
//   * Russian roulette keeps the walk with probability s = min(1, |w|) and
//     multiplies its throughput tau by w / s, so tau stays 1 unless the
//     Robin term flips its sign or a weight exceeds 1; every term the walk
//     adds and its terminal value are multiplied by tau.
// Random numbers: one draw per step, w0 (and w1 in 3D) the direction, w1
// (2D) the Robin branch, w2 the roulette, w3 the source radius; and the
// boundary sample's own draws (boundary_sample).
// ---------------------------------------------------------------------------
struct StarStep {
    bool stop = false;     // stopped by roulette
    int on = -1;           // reflecting segment of the new point, -1 none
};

StarStep star_step(const Scene& sc, double* x, int on, double* nin, double d2, uint32_t k,
                   const Stream& st, uint32_t extra, double& acc, double& tau) {
    const int D = sc.D;
    const double mu = sc.s.robin_mu;
    double R = std::sqrt(sc.silhouette_d2(x, on, nin, d2));
    if (mu > 0) R = std::min(R, 1.0 / mu);
    uint32_t w[4];
    st.draw(k, extra, w);
    double v[3];
    sphere_dir(D, w[0], w[1], v);
    if (on >= 0) {
        const double c = dot(v, nin, D);
        if (c < 0) for (int i = 0; i < D; ++i) v[i] -= 2 * c * nin[i];
    }
    double t;
    const int seg = sc.ray(x, v, R, on, t);
    if (sc.has_source()) {
        const double rho = R * std::pow(u24pos(w[3]), 1.0 / D);
        if (seg < 0 || rho < t) {
            double y[3] = {0, 0, 0};
            for (int i = 0; i < D; ++i) y[i] = x[i] + rho * v[i];
            acc += tau * green(D, sc.s.sigma, rho, R) * ball_volume(D, R) * sc.f(y);
        }
    }
    // Robin terms over the reflecting boundary inside the ball
    const double cx = on >= 0 ? 2.0 : 1.0;
    double z[3] = {0, 0, 0}, L = 0, Gz = 0;
    int zseg = -1;
    uint32_t wbranch = w[1];   // 2D: word 1 of the step's draw; 3D: the boundary sample's
    if (sc.has_robin()) {
        zseg = sc.boundary_sample(x, R, st, k, extra, L, z, &wbranch);
        if (zseg >= 0) {
            double r2 = 0;
            for (int i = 0; i < D; ++i) r2 += (z[i] - x[i]) * (z[i] - x[i]);
            Gz = green(D, sc.s.sigma, std::sqrt(r2), R);
            acc -= tau * cx * L * Gz * sc.robin_h(z);
        }
    }
    const double q = (mu > 0 && zseg >= 0) ? std::min(0.5, cx * mu * L * Gz) : 0.0;
    const bool to_z = q > 0 && u24(wbranch) < q;
    const double wgt = to_z ? -cx * mu * L * Gz / q
                            : (seg >= 0 ? neumann_weight(D, sc.s.sigma, t, R) : poisson_scale(D, sc.s.sigma, R)) /
                                  (1 - q);
    StarStep out;
    if (sc.s.rr) {
        const double keep = std::min(1.0, std::fabs(wgt));
        if (!(keep > 0) || keep < u24(w[2])) { out.stop = true; return out; }
        tau *= wgt / keep;
    } else {
        tau *= wgt;
    }
    if (to_z) {   // continue on the wall at z; domain side: towards x
        if (zseg != on) {
            sc.nleft(zseg, nin);
            double dx[3] = {0, 0, 0};
            for (int i = 0; i < D; ++i) dx[i] = x[i] - z[i];
            if (dot(nin, dx, D) < 0) for (int i = 0; i < D; ++i) nin[i] = -nin[i];
        }
        for (int i = 0; i < D; ++i) x[i] = z[i];
        out.on = zseg;
        return out;
    }
    for (int i = 0; i < D; ++i) x[i] += t * v[i];
    out.on = seg;
    if (seg >= 0) {   // domain side of the segment: the side the walk came from
        sc.nleft(seg, nin);
        if (dot(nin, v, D) > 0) for (int i = 0; i < D; ++i) nin[i] = -nin[i];
    }
    return out;
}

double walk_on_stars(const Scene& sc, const double* x0, int on0, const double* nin0,
                     const Stream& st, uint32_t extra, WalkCount& cnt) {
    const int D = sc.D;
    double x[3] = {0, 0, 0}, nin[3] = {0, 0, 0};
    for (int i = 0; i < D; ++i) { x[i] = x0[i]; if (on0 >= 0) nin[i] = nin0[i]; }
    int on = on0;
    double acc = 0.0, tau = 1.0;
    for (uint32_t k = 0;; ++k) {
        Hit h = sc.closest(x);                          // Dirichlet boundary only
        cnt.steps++;
        const double d = std::sqrt(h.d2);
        const bool cap = (int64_t)k + 1 >= sc.s.kmax;
        if (d < sc.s.eps || cap) {
            if (cap && !(d < sc.s.eps)) cnt.truncated++;
            return acc + tau * sc.g(h);
        }
        StarStep r = star_step(sc, x, on, nin, h.d2, k, st, extra, acc, tau);
        if (r.stop) return acc;
        on = r.on;
    }
}

// ---------------------------------------------------------------------------
// Algorithm 1 on the implicit boundary of Sec. 7.4.  The ball is the safe
// disk of the point (safe_radius: inside the domain, not the largest empty
// one); the walk stops in the shell (in_shell) at the boundary point of one
// Newton projection xbar = x - h grad h / |grad h|^2.  Every other step is
// Algorithm 1's, with the same random numbers.
// ---------------------------------------------------------------------------
void source_and_step(const Scene& sc, double* x, double d, const uint32_t w[4], const Stream& st,
                     uint32_t k, uint32_t extra, double& acc) {
    const int D = sc.D;
    if (sc.has_source()) {
        uint32_t wb[4] = {w[1], 0, 0, 0};
        if (D == 3) st.draw(k, extra | 2u, wb);
        double dir[3];
        sphere_dir(D, wb[0], wb[1], dir);
        double rad = d * std::pow(u24pos(w[3]), 1.0 / D);
        double y[3] = {0, 0, 0};
        for (int i = 0; i < D; ++i) y[i] = x[i] + rad * dir[i];
        acc += green(D, sc.s.sigma, rad, d) * ball_volume(D, d) * sc.f(y);
    }
}

double walk_implicit(const Scene& sc, const double* x0, const Stream& st, uint32_t extra, WalkCount& cnt) {
    double x[3] = {x0[0], x0[1], 0};
    double acc = 0.0;
    for (uint32_t k = 0;; ++k) {
        double gr[2];
        const double h = sc.hval(x, gr);
        cnt.steps++;
        const double gn = std::hypot(gr[0], gr[1]);
        const bool shell = sc.in_shell(h, gn);
        const bool cap = (int64_t)k + 1 >= sc.s.kmax;
        if (shell || cap) {
            if (cap && !shell) cnt.truncated++;
            double xb[3] = {x[0] - h * gr[0] / (gn * gn), x[1] - h * gr[1] / (gn * gn), 0}, gg[3];
            return acc + sc.g_field(xb, gg);
        }
        const double d = sc.safe_radius(x, h);
        uint32_t w[4];
        st.draw(k, extra, w);
        source_and_step(sc, x, d, w, st, k, extra, acc);
        if (sc.s.rr && poisson_scale(2, sc.s.sigma, d) < u24(w[2])) return acc;
        double dir[3];
        sphere_dir(2, w[0], w[1], dir);
        for (int i = 0; i < 2; ++i) x[i] += d * dir[i];
    }
}

struct DiffOut {
    double u = 0;          // joint estimate of u (sources + g at the terminal)
    bool terminal = false; // reached the shell (false: stopped by roulette)
    int prim = -1;
    double xbar[3] = {0, 0, 0};   // terminal closest point
    double uoff = 0;       // mean of the K nested walks at the offset point
    double tau = 1;        // walk-on-stars throughput at the terminal (udot carries it)
    int64_t nested_steps = 0;
    std::vector<double> udot;  // dense N-vector
    // with the control variate:
    int run = -1;          // -1 no terminal, 0 nested walks skipped, 1 run
    double xoff[3] = {0, 0, 0};
    double uoff_cv = 0;    // estimate of u(xoff) used in du/dn
    double target = 0;     // N(xoff) + (mean of uhat + C), run == 1 only
    std::vector<CvTrace> traces;
};

// The control-variate estimate of u(xoff) from the nested walks' traces:
//   N(xoff) + [run] (uhat - mean_i corr_i) / q,
//   corr_i = S_i |B| G (-Lap N + sigma N)(y_i) / m(d_i) + [alive_i] N(xstop_i).
void cv_combine(const Scene& sc, const oracle_cv& cv, DiffOut& o) {
    const int D = sc.D;
    double Noff = mlp_eval(D, cv.F, cv.B, cv.theta, o.xoff).N;
    if (o.run == 0) { o.uoff_cv = Noff; return; }
    double corr = 0;
    for (const CvTrace& t : o.traces) {
        if (t.any) {
            MlpOut e = mlp_eval(D, cv.F, cv.B, cv.theta, t.y);
            double fN = -e.lap + sc.s.sigma * e.N;
            corr += t.S * green(D, sc.s.sigma, t.rho * t.d, t.d) * ball_volume(D, t.d) /
                    green_mass(D, sc.s.sigma, t.d) * fN;
        }
        if (t.alive) corr += mlp_eval(D, cv.F, cv.B, cv.theta, t.xstop).N;
    }
    corr /= (double)o.traces.size();
    double q = (double)cv_threshold(cv.q) * 0x1p-24;
    o.target = Noff + o.uoff - corr;
    o.uoff_cv = Noff + (o.uoff - corr) / q;
}

// ---------------------------------------------------------------------------
// Boundary value of the differential problem at the boundary point h with
// outward normal n, for every parameter j (eq. (boundary_deriv_restricted);
// for mapped data eq. (boundary_deriv_mapped) with the tangential components
// of the velocity kept explicitly, Appendix A), given du/dn there.  vn, if
// given, receives the normal velocity V_n,j = n . V_j.
// ---------------------------------------------------------------------------
void boundary_udot(const Scene& sc, const Hit& h, const double* n, double dudn, std::vector<double>& udot,
                   std::vector<double>* vn) {
    const int D = sc.D;
    const int N = sc.s.N;
    udot.assign(N, 0.0);
    if (vn) vn->assign(N, 0.0);
    // velocity field at xbar for each parameter: V_j = sum_k b_k dv_{i_k}/dpi_j
    std::vector<double> Vj((size_t)N * 3, 0.0);
    std::vector<char> touched(N, 0);
    std::vector<double> gdot(N, 0.0);
    for (int kk = 0; kk < D; ++kk) {
        int vi = sc.pv(h.prim, kk);
        for (int64_t e = sc.s.rowptr[vi]; e < sc.s.rowptr[vi + 1]; ++e) {
            int j = sc.s.pid[e];
            touched[j] = 1;
            for (int c = 0; c < D; ++c) Vj[(size_t)j * 3 + c] += h.bary[kk] * sc.s.vel[e * D + c];
        }
        if (sc.s.bc_pid && sc.s.bc_pid[vi] >= 0 && sc.mapped(h.prim)) {
            gdot[sc.s.bc_pid[vi]] += h.bary[kk];
            touched[sc.s.bc_pid[vi]] = 1;
        }
    }
    bool mp = sc.mapped(h.prim);
    double gr[3];
    if (mp) sc.grad_surface(h, gr); else sc.grad_field(h, gr);
    double dgdn = dot(gr, n, D);
    for (int j = 0; j < N; ++j) {
        if (!touched[j]) continue;
        const double* V = &Vj[(size_t)j * 3];
        double Vn = dot(n, V, D);
        if (vn) (*vn)[j] = Vn;
        if (mp) {
            // gdot_ref - grad_G g . V - V_n du/dn
            udot[j] = gdot[j] - dot(gr, V, D) - Vn * dudn;
        } else {
            // eq. (boundary_deriv_restricted): gdot_field (= 0) + (dg/dn - du/dn) V_n
            udot[j] = (dgdn - dudn) * Vn;
        }
    }
}

// ---------------------------------------------------------------------------
// Algorithm 2: DiffWalkOnSpheres(x, eps, delta).  The walk follows the same
// steps (and random numbers) as Algorithm 1 so that it also returns the joint
// estimate of u.  At the shell it launches K forward walks from the offset
// point xbar - delta n and forms the differential boundary value.
// ---------------------------------------------------------------------------
// With a reflecting boundary the walk takes walk-on-stars steps (Sec. 4.4:
// the differential walk on stars nests through the Dirichlet boundary
// only), starting on reflecting segment on0 (domain side nin0) or inside.
DiffOut diff_walk_on_spheres(const Scene& sc, const double* x0, const Stream& st,
                             WalkCount& cnt, bool want_udot, const oracle_cv* cv = nullptr,
                             int on0 = -1, const double* nin0 = nullptr) {
    const int D = sc.D;
    const int N = sc.s.N;
    DiffOut out;
    if (want_udot) out.udot.assign(N, 0.0);
    double x[3] = {0, 0, 0}, nin[3] = {0, 0, 0}, xprev[3] = {0, 0, 0};
    for (int i = 0; i < D; ++i) { x[i] = x0[i]; if (on0 >= 0) nin[i] = nin0[i]; }
    int on = on0;
    double acc = 0.0, tau = 1.0;   // tau: walk-on-stars throughput (1 otherwise)
    for (uint32_t k = 0;; ++k) {
        Hit h = sc.closest(x);
        cnt.steps++;
        double d = std::sqrt(h.d2);
        bool cap = (int64_t)k + 1 >= sc.s.kmax;
        if (d < sc.s.eps || cap) {
            if (cap && !(d < sc.s.eps)) cnt.truncated++;
            double n[3];
            sc.normal(h, k > 0 ? xprev : x, n);                // BoundaryNormal
            double xoff[3] = {0, 0, 0};
            for (int i = 0; i < D; ++i) xoff[i] = h.xbar[i] - sc.s.delta * n[i];
            double usum = 0;
            out.run = 1;
            // At a primitive that depends on no parameter the nested estimate is
            // multiplied by V_n = 0 and gdot = 0 in every derivative, so the
            // nested walks are not run (their mean is reported as g).
            const bool dep = sc.depends(h.prim);
            if (!dep) out.run = -1;
            if (dep && cv && cv_threshold(cv->q) < (1u << 24)) {   // run the nested walks w.p. q
                uint32_t wq[4];
                st.draw(k, 4u, wq);
                out.run = (wq[0] >> 8) < cv_threshold(cv->q) ? 1 : 0;
            }
            if (cv) out.traces.assign(out.run == 1 ? sc.s.K : 0, CvTrace());
            const double gx = sc.g(h);
            // offset-point gradient estimator (eq. (dudn_mc_estimate)): the
            // largest empty ball around xoff has radius R; the first step of
            // a nested walk from xoff lands at y = xoff + R s, s uniform on
            // the unit sphere, and (without source or roulette, sigma = 0)
            // the walk's value is u(y).  D/R (s.n) u(y) is unbiased for
            // n . grad u(xoff) (the mean-value property differentiated at
            // the centre); g(xbar) is subtracted as a control variate
            // (E[s] = 0).  The paper prints 3/delta (3D, R = delta); D/R is
            // that factor in D dimensions for the ball the walk samples.
            double bsum = 0;
            double R0 = 0;
            if (sc.s.dudn == 1 && out.run == 1) R0 = std::sqrt(sc.closest(xoff).d2);
            for (int i = 0; out.run == 1 && i < sc.s.K; ++i) {  // nested forward walks
                WalkCount c2;
                const uint32_t tag = 1u | ((uint32_t)i << 8);
                const double v = sc.has_neumann()
                            ? walk_on_stars(sc, xoff, -1, nullptr, st, tag, c2)
                            : walk_on_spheres(sc, xoff, st, tag, c2, cv ? &out.traces[i] : nullptr);
                usum += v;
                if (sc.s.dudn == 1 && R0 >= sc.s.eps && sc.s.kmax > 1) {
                    uint32_t w0[4];
                    st.draw(0, tag, w0);
                    double s0[3];
                    sphere_dir(D, w0[0], w0[1], s0);
                    bsum += D / R0 * dot(s0, n, D) * (v - gx);
                }
                out.nested_steps += c2.steps;
                cnt.truncated += c2.truncated;
            }
            double uhat = dep ? usum / sc.s.K : gx;
            // the gradient estimate, stated as the offset value that the
            // backward difference would turn into it
            if (sc.s.dudn == 1 && dep && out.run == 1) uhat = gx - sc.s.delta * (bsum / sc.s.K);
            for (int i = 0; i < 3; ++i) out.xoff[i] = xoff[i];
            out.uoff = uhat;
            if (cv && dep) {
                cv_combine(sc, *cv, out);
                uhat = out.uoff_cv;
            }
            double dudn = (gx - uhat) / sc.s.delta;            // eq. (dudn_fd_estimate)
            out.u = acc + tau * gx;
            out.tau = tau;
            out.terminal = true;
            out.prim = h.prim;
            for (int i = 0; i < 3; ++i) out.xbar[i] = h.xbar[i];
            if (want_udot) {
                boundary_udot(sc, h, n, dudn, out.udot, nullptr);
                if (tau != 1.0) for (double& e : out.udot) e *= tau;
            }
            return out;
        }
        if (sc.has_neumann()) {
            for (int i = 0; i < D; ++i) xprev[i] = x[i];
            StarStep r = star_step(sc, x, on, nin, h.d2, k, st, 0u, acc, tau);
            if (r.stop) { out.u = acc; return out; }   // roulette: udot = 0, u = sources
            on = r.on;
            continue;
        }
        uint32_t w[4];
        st.draw(k, 0u, w);
        if (sc.has_source()) {   // sources only enter the joint u estimate
            uint32_t wb[4] = {w[1], 0, 0, 0};
            if (D == 3) st.draw(k, 2u, wb);
            double dir[3];
            sphere_dir(D, wb[0], wb[1], dir);
            double rad = d * std::pow(u24pos(w[3]), 1.0 / D);
            double y[3] = {0, 0, 0};
            for (int i = 0; i < D; ++i) y[i] = x[i] + rad * dir[i];
            acc += green(D, sc.s.sigma, rad, d) * ball_volume(D, d) * sc.f(y);
        }
        double alpha = poisson_scale(D, sc.s.sigma, d);
        if (sc.s.rr && alpha < u24(w[2])) {   // roulette: udot = 0, u = sources
            out.u = acc;
            return out;
        }
        double s[3];
        sphere_dir(D, w[0], w[1], s);
        for (int i = 0; i < D; ++i) xprev[i] = x[i];
        for (int i = 0; i < D; ++i) x[i] += d * s[i];
    }
}

// Algorithm 2 on the implicit boundary: at the shell, the boundary point
// xbar (Newton projection), the outward normal n = -grad h / |grad h| there,
// K nested walks from xbar - delta n, and for each parameter the normal
// velocity V_n = (dh/dpi) / |grad h| (the paper's level-set formula, Sec.
// 3.1) in eq. (boundary_deriv_restricted): udot = V_n (dg/dn - du/dn).
DiffOut diff_walk_implicit(const Scene& sc, const double* x0, const Stream& st, WalkCount& cnt,
                           bool want_udot) {
    const int N = sc.s.N;
    DiffOut out;
    if (want_udot) out.udot.assign(N, 0.0);
    double x[3] = {x0[0], x0[1], 0};
    double acc = 0.0;
    for (uint32_t k = 0;; ++k) {
        double gr[2];
        const double h = sc.hval(x, gr);
        cnt.steps++;
        const double gn = std::hypot(gr[0], gr[1]);
        const bool shell = sc.in_shell(h, gn);
        const bool cap = (int64_t)k + 1 >= sc.s.kmax;
        if (shell || cap) {
            if (cap && !shell) cnt.truncated++;
            double xb[3] = {x[0] - h * gr[0] / (gn * gn), x[1] - h * gr[1] / (gn * gn), 0};
            double gb[2];
            sc.hval(xb, gb);
            const double gbn = std::hypot(gb[0], gb[1]);
            const double n[3] = {-gb[0] / gbn, -gb[1] / gbn, 0};
            double xoff[3] = {xb[0] - sc.s.delta * n[0], xb[1] - sc.s.delta * n[1], 0};
            double usum = 0;
            for (int i = 0; i < sc.s.K; ++i) {
                WalkCount c2;
                usum += walk_implicit(sc, xoff, st, 1u | ((uint32_t)i << 8), c2);
                out.nested_steps += c2.steps;
                cnt.truncated += c2.truncated;
            }
            double ggr[3];
            const double gx = sc.g_field(xb, ggr);
            out.uoff = usum / sc.s.K;
            out.run = 1;
            for (int i = 0; i < 3; ++i) { out.xoff[i] = xoff[i]; out.xbar[i] = xb[i]; }
            const double dudn = (gx - out.uoff) / sc.s.delta;
            const double dgdn = ggr[0] * n[0] + ggr[1] * n[1];
            out.u = acc + gx;
            out.terminal = true;
            out.prim = 0;
            if (want_udot) {
                std::vector<double> dh(3 * sc.s.n_mono);
                sc.hparam(xb, dh.data());
                for (int j = 0; j < N && j < 3 * sc.s.n_mono; ++j) out.udot[j] = dh[j] / gbn * (dgdn - dudn);
            }
            return out;
        }
        const double d = sc.safe_radius(x, h);
        uint32_t w[4];
        st.draw(k, 0u, w);
        source_and_step(sc, x, d, w, st, k, 0u, acc);
        if (sc.s.rr && poisson_scale(2, sc.s.sigma, d) < u24(w[2])) { out.u = acc; return out; }
        double dir[3];
        sphere_dir(2, w[0], w[1], dir);
        for (int i = 0; i < 2; ++i) x[i] += d * dir[i];
    }
}

Stream make_stream(uint64_t seed, uint32_t p, uint32_t m, uint32_t instance) {
    Stream st;
    st.key[0] = (uint32_t)seed; st.key[1] = (uint32_t)(seed >> 32);
    st.m = m; st.p = p; st.tag = instance << 16;
    return st;
}

template <class F>
void parallel_points(int64_t P, int threads, F&& fn) {
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    if (threads > P) threads = (int)std::max<int64_t>(1, P);
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&, t] { for (int64_t p = t; p < P; p += threads) fn(t, p); });
    for (auto& th : pool) th.join();
}

int check_scene(const oracle_scene* s) {
    if (!s) return 1;
    if (s->n_mono < 0) return 1;
    if (s->dudn != 0 && (s->dudn != 1 || s->n_mono > 0)) return 1;
    if (s->n_mono > 0) {   // implicit boundary: 2D, c < 0, positive scales, restricted data
        if (s->dim != 2 || !s->mono || !(s->mono_c < 0) || s->n_ns > 0 || !s->bc_kind || s->bc_kind[0] != 0)
            return 1;
        for (int n = 0; n < s->n_mono; ++n) if (!(s->mono[3 * n] > 0)) return 1;
        if (!(s->eps > 0) || s->sigma < 0 || s->K < 1 || s->kmax < 1 || (!s->rr && s->sigma > 0)) return 1;
        return 0;
    }
    if (s->dudn != 0 && s->dudn != 1) return 1;
    if (s->dudn == 1 && (s->sigma != 0 || s->src_c0 != 0 || s->n_gauss > 0 || s->n_ns > 0 || s->n_mono > 0))
        return 1;
    if ((s->dim != 2 && s->dim != 3) || s->nv <= 0 || s->np <= 0) return 1;
    if (!(s->eps > 0) || s->sigma < 0 || s->K < 1 || s->kmax < 1) return 1;
    // without roulette the walks would have to carry the product of the
    // alpha factors; only sigma = 0 (alpha = 1) is accepted then
    if (!s->rr && s->sigma > 0) return 1;
    if (s->n_ns < 0) return 1;
    if (s->n_ns > 0) {
        if (!s->NV || !s->nsegs || s->n_nv <= 0) return 1;
        for (int64_t i = 0; i < s->dim * (int64_t)s->n_ns; ++i)
            if (s->nsegs[i] < 0 || s->nsegs[i] >= s->n_nv) return 1;
    }
    // the Robin condition lives on the reflecting boundary; the boundary
    // sample's counter holds a segment index in 16 bits
    if (!(s->robin_mu >= 0) || !std::isfinite(s->robin_mu)) return 1;
    if ((s->robin_mu > 0 || s->robin_quad) && (s->n_ns <= 0 || s->n_ns > 65536)) return 1;
    return 0;
}

// start segments of P query points must name reflecting segments (or -1)
int check_starts(const oracle_scene* s, int64_t P) {
    if (!s->start_seg) return 0;
    for (int64_t p = 0; p < P; ++p)
        if (s->start_seg[p] < -1 || s->start_seg[p] >= s->n_ns) return 1;
    return 0;
}

// Where the walks of query point p start: on a reflecting segment (the
// domain to its left) or inside the domain.
struct Start {
    int on = -1;
    double nin[3] = {0, 0, 0};
};

Start start_of(const Scene& sc, int64_t p) {
    Start s0;
    if (sc.has_neumann() && sc.s.start_seg && sc.s.start_seg[p] >= 0) {
        s0.on = sc.s.start_seg[p];
        sc.nleft(s0.on, s0.nin);
    }
    return s0;
}

// Algorithm 1, or walk on stars when there is a reflecting boundary.
double forward_walk(const Scene& sc, const double* x, const Start& s0, const Stream& st,
                    WalkCount& c) {
    if (sc.implicit()) return walk_implicit(sc, x, st, 0u, c);
    return sc.has_neumann() ? walk_on_stars(sc, x, s0.on, s0.nin, st, 0u, c)
                            : walk_on_spheres(sc, x, st, 0u, c);
}

DiffOut diff_walk(const Scene& sc, const double* x, const Start& s0, const Stream& st,
                  WalkCount& c, bool want_udot, const oracle_cv* cv) {
    if (sc.implicit()) return diff_walk_implicit(sc, x, st, c, want_udot);
    return diff_walk_on_spheres(sc, x, st, c, want_udot, cv, s0.on, s0.nin);
}

// ---------------------------------------------------------------------------
// The adjoint formulation of the shape derivative (Appendix B, eq.
// (functional_deriv_adjoint)), which the paper sets against Algorithm 2 and
// rejects for its quadratic nesting; built here as that ablation.  For the
// squared loss J = int_Omega l(u), l(u) = 1/2 (u - uref)^2, with a quadratic
// reference uref(x) = c + b.x + x^T A x, the adjoint solves
//   -Lap lambda + sigma lambda = l'(u) = u - uref  in Omega,  lambda = 0 on
//   the boundary
// (eq. (bvp_adjoint) writes the operator with the other sign, so its adjoint
// is minus this one), and Green's second identity turns the domain term of
// eq. (functional_deriv) into a boundary integral:
//   dJ/dpi_j = int_boundary [ -dlambda/dn udot_j + l(g) V_n,j ] dsigma,
// udot_j the boundary value of the differential problem (as at a terminal of
// Algorithm 2), l(g) V_n,j the boundary term of eq. (functional_deriv), which
// the printed adjoint formula leaves out (it vanishes where uref = g).
// At a boundary sample y with outward normal n, dlambda/dn is the backward
// difference (0 - lambda(y - delta n)) / delta and du/dn the backward
// difference of the mean of K forward walks from the same offset point.
// ---------------------------------------------------------------------------
double uref_quad(int D, const double* q, const double* x) {
    double v = q[0];
    for (int i = 0; i < D; ++i) v += q[1 + i] * x[i];
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) v += x[i] * q[1 + D + i * D + j] * x[j];
    return v;
}

// Random streams of one adjoint sample walk (key = seed, counter (k, m, s,
// purpose)): purpose 0x10 the adjoint walk's step k (0x12 its second draw in
// 3D), 0x20 | k' << 8 the forward walk at the source point of adjoint step
// k', 0x30 | i << 8 the i-th forward walk from the offset point.
constexpr uint32_t kAdjStep = 0x10u, kAdjSource = 0x20u, kAdjOffset = 0x30u;

// Algorithm 1 for the adjoint problem: zero boundary data, and at every step
// the source term G |B| l'(u(y)) at a uniform point y of the ball, with u(y)
// from a whole forward walk started at y.
double adjoint_walk(const Scene& sc, const double* x0, const double* ref, const Stream& st, WalkCount& cnt,
                    int64_t& nested_steps) {
    const int D = sc.D;
    double x[3] = {0, 0, 0};
    for (int i = 0; i < D; ++i) x[i] = x0[i];
    double acc = 0.0;
    for (uint32_t k = 0;; ++k) {
        Hit h = sc.closest(x);
        cnt.steps++;
        double d = std::sqrt(h.d2);
        bool cap = (int64_t)k + 1 >= sc.s.kmax;
        if (d < sc.s.eps || cap) {
            if (cap && !(d < sc.s.eps)) cnt.truncated++;
            return acc;                                     // lambda = 0 on the boundary
        }
        uint32_t w[4];
        st.draw(k, kAdjStep, w);
        uint32_t wb[4] = {w[1], 0, 0, 0};
        if (D == 3) st.draw(k, kAdjStep | 2u, wb);
        double dir[3];
        sphere_dir(D, wb[0], wb[1], dir);
        double rad = d * std::pow(u24pos(w[3]), 1.0 / D);
        double y[3] = {0, 0, 0};
        for (int i = 0; i < D; ++i) y[i] = x[i] + rad * dir[i];
        WalkCount c2;
        const double uy = walk_on_spheres(sc, y, st, kAdjSource | (k << 8), c2);
        nested_steps += c2.steps;
        cnt.truncated += c2.truncated;
        acc += green(D, sc.s.sigma, rad, d) * ball_volume(D, d) * (uy - uref_quad(D, ref, y));
        double alpha = poisson_scale(D, sc.s.sigma, d);
        if (sc.s.rr && alpha < u24(w[2])) return acc;
        double s[3];
        sphere_dir(D, w[0], w[1], s);
        for (int i = 0; i < D; ++i) x[i] += d * s[i];
    }
}

// Outward normal of primitive `prim` from a side code: the geometric normal
// (segment a->b: (b - a) turned clockwise; triangle: (b - a) x (c - a)),
// negated when the code's flip bit is set.
void side_normal(const Scene& sc, int prim, int flip, double n[3]) {
    const int D = sc.D;
    n[0] = n[1] = n[2] = 0;
    if (D == 2) {
        const double* a = sc.vert(sc.pv(prim, 0));
        const double* b = sc.vert(sc.pv(prim, 1));
        double tx = b[0] - a[0], ty = b[1] - a[1];
        double L = std::sqrt(tx * tx + ty * ty);
        n[0] = ty / L; n[1] = -tx / L;
    } else {
        const double* a = sc.vert(sc.pv(prim, 0));
        const double* b = sc.vert(sc.pv(prim, 1));
        const double* c = sc.vert(sc.pv(prim, 2));
        double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        double L = std::sqrt(dot(cr, cr, 3));
        for (int i = 0; i < 3; ++i) n[i] = cr[i] / L;
    }
    if (flip) for (int i = 0; i < 3; ++i) n[i] = -n[i];
}

}  // namespace

extern "C" {

int oracle_threads(void) { return (int)std::max(1u, std::thread::hardware_concurrency()); }

// Adjoint formulation (Appendix B) of the squared-loss shape derivative:
// S boundary samples (primitive code = prim * 2 + flip, barycentrics
// b1 (, b2), quadrature weight wq), W walks each; grad (N) receives
//   sum_s wq_s / W sum_m [ lambda_m / delta udot_j(y_s; uoff_m) + l(g) V_n,j ]
// (lambda_m the adjoint estimate at the offset point, uoff_m the mean of the
// K forward walks there).  lam, uoff, steps (S x W, may be NULL) receive the
// per-walk records (steps: all walks of the record, nested included).
int oracle_adjoint_grad(const oracle_scene* s, const int32_t* code, const double* bary, const double* wq,
                        int64_t S, const double* ref, int32_t W, uint64_t seed, double* grad, double* lam,
                        double* uoff, int64_t* steps, int threads) {
    if (check_scene(s) || s->n_ns > 0 || s->n_mono > 0 || s->dudn != 0 || W < 1 || S < 0 || !ref) return 1;
    if (s->N < 0 || (s->N > 0 && !s->rowptr)) return 1;
    for (int64_t i = 0; i < S; ++i)
        if (code[i] < 0 || (code[i] >> 1) >= s->np) return 1;
    Scene sc(*s);
    const int D = s->dim;
    const int N = s->N;
    if (threads <= 0) threads = (int)std::max(1u, std::thread::hardware_concurrency());
    std::vector<std::vector<double>> part(threads, std::vector<double>(N, 0.0));
    parallel_points(S, threads, [&](int t, int64_t si) {
        Hit h;
        h.prim = code[si] >> 1;
        if (D == 2) { h.bary[1] = bary[si]; h.bary[0] = 1 - h.bary[1]; }
        else { h.bary[1] = bary[2 * si]; h.bary[2] = bary[2 * si + 1]; h.bary[0] = 1 - h.bary[1] - h.bary[2]; }
        for (int c = 0; c < D; ++c) {
            double v = 0;
            for (int k = 0; k < D; ++k) v += h.bary[k] * sc.vert(sc.pv(h.prim, k))[c];
            h.xbar[c] = v;
        }
        h.d2 = 0;
        double n[3];
        side_normal(sc, h.prim, code[si] & 1, n);
        double xoff[3] = {0, 0, 0};
        for (int c = 0; c < D; ++c) xoff[c] = h.xbar[c] - s->delta * n[c];
        const double gx = sc.g(h);
        const double e = gx - uref_quad(D, ref, h.xbar);
        const bool dep = sc.depends(h.prim);
        std::vector<double> ud, vn;
        for (int32_t m = 0; m < W; ++m) {
            const Stream st = make_stream(seed, (uint32_t)si, (uint32_t)m, 0);
            WalkCount c1;
            int64_t nested = 0;
            double lm = 0, uo = gx;
            if (dep) {   // a primitive that moves with no parameter adds nothing; its walks are not run
                lm = adjoint_walk(sc, xoff, ref, st, c1, nested);
                double usum = 0;
                for (int i = 0; i < s->K; ++i) {
                    WalkCount c2;
                    usum += walk_on_spheres(sc, xoff, st, kAdjOffset | ((uint32_t)i << 8), c2);
                    nested += c2.steps;
                }
                uo = usum / s->K;
                if (N > 0) {
                    boundary_udot(sc, h, n, (gx - uo) / s->delta, ud, &vn);
                    for (int j = 0; j < N; ++j)
                        part[t][j] += wq[si] / W * (lm / s->delta * ud[j] + 0.5 * e * e * vn[j]);
                }
            }
            const int64_t r = si * W + m;
            if (lam) lam[r] = lm;
            if (uoff) uoff[r] = uo;
            if (steps) steps[r] = c1.steps + nested;
        }
    });
    for (int j = 0; j < N; ++j) {
        double v = 0;
        for (int t = 0; t < threads; ++t) v += part[t][j];
        grad[j] = v;
    }
    return 0;
}

void oracle_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    philox4x32_10(ctr, key, out);
}

double oracle_green(int dim, double sigma, double r, double R) { return green(dim, sigma, r, R); }
double oracle_poisson_scale(int dim, double sigma, double R) { return poisson_scale(dim, sigma, R); }
double oracle_green_mass(int dim, double sigma, double R) { return green_mass(dim, sigma, R); }

// closest point: out = {d, prim, bary0, bary1, bary2, xbar0, xbar1, xbar2}
int oracle_closest(const oracle_scene* s, const double* x, double* out) {
    if (check_scene(s)) return 1;
    Scene sc(*s);
    Hit h = sc.closest(x);
    out[0] = std::sqrt(h.d2); out[1] = h.prim;
    for (int i = 0; i < 3; ++i) { out[2 + i] = h.bary[i]; out[5 + i] = h.xbar[i]; }
    return 0;
}

// Safe disk radius at x for an implicit boundary (h(x) > 0): out[0] the
// radius used by the walks, out[1] the Harnack radius alone.
int oracle_safe_radius(const oracle_scene* s, const double* x, double* out) {
    if (check_scene(s) || s->n_mono <= 0) return 1;
    Scene sc(*s);
    double gr[2];
    const double h = sc.hval(x, gr);
    out[0] = sc.safe_radius(x, h);
    out[1] = sc.harnack_radius(x, h);
    return 0;
}

// Band term of the shape-functional derivative on an implicit boundary
// (Sec. 7.4, implicit boundary integrals): the boundary integral of
// eq. (functional_deriv) becomes a volume integral over the points of the
// domain next to the zero set.  A point is in the band when h > 0 and its
// first-order distance h / |grad h| to the zero set is below eps_band (and
// h < -c, away from the poles); each such point adds coef_p times the normal
// velocity (dh/dpi) / |grad h| of eq. (normal_velocity) to grad (3n values,
// accumulated).  region (may be NULL) receives per point 1 in the band, 2
// elsewhere in the domain (h > 0), 0 outside.
int oracle_band_grad(const oracle_scene* s, const double* X, int64_t P, const double* coef, double eps_band,
                     double* grad, int32_t* region) {
    if (check_scene(s) || s->n_mono <= 0 || !(eps_band > 0) || P < 0) return 1;
    Scene sc(*s);
    std::vector<double> dh(3 * s->n_mono);
    for (int64_t p = 0; p < P; ++p) {
        double gr[2];
        const double h = sc.hval(X + 2 * p, gr);
        const double gn = std::hypot(gr[0], gr[1]);
        const bool band = h > 0 && h < eps_band * gn && h < -s->mono_c;
        if (region) region[p] = band ? 1 : (h > 0 ? 2 : 0);
        if (!band) continue;
        sc.hparam(X + 2 * p, dh.data());
        for (int j = 0; j < 3 * s->n_mono; ++j) grad[j] += coef[p] * dh[j] / gn;
    }
    return 0;
}

double oracle_neumann_weight(int dim, double sigma, double r, double R) {
    return neumann_weight(dim, sigma, r, R);
}

// Distance from x to its closest silhouette point of the reflecting boundary
// (capped at cap), for x inside the domain (on = -1) or on reflecting
// segment `on` with the domain on the side of nin.
int oracle_silhouette(const oracle_scene* s, const double* x, int32_t on, const double* nin,
                      double cap, double* out) {
    if (check_scene(s) || s->n_ns <= 0 || on < -1 || on >= s->n_ns) return 1;
    Scene sc(*s);
    const double zero[3] = {0, 0, 0};
    *out = std::sqrt(sc.silhouette_d2(x, on, on >= 0 ? nin : zero, cap * cap));
    return 0;
}

// First reflecting segment hit by x + t dir, 0 < t < tmax (skipping `skip`):
// out = {t (tmax if none), segment or -1}.
int oracle_ray(const oracle_scene* s, const double* x, const double* dir, double tmax,
               int32_t skip, double* out) {
    if (check_scene(s) || s->n_ns <= 0) return 1;
    Scene sc(*s);
    double t;
    out[1] = sc.ray(x, dir, tmax, skip, t);
    out[0] = t;
    return 0;
}

// Draws of the Robin boundary sample around x with radius R: draw m uses the
// stream of walk m of point 0 (seed, instance 0) at step k.  out[5 m ..]:
// {reflecting primitive or -1, L, z[0], z[1], z[2]}.
int oracle_boundary_sample(const oracle_scene* s, const double* x, double R, uint64_t seed, uint32_t k,
                           int32_t n, double* out) {
    if (check_scene(s) || s->n_ns <= 0 || n < 0 || !(R > 0)) return 1;
    Scene sc(*s);
    for (int32_t m = 0; m < n; ++m) {
        const Stream st = make_stream(seed, 0u, (uint32_t)m, 0u);
        double L = 0, z[3] = {0, 0, 0};
        const int t = sc.boundary_sample(x, R, st, k, 0u, L, z);
        double* o = out + 5 * (size_t)m;
        o[0] = t; o[1] = L; o[2] = z[0]; o[3] = z[1]; o[4] = z[2];
    }
    return 0;
}

// Per-walk records.  mode 0: Algorithm 1 from each point; mode 1: Algorithm 2.
// u[P*W]; udot[P*W*N] (mode 1, may be NULL); steps[P*W] total closest-point
// queries including nested walks (may be NULL); prim[P*W] terminal primitive or
// -1 (may be NULL); uoff[P*W] nested mean (may be NULL); xbar[P*W*3] the
// terminal closest point of a differential walk (may be NULL).
int oracle_walk_records(const oracle_scene* s, const double* X, int64_t P, int32_t W,
                        uint64_t seed, int32_t mode, int32_t instance, double* u, double* udot,
                        int64_t* steps, int32_t* prim, double* uoff, int64_t* truncated,
                        double* xbar, int threads) {
    if (check_scene(s) || W < 1 || P < 0 || check_starts(s, P)) return 1;
    Scene sc(*s);
    const int D = s->dim;
    std::vector<int64_t> trunc(std::max(1, threads > 0 ? threads : oracle_threads()) + 64, 0);
    parallel_points(P, threads, [&](int t, int64_t p) {
        for (int m = 0; m < W; ++m) {
            size_t id = (size_t)p * W + m;
            Stream st = make_stream(seed, (uint32_t)p, (uint32_t)m, (uint32_t)instance);
            WalkCount c;
            if (mode == 0) {
                u[id] = forward_walk(sc, X + p * D, start_of(sc, p), st, c);
                if (prim) prim[id] = -1;
                if (uoff) uoff[id] = 0;
            } else {
                DiffOut o = diff_walk(sc, X + p * D, start_of(sc, p), st, c, udot != nullptr, nullptr);
                u[id] = o.u;
                c.steps += o.nested_steps;
                if (udot) std::memcpy(udot + id * s->N, o.udot.data(), sizeof(double) * s->N);
                if (prim) prim[id] = o.terminal ? o.prim : -1;
                if (uoff) uoff[id] = o.uoff;
                if (xbar) for (int i = 0; i < 3; ++i) xbar[id * 3 + i] = o.xbar[i];
            }
            if (steps) steps[id] = c.steps;
            trunc[t] += c.truncated;
        }
    });
    if (truncated) { int64_t a = 0; for (auto v : trunc) a += v; *truncated = a; }
    return 0;
}

// Per-point mean and (sample) variance of the mean of W forward walks.
int oracle_solve(const oracle_scene* s, const double* X, int64_t P, int32_t W, uint64_t seed,
                 int32_t instance, double* u_mean, double* u_var, int64_t* steps_total, int threads) {
    if (check_scene(s) || W < 1 || P < 0 || check_starts(s, P)) return 1;
    Scene sc(*s);
    const int D = s->dim;
    std::vector<int64_t> st_steps(256, 0);
    int T = threads > 0 ? threads : oracle_threads();
    if (T > 256) T = 256;
    parallel_points(P, T, [&](int t, int64_t p) {
        double s1 = 0, s2 = 0;
        for (int m = 0; m < W; ++m) {
            Stream st = make_stream(seed, (uint32_t)p, (uint32_t)m, (uint32_t)instance);
            WalkCount c;
            double v = forward_walk(sc, X + p * D, start_of(sc, p), st, c);
            s1 += v; s2 += v * v;
            st_steps[t] += c.steps;
        }
        double mean = s1 / W;
        u_mean[p] = mean;
        if (u_var) u_var[p] = W > 1 ? (s2 - W * mean * mean) / (W - 1) / W : 0.0;
    });
    if (steps_total) { int64_t a = 0; for (auto v : st_steps) a += v; *steps_total = a; }
    return 0;
}

// Forward mode: per point mean of the N-vector udot and the variance of that mean.
int oracle_jvp(const oracle_scene* s, const double* X, int64_t P, int32_t W, uint64_t seed,
               int32_t instance, double* udot_mean, double* udot_var, double* u_mean,
               int64_t* steps_total, int threads, const oracle_cv* cv) {
    if (check_scene(s) || W < 1 || P < 0 || check_starts(s, P)) return 1;
    if (cv && (s->n_ns > 0 || s->n_mono > 0 || s->dudn != 0)) return 1;   // the control variate is for walk on spheres only
    Scene sc(*s);
    const int D = s->dim, N = s->N;
    std::vector<int64_t> st_steps(256, 0);
    int T = threads > 0 ? threads : oracle_threads();
    if (T > 256) T = 256;
    parallel_points(P, T, [&](int t, int64_t p) {
        std::vector<double> s1(N, 0.0), s2(N, 0.0);
        double us = 0;
        for (int m = 0; m < W; ++m) {
            Stream st = make_stream(seed, (uint32_t)p, (uint32_t)m, (uint32_t)instance);
            WalkCount c;
            DiffOut o = diff_walk(sc, X + p * D, start_of(sc, p), st, c, true, cv);
            for (int j = 0; j < N; ++j) { s1[j] += o.udot[j]; s2[j] += o.udot[j] * o.udot[j]; }
            us += o.u;
            st_steps[t] += c.steps + o.nested_steps;
        }
        for (int j = 0; j < N; ++j) {
            double mean = s1[j] / W;
            udot_mean[p * N + j] = mean;
            if (udot_var) udot_var[p * N + j] = W > 1 ? (s2[j] - W * mean * mean) / (W - 1) / W : 0.0;
        }
        if (u_mean) u_mean[p] = us / W;
    });
    if (steps_total) { int64_t a = 0; for (auto v : st_steps) a += v; *steps_total = a; }
    return 0;
}

// Reverse mode: grad_j = sum_p w_p * mean_m udot_m[j]; also the joint u mean.
int oracle_grad(const oracle_scene* s, const double* X, int64_t P, const double* w, int32_t W,
                uint64_t seed, int32_t instance, double* grad, double* u_mean,
                int64_t* steps_total, int threads, const oracle_cv* cv) {
    if (check_scene(s) || W < 1 || P < 0 || check_starts(s, P)) return 1;
    if (cv && (s->n_ns > 0 || s->n_mono > 0 || s->dudn != 0)) return 1;   // the control variate is for walk on spheres only
    Scene sc(*s);
    const int D = s->dim, N = s->N;
    int T = threads > 0 ? threads : oracle_threads();
    if (T > 256) T = 256;
    std::vector<std::vector<double>> part(T, std::vector<double>(N, 0.0));
    std::vector<int64_t> st_steps(T, 0);
    parallel_points(P, T, [&](int t, int64_t p) {
        std::vector<double> s1(N, 0.0);
        double us = 0;
        for (int m = 0; m < W; ++m) {
            Stream st = make_stream(seed, (uint32_t)p, (uint32_t)m, (uint32_t)instance);
            WalkCount c;
            DiffOut o = diff_walk(sc, X + p * D, start_of(sc, p), st, c, true, cv);
            for (int j = 0; j < N; ++j) s1[j] += o.udot[j];
            us += o.u;
            st_steps[t] += c.steps + o.nested_steps;
        }
        for (int j = 0; j < N; ++j) part[t][j] += w[p] * s1[j] / W;
        if (u_mean) u_mean[p] = us / W;
    });
    for (int j = 0; j < N; ++j) { double a = 0; for (int t = 0; t < T; ++t) a += part[t][j]; grad[j] = a; }
    if (steps_total) { int64_t a = 0; for (auto v : st_steps) a += v; *steps_total = a; }
    return 0;
}

// Squared loss L = sum_p 1/2 (u_p - uref_p)^2.  Gradient
// dL/dpi = sum_p (u u' - uref u') (eq. (squared_loss_deriv)) with the product
// u u' estimated by the U-statistic of eq. (ustatistics) over batches of B
// walks, averaged over the W/B batches of each point.  loss uses the plain
// per-point walk mean.
int oracle_grad_sqloss(const oracle_scene* s, const double* X, int64_t P, const double* uref,
                       int32_t W, int32_t B, uint64_t seed, int32_t instance, double* loss,
                       double* grad, double* u_mean, int64_t* steps_total, int threads,
                       const oracle_cv* cv) {
    if (check_scene(s) || W < 1 || P < 0 || B < 2 || W % B != 0 || check_starts(s, P)) return 1;
    if (cv && (s->n_ns > 0 || s->n_mono > 0 || s->dudn != 0)) return 1;   // the control variate is for walk on spheres only
    Scene sc(*s);
    const int D = s->dim, N = s->N;
    int T = threads > 0 ? threads : oracle_threads();
    if (T > 256) T = 256;
    std::vector<std::vector<double>> part(T, std::vector<double>(N, 0.0));
    std::vector<double> lpart(T, 0.0);
    std::vector<int64_t> st_steps(T, 0);
    const int nb = W / B;
    parallel_points(P, T, [&](int t, int64_t p) {
        std::vector<double> gsum(N, 0.0);
        std::vector<std::vector<double>> ud(B);
        std::vector<double> uh(B);
        double us = 0;
        for (int b = 0; b < nb; ++b) {
            for (int q = 0; q < B; ++q) {
                int m = b * B + q;
                Stream st = make_stream(seed, (uint32_t)p, (uint32_t)m, (uint32_t)instance);
                WalkCount c;
                DiffOut o = diff_walk(sc, X + p * D, start_of(sc, p), st, c, true, cv);
                ud[q] = o.udot; uh[q] = o.u; us += o.u;
                st_steps[t] += c.steps + o.nested_steps;
            }
            double S = 0;
            for (int q = 0; q < B; ++q) S += uh[q];
            // U-statistic: 1/(B(B-1)) sum_m udot_m (S - u_m); minus uref * mean udot
            for (int q = 0; q < B; ++q) {
                double wq = (S - uh[q]) / ((double)B * (B - 1)) - uref[p] / B;
                for (int j = 0; j < N; ++j) gsum[j] += wq * ud[q][j];
            }
        }
        for (int j = 0; j < N; ++j) part[t][j] += gsum[j] / nb;
        double mean = us / W;
        if (u_mean) u_mean[p] = mean;
        lpart[t] += 0.5 * (mean - uref[p]) * (mean - uref[p]);
    });
    double L = 0;
    for (int t = 0; t < T; ++t) L += lpart[t];
    if (loss) *loss = L;
    for (int j = 0; j < N; ++j) { double a = 0; for (int t = 0; t < T; ++t) a += part[t][j]; grad[j] = a; }
    if (steps_total) { int64_t a = 0; for (auto v : st_steps) a += v; *steps_total = a; }
    return 0;
}

// ----- control variate --------------------------------------------------
// N, grad N (n x dim) and Lap N at n points (grad and lap may be NULL).
int oracle_mlp_eval(int32_t dim, int32_t F, const double* B, const double* theta,
                    const double* X, int64_t n, double* N, double* grad, double* lap) {
    if ((dim != 2 && dim != 3) || F < 0 || 2 * F + dim > kWidth || n < 0) return 1;
    for (int64_t i = 0; i < n; ++i) {
        MlpOut o = mlp_eval(dim, F, B, theta, X + i * dim);
        N[i] = o.N;
        if (grad) for (int c = 0; c < dim; ++c) grad[i * dim + c] = o.grad[c];
        if (lap) lap[i] = o.lap;
    }
    return 0;
}

int32_t oracle_mlp_theta_size(void) { return kThetaSize; }

// loss = sum_i 1/2 w_i (N(x_i) - t_i)^2 (w may be NULL: all 1); grad
// (kThetaSize) is overwritten with d loss / d theta.
int oracle_mlp_loss_grad(int32_t dim, int32_t F, const double* B, const double* theta,
                         const double* X, const double* T, const double* w, int64_t n,
                         double* loss, double* grad) {
    if ((dim != 2 && dim != 3) || F < 0 || 2 * F + dim > kWidth || n < 0) return 1;
    std::fill(grad, grad + kThetaSize, 0.0);
    double L = mlp_loss_grad(dim, F, B, theta, X, T, w, n, grad);
    if (loss) *loss = L;
    return 0;
}

// grad (kThetaSize) := d/dtheta sum_i (Nbar_i N(x_i) + Lbar_i Lap N(x_i)).
int oracle_mlp_vjp(int32_t dim, int32_t F, const double* B, const double* theta, const double* X,
                   const double* Nbar, const double* Lbar, int64_t n, double* grad) {
    if ((dim != 2 && dim != 3) || F < 0 || 2 * F + dim > kWidth || n < 0) return 1;
    std::fill(grad, grad + kThetaSize, 0.0);
    for (int64_t i = 0; i < n; ++i)
        mlp_vjp(dim, F, B, theta, X + i * dim, Nbar[i], Lbar ? Lbar[i] : 0.0, grad);
    return 0;
}

// One Adam step (Kingma and Ba, ICLR 2015, Algorithm 1) on n parameters;
// step is the 1-based step count used in the bias corrections.
void oracle_adam(int64_t n, double* theta, double* m, double* v, const double* g, double lr,
                 double beta1, double beta2, double eps, int64_t step) {
    double c1 = 1 - std::pow(beta1, (double)step), c2 = 1 - std::pow(beta2, (double)step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1 - beta2) * g[i] * g[i];
        theta[i] -= lr * (m[i] / c1) / (std::sqrt(v[i] / c2) + eps);
    }
}

// Differential-walk records with the control variate.
// walk (P*W*9): run, xoff[3], uoff (plain nested mean), uoff_cv, target, u, prim
// nested (P*W*K*10): S, alive, xstop[3], y[3], rho, d  (zeros when not run)
int oracle_walk_records_cv(const oracle_scene* s, const oracle_cv* cv, const double* X,
                           int64_t P, int32_t W, uint64_t seed, int32_t instance,
                           double* walk, double* nested, int threads) {
    if (check_scene(s) || !cv || W < 1 || P < 0 || check_starts(s, P)) return 1;
    if (s->n_ns > 0 || s->n_mono > 0 || s->dudn != 0) return 1;   // the control variate is for walk on spheres only
    Scene sc(*s);
    const int D = s->dim, K = s->K;
    parallel_points(P, threads, [&](int, int64_t p) {
        for (int m = 0; m < W; ++m) {
            size_t id = (size_t)p * W + m;
            Stream st = make_stream(seed, (uint32_t)p, (uint32_t)m, (uint32_t)instance);
            WalkCount c;
            DiffOut o = diff_walk(sc, X + p * D, start_of(sc, p), st, c, false, cv);
            double* r = walk + id * 9;
            r[0] = o.run;
            for (int i = 0; i < 3; ++i) r[1 + i] = o.xoff[i];
            r[4] = o.run >= 0 ? o.uoff : 0.0;
            r[5] = o.run >= 0 ? o.uoff_cv : 0.0;
            r[6] = o.target; r[7] = o.u;
            r[8] = o.terminal ? o.prim : -1;
            for (int i = 0; i < K; ++i) {
                double* q = nested + (id * K + i) * 10;
                std::fill(q, q + 10, 0.0);
                if (i >= (int)o.traces.size()) continue;
                const CvTrace& t = o.traces[i];
                q[0] = t.S; q[1] = t.alive ? 1 : 0;
                for (int c2 = 0; c2 < 3; ++c2) { q[2 + c2] = t.xstop[c2]; q[5 + c2] = t.y[c2]; }
                q[8] = t.rho; q[9] = t.d;
            }
        }
    });
    return 0;
}

}  // extern "C"
