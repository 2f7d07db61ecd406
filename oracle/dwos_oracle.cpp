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
//     backward-difference normal derivative (eq. (dudn_fd_estimate)), the
//     joint solution estimate from the same walk (Sec. 5.1, observation 2)
//     and K nested forward walks per differential walk (Table 1).
//   * Differential boundary data for restricted fields
//     (eq. (boundary_deriv_restricted)) and for mapped data
//     (eq. (boundary_deriv_mapped), Appendix A).
//   * Reverse-mode accumulation with the U-statistic product estimator
//     (Sec. 5.3, eq. (ustatistics)).
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
//     flipped so that n.(xbar - x) >= 0 (points out of the domain).  The
//     closest primitive is the lowest-index one among those whose squared
//     distance is within a relative 1e-12 of the minimum.
//   * Walk-length cap kmax: the kmax-th query is treated as terminal.
//   * Mapped data: udot = gdot_ref - grad_G g . V - V_n du/dn (Appendix A
//     with tangential components of the velocity kept explicitly).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>
#include <algorithm>

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
// purpose bit 1: nested walk; bit 2: second draw of a step (source sample).
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
    explicit Scene(const oracle_scene& sc) : s(sc), D(sc.dim) {}
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
    // oriented so that it points from x towards xbar (out of the domain).
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

struct WalkCount { int64_t steps = 0; int64_t truncated = 0; };

// ---------------------------------------------------------------------------
// Algorithm 1: WalkOnSpheres(x, eps).  The recursion
//   u(x_k) = S_k + [continue] u(x_{k+1})
// is tail-recursive with an additive term, so it is unrolled into a loop that
// carries the running sum of source contributions.
// ---------------------------------------------------------------------------
double walk_on_spheres(const Scene& sc, const double* x0, const Stream& st, uint32_t extra,
                       WalkCount& cnt) {
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
            return acc + sc.g(h);
        }
        uint32_t w[4];
        st.draw(k, extra, w);
        if (sc.has_source()) {                          // source contribution
            uint32_t wb[4];
            st.draw(k, extra | 2u, wb);
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

struct DiffOut {
    double u = 0;          // joint estimate of u (sources + g at the terminal)
    bool terminal = false; // reached the shell (false: stopped by roulette)
    int prim = -1;
    double xbar[3] = {0, 0, 0};   // terminal closest point
    double uoff = 0;       // mean of the K nested walks at the offset point
    int64_t nested_steps = 0;
    std::vector<double> udot;  // dense N-vector
};

// ---------------------------------------------------------------------------
// Algorithm 2: DiffWalkOnSpheres(x, eps, delta).  The walk follows the same
// steps (and random numbers) as Algorithm 1 so that it also returns the joint
// estimate of u.  At the shell it launches K forward walks from the offset
// point xbar - delta n and forms the differential boundary value.
// ---------------------------------------------------------------------------
DiffOut diff_walk_on_spheres(const Scene& sc, const double* x0, const Stream& st,
                             WalkCount& cnt, bool want_udot) {
    const int D = sc.D;
    const int N = sc.s.N;
    DiffOut out;
    if (want_udot) out.udot.assign(N, 0.0);
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
            double n[3];
            sc.normal(h, x, n);                                // BoundaryNormal
            double xoff[3] = {0, 0, 0};
            for (int i = 0; i < D; ++i) xoff[i] = h.xbar[i] - sc.s.delta * n[i];
            double usum = 0;
            for (int i = 0; i < sc.s.K; ++i) {                 // nested forward walks
                WalkCount c2;
                usum += walk_on_spheres(sc, xoff, st, 1u | ((uint32_t)i << 8), c2);
                out.nested_steps += c2.steps;
                cnt.truncated += c2.truncated;
            }
            double uhat = usum / sc.s.K;
            double gx = sc.g(h);
            double dudn = (gx - uhat) / sc.s.delta;            // eq. (dudn_fd_estimate)
            out.u = acc + gx;
            out.terminal = true;
            out.prim = h.prim;
            for (int i = 0; i < 3; ++i) out.xbar[i] = h.xbar[i];
            out.uoff = uhat;
            if (want_udot) {
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
                    double val;
                    if (mp) {
                        // gdot_ref - grad_G g . V - V_n du/dn
                        val = gdot[j] - dot(gr, V, D) - Vn * dudn;
                    } else {
                        // eq. (boundary_deriv_restricted): gdot_field (= 0) + (dg/dn - du/dn) V_n
                        val = (dgdn - dudn) * Vn;
                    }
                    out.udot[j] = val;
                }
            }
            return out;
        }
        uint32_t w[4];
        st.draw(k, 0u, w);
        if (sc.has_source()) {   // sources only enter the joint u estimate
            uint32_t wb[4];
            st.draw(k, 2u, wb);
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
        for (int i = 0; i < D; ++i) x[i] += d * s[i];
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
    if (!s || (s->dim != 2 && s->dim != 3) || s->nv <= 0 || s->np <= 0) return 1;
    if (!(s->eps > 0) || s->sigma < 0 || s->K < 1 || s->kmax < 1) return 1;
    return 0;
}

}  // namespace

extern "C" {

int oracle_threads(void) { return (int)std::max(1u, std::thread::hardware_concurrency()); }

void oracle_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    philox4x32_10(ctr, key, out);
}

double oracle_green(int dim, double sigma, double r, double R) { return green(dim, sigma, r, R); }
double oracle_poisson_scale(int dim, double sigma, double R) { return poisson_scale(dim, sigma, R); }

// closest point: out = {d, prim, bary0, bary1, bary2, xbar0, xbar1, xbar2}
int oracle_closest(const oracle_scene* s, const double* x, double* out) {
    if (check_scene(s)) return 1;
    Scene sc(*s);
    Hit h = sc.closest(x);
    out[0] = std::sqrt(h.d2); out[1] = h.prim;
    for (int i = 0; i < 3; ++i) { out[2 + i] = h.bary[i]; out[5 + i] = h.xbar[i]; }
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
    if (check_scene(s) || W < 1 || P < 0) return 1;
    Scene sc(*s);
    const int D = s->dim;
    std::vector<int64_t> trunc(std::max(1, threads > 0 ? threads : oracle_threads()) + 64, 0);
    parallel_points(P, threads, [&](int t, int64_t p) {
        for (int m = 0; m < W; ++m) {
            size_t id = (size_t)p * W + m;
            Stream st = make_stream(seed, (uint32_t)p, (uint32_t)m, (uint32_t)instance);
            WalkCount c;
            if (mode == 0) {
                u[id] = walk_on_spheres(sc, X + p * D, st, 0u, c);
                if (prim) prim[id] = -1;
                if (uoff) uoff[id] = 0;
            } else {
                DiffOut o = diff_walk_on_spheres(sc, X + p * D, st, c, udot != nullptr);
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
    if (check_scene(s) || W < 1 || P < 0) return 1;
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
            double v = walk_on_spheres(sc, X + p * D, st, 0u, c);
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
               int64_t* steps_total, int threads) {
    if (check_scene(s) || W < 1 || P < 0) return 1;
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
            DiffOut o = diff_walk_on_spheres(sc, X + p * D, st, c, true);
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
                int64_t* steps_total, int threads) {
    if (check_scene(s) || W < 1 || P < 0) return 1;
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
            DiffOut o = diff_walk_on_spheres(sc, X + p * D, st, c, true);
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
                       double* grad, double* u_mean, int64_t* steps_total, int threads) {
    if (check_scene(s) || W < 1 || P < 0 || B < 2 || W % B != 0) return 1;
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
                DiffOut o = diff_walk_on_spheres(sc, X + p * D, st, c, true);
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

}  // extern "C"
