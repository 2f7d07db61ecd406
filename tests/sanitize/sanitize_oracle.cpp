// Drives the oracle's entry points on small scenes for an AddressSanitizer /
// UndefinedBehaviorSanitizer build (tests/test_sanitizers.py compiles this
// file together with oracle/dwos_oracle.cpp and runs it): forward and
// differential walks on spheres in 2D and 3D (sources, screening, nested
// walks, mapped and restricted data), walks on stars with reflecting walls
// and a Robin condition, an implicit boundary, the adjoint formulation and
// the control-variate network.  Exit 0 and no sanitizer report = clean.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../oracle/dwos_oracle.cpp"

namespace {

int fails = 0;
void check(int rc, const char* what) {
    if (rc != 0) { std::printf("FAIL %s rc=%d\n", what, rc); ++fails; }
}

struct Scene2D {
    std::vector<double> V, quad, gv, vel, NV, gauss, rquad;
    std::vector<int32_t> P, lab, kind, pid, ns, start;
    std::vector<int64_t> rowptr;
    oracle_scene s{};
};

// regular n-gon of radius R, parameter R (dv/dR = v/R), restricted x^2 - y^2
void polygon(Scene2D& sc, int n, double R, double sigma, int K) {
    for (int i = 0; i < n; ++i) {
        const double t = 2 * M_PI * i / n;
        sc.V.push_back(R * std::cos(t)); sc.V.push_back(R * std::sin(t));
        sc.P.push_back(i); sc.P.push_back((i + 1) % n);
        sc.lab.push_back(0);
        sc.gv.push_back(std::cos(2 * t));
        sc.rowptr.push_back(i);
        sc.pid.push_back(0);
        sc.vel.push_back(std::cos(t)); sc.vel.push_back(std::sin(t));
    }
    sc.rowptr.push_back(n);
    sc.kind = {0};
    sc.quad = {0.1, 0.2, -0.1, 1.0, 0.0, 0.0, -1.0};
    sc.gauss = {50.0, 0.2, 0.1, 0.2};
    oracle_scene& s = sc.s;
    s.dim = 2; s.nv = n; s.V = sc.V.data(); s.np = n; s.prims = sc.P.data(); s.label = sc.lab.data();
    s.sigma = sigma; s.eps = 1e-3; s.delta = 1e-2; s.K = K; s.kmax = 4096; s.rr = 1;
    s.src_c0 = 1.0; s.n_gauss = 1; s.gauss = sc.gauss.data();
    s.n_labels = 1; s.bc_kind = sc.kind.data(); s.bc_quad = sc.quad.data(); s.gvert = sc.gv.data();
    s.N = 1; s.rowptr = sc.rowptr.data(); s.pid = sc.pid.data(); s.vel = sc.vel.data();
}

void run_walks(const oracle_scene& s, const std::vector<double>& X, int W, const char* tag) {
    const int64_t P = (int64_t)X.size() / s.dim;
    std::vector<double> m(P), v(P), um(P), jm(P * s.N), jv(P * s.N), g(s.N), w(P, 1.0), uref(P, 0.2),
        u(P * W), ud(P * W * s.N), uo(P * W), xb(P * W * 3), L(1);
    std::vector<int64_t> st(P * W), tr(1), tot(1);
    std::vector<int32_t> pr(P * W);
    check(oracle_solve(&s, X.data(), P, W, 7, 0, m.data(), v.data(), tot.data(), 2), tag);
    check(oracle_jvp(&s, X.data(), P, W, 8, 0, jm.data(), jv.data(), um.data(), tot.data(), 2, nullptr), tag);
    check(oracle_grad(&s, X.data(), P, w.data(), W, 9, 0, g.data(), um.data(), tot.data(), 2, nullptr), tag);
    check(oracle_grad_sqloss(&s, X.data(), P, uref.data(), W, 4, 10, 0, L.data(), g.data(), um.data(),
                             tot.data(), 2, nullptr), tag);
    for (int mode = 0; mode < 2; ++mode)
        check(oracle_walk_records(&s, X.data(), P, W, 11, mode, 0, u.data(), ud.data(), st.data(), pr.data(),
                                  uo.data(), tr.data(), xb.data(), 2), tag);
    for (double e : m) if (!std::isfinite(e)) { std::printf("FAIL %s non-finite mean\n", tag); ++fails; break; }
}

}  // namespace

int main() {
    // 2D polygon: source, screening, K = 2 nested walks, restricted and mapped data
    {
        Scene2D sc;
        polygon(sc, 48, 1.0, 4.0, 2);
        std::vector<double> X = {0.1, 0.2, -0.3, 0.4, 0.5, -0.1};
        run_walks(sc.s, X, 16, "polygon restricted");
        sc.kind[0] = 1;
        run_walks(sc.s, X, 16, "polygon mapped");
    }
    // walk on stars: reflecting diameter of a half disk with a Robin condition
    {
        Scene2D sc;
        const int n = 32;
        for (int i = 0; i <= n; ++i) {
            const double t = M_PI * i / n;
            sc.V.push_back(std::cos(t)); sc.V.push_back(std::sin(t));
            sc.rowptr.push_back(i); sc.pid.push_back(0);
            sc.vel.push_back(std::cos(t)); sc.vel.push_back(std::sin(t));
            sc.gv.push_back(0.0);
        }
        sc.rowptr.push_back(n + 1);
        for (int i = 0; i < n; ++i) { sc.P.push_back(i); sc.P.push_back(i + 1); sc.lab.push_back(0); }
        for (int i = 0; i <= 8; ++i) { sc.NV.push_back(-1.0 + 2.0 * i / 8); sc.NV.push_back(0.0); }
        for (int i = 0; i < 8; ++i) { sc.ns.push_back(i); sc.ns.push_back(i + 1); }
        sc.kind = {0};
        sc.quad = {0.0, 0.0, 1.0, 1.0, 0.0, 0.0, -1.0};
        sc.rquad = {1.0, 0.0, 0.0, -0.7, 0.0, 0.0, 0.0};
        oracle_scene& s = sc.s;
        s.dim = 2; s.nv = n + 1; s.V = sc.V.data(); s.np = n; s.prims = sc.P.data(); s.label = sc.lab.data();
        s.sigma = 1.0; s.eps = 1e-3; s.delta = 1e-2; s.K = 1; s.kmax = 4096; s.rr = 1;
        s.n_labels = 1; s.bc_kind = sc.kind.data(); s.bc_quad = sc.quad.data(); s.gvert = sc.gv.data();
        s.N = 1; s.rowptr = sc.rowptr.data(); s.pid = sc.pid.data(); s.vel = sc.vel.data();
        s.n_nv = 9; s.NV = sc.NV.data(); s.n_ns = 8; s.nsegs = sc.ns.data();
        s.robin_mu = 0.7; s.robin_quad = sc.rquad.data();
        std::vector<double> X = {0.1, 0.3, -0.4, 0.2, 0.3, 0.5};
        run_walks(s, X, 16, "robin half disk");
        sc.start = {2, -1, 5};
        std::vector<double> Xw = {-0.45, 0.0, -0.4, 0.2, 0.3, 0.0};
        s.start_seg = sc.start.data();
        run_walks(s, Xw, 16, "robin half disk, wall starts");
        double out[1];
        const double nin[2] = {0.0, 1.0};
        check(oracle_silhouette(&s, X.data(), -1, nin, 2.0, out), "silhouette");
    }
    // 3D: an octahedron (g = 1, parameter: its scale) inside a box (g = 0)
    {
        std::vector<double> V = {-2, -2, -2, 2, -2, -2, -2, 2, -2, 2, 2, -2, -2, -2, 2, 2, -2, 2, -2, 2, 2, 2, 2, 2,
                                 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
        std::vector<int32_t> P = {0, 1, 3, 0, 3, 2, 4, 6, 7, 4, 7, 5, 0, 4, 5, 0, 5, 1, 2, 3, 7, 2, 7, 6,
                                  0, 2, 6, 0, 6, 4, 1, 5, 7, 1, 7, 3,
                                  8, 10, 12, 10, 9, 12, 9, 11, 12, 11, 8, 12, 10, 8, 13, 9, 10, 13, 11, 9, 13, 8, 11, 13};
        std::vector<int32_t> lab(20, 0);
        for (int i = 12; i < 20; ++i) lab[i] = 1;
        std::vector<int32_t> kind = {0, 0};
        std::vector<double> quad = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0,
                                    1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        std::vector<double> gv(14, 0.0), vel;
        std::vector<int64_t> rowptr(15, 0);
        std::vector<int32_t> pid;
        for (int i = 0; i < 14; ++i) {
            rowptr[i + 1] = rowptr[i];
            if (i >= 8) {
                pid.push_back(0);
                for (int c = 0; c < 3; ++c) vel.push_back(V[3 * i + c]);
                rowptr[i + 1] += 1;
            }
        }
        oracle_scene s{};
        s.dim = 3; s.nv = 14; s.V = V.data(); s.np = 20; s.prims = P.data(); s.label = lab.data();
        s.sigma = 4.0; s.eps = 4e-3; s.delta = 4e-2; s.K = 3; s.kmax = 4096; s.rr = 1;
        s.n_labels = 2; s.bc_kind = kind.data(); s.bc_quad = quad.data(); s.gvert = gv.data();
        s.N = 1; s.rowptr = rowptr.data(); s.pid = pid.data(); s.vel = vel.data();
        std::vector<double> X = {1.5, 0.2, 0.1, -0.3, 1.6, 0.4, 0.5, -0.5, -1.7};
        run_walks(s, X, 16, "3D octahedron in a box");
    }
    // implicit boundary: two monopoles
    {
        std::vector<double> mono = {0.3, -0.2, 0.0, 0.25, 0.25, 0.1};
        std::vector<int32_t> kind = {0};
        std::vector<double> quad = {0.0, 0.0, 0.0, 1.0, 0.0, 0.0, -1.0};
        oracle_scene s{};
        s.dim = 2; s.sigma = 0.0; s.eps = 1e-3; s.delta = 1e-2; s.K = 2; s.kmax = 4096; s.rr = 1;
        s.src_c0 = 4.0; s.n_labels = 1; s.bc_kind = kind.data(); s.bc_quad = quad.data();
        s.N = 6; s.n_mono = 2; s.mono = mono.data(); s.mono_c = -1.0;
        std::vector<double> X = {-0.2, 0.05, 0.25, 0.2};
        run_walks(s, X, 16, "implicit monopoles");
    }
    // the control-variate network: evaluation, loss gradient, vector-Jacobian product, Adam
    {
        const int F = 4, D = 2, n = 5;
        std::vector<double> B = {0.3, -0.2, 0.1, 0.4, -0.5, 0.2, 0.25, 0.15}, theta(kThetaSize);
        for (size_t i = 0; i < theta.size(); ++i) theta[i] = 0.01 * std::sin(0.37 * (double)i);
        std::vector<double> X = {0.1, 0.2, 0.3, -0.1, -0.4, 0.5, 0.0, 0.0, 0.9, -0.9};
        std::vector<double> N(n), G(n * 3), Lp(n), T(n, 0.3), g(kThetaSize), Nb(n, 1.0), Lb(n, 0.5), loss(1);
        check(oracle_mlp_eval(D, F, B.data(), theta.data(), X.data(), n, N.data(), G.data(), Lp.data()), "mlp eval");
        check(oracle_mlp_loss_grad(D, F, B.data(), theta.data(), X.data(), T.data(), nullptr, n, loss.data(),
                                   g.data()), "mlp loss");
        check(oracle_mlp_vjp(D, F, B.data(), theta.data(), X.data(), Nb.data(), Lb.data(), n, g.data()), "mlp vjp");
        std::vector<double> mm(kThetaSize, 0.0), vv(kThetaSize, 0.0);
        oracle_adam(kThetaSize, theta.data(), mm.data(), vv.data(), g.data(), 1e-3, 0.9, 0.999, 1e-8, 1);
    }
    std::printf("%s\n", fails ? "sanitize_oracle: failures" : "sanitize_oracle: ok");
    return fails ? 1 : 0;
}
