// Drives the library's host code -- the BVH builder (bvh_build.cpp) and the
// remesher (remesh.cpp) -- on small meshes for an AddressSanitizer /
// UndefinedBehaviorSanitizer build (tests/test_sanitizers.py compiles this
// file with those two sources and runs it).  Exit 0 and no sanitizer report
// = clean.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../include/dwos.h"
#include "../../paper_2405_12964_amd/csrc/bvh.hpp"

namespace {

int fails = 0;
void expect(bool ok, const char* what) {
    if (!ok) { std::printf("FAIL %s\n", what); ++fails; }
}

// octahedron subdivided `levels` times, vertices pushed to the unit sphere
void sphere_mesh(int levels, std::vector<double>& V, std::vector<int32_t>& T) {
    V = {1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
    T = {0, 2, 4, 2, 1, 4, 1, 3, 4, 3, 0, 4, 2, 0, 5, 1, 2, 5, 3, 1, 5, 0, 3, 5};
    for (int l = 0; l < levels; ++l) {
        std::vector<int32_t> out;
        std::vector<std::pair<std::pair<int, int>, int>> mids;
        auto mid = [&](int a, int b) {
            if (a > b) std::swap(a, b);
            for (auto& m : mids) if (m.first.first == a && m.first.second == b) return m.second;
            double p[3];
            double n = 0;
            for (int c = 0; c < 3; ++c) { p[c] = 0.5 * (V[3 * a + c] + V[3 * b + c]); n += p[c] * p[c]; }
            n = std::sqrt(n);
            for (int c = 0; c < 3; ++c) V.push_back(p[c] / n);
            const int id = (int)V.size() / 3 - 1;
            mids.push_back({{a, b}, id});
            return id;
        };
        for (size_t t = 0; t < T.size(); t += 3) {
            const int a = T[t], b = T[t + 1], c = T[t + 2];
            const int ab = mid(a, b), bc = mid(b, c), ca = mid(c, a);
            out.insert(out.end(), {a, ab, ca, ab, b, bc, ca, bc, c, ab, bc, ca});
        }
        T = out;
    }
}

void check_bvh(const std::vector<double>& V, const std::vector<int32_t>& P, int D, const char* what) {
    const int64_t np = (int64_t)P.size() / D;
    dwos::HostBVH b = dwos::build_bvh(V.data(), P.data(), np, D);
    dwos::reorder_bfs(b);
    expect((int64_t)b.order.size() == np, what);
    std::vector<int> seen(np, 0);
    for (int32_t o : b.order) if (o >= 0 && o < np) seen[o]++;
    for (int s : seen) if (s != 1) { expect(false, what); break; }
    expect(b.max_depth < dwos::kMaxDepth, what);
}

}  // namespace

int main() {
    std::vector<double> V;
    std::vector<int32_t> T;
    sphere_mesh(3, V, T);
    check_bvh(V, T, 3, "bvh sphere");
    // a random triangle soup and a random polyline
    std::mt19937 rng(5);
    std::uniform_real_distribution<double> U(-1, 1);
    std::vector<double> Vs;
    std::vector<int32_t> Ts;
    for (int i = 0; i < 300; ++i) {
        for (int k = 0; k < 9; ++k) Vs.push_back(U(rng));
        Ts.insert(Ts.end(), {3 * i, 3 * i + 1, 3 * i + 2});
    }
    check_bvh(Vs, Ts, 3, "bvh soup");
    std::vector<double> V2;
    std::vector<int32_t> S2;
    const int n = 200;
    for (int i = 0; i < n; ++i) {
        const double t = 2 * M_PI * i / n, r = 1 + 0.1 * std::sin(5 * t);
        V2.push_back(r * std::cos(t)); V2.push_back(r * std::sin(t));
        S2.push_back(i); S2.push_back((i + 1) % n);
    }
    check_bvh(V2, S2, 2, "bvh polyline");
    // remeshing: refine and coarsen a sphere, remesh a closed polyline with
    // fixed vertices, and the error paths
    for (double L : {0.1, 0.6}) {
        dwos_mesh* m = nullptr;
        expect(dwos_remesh(3, V.data(), (int64_t)V.size() / 3, T.data(), (int64_t)T.size() / 3, nullptr, L, 5, &m) ==
                   DWOS_OK, "remesh sphere");
        int64_t nv = 0, nt = 0;
        expect(dwos_mesh_size(m, &nv, &nt) == DWOS_OK && nv > 0 && nt > 0, "remesh size");
        std::vector<double> Vo(nv * 3);
        std::vector<int32_t> To(nt * 3);
        std::vector<int64_t> src(nv);
        expect(dwos_mesh_get(m, Vo.data(), To.data(), src.data()) == DWOS_OK, "remesh get");
        for (int32_t i : To) if (i < 0 || i >= nv) { expect(false, "remesh index"); break; }
        dwos_mesh_destroy(m);
    }
    std::vector<int32_t> fixed(n, 0);
    fixed[0] = fixed[50] = 1;
    dwos_mesh* m2 = nullptr;
    expect(dwos_remesh(2, V2.data(), n, S2.data(), n, fixed.data(), 0.02, 4, &m2) == DWOS_OK, "remesh polyline");
    dwos_mesh_destroy(m2);
    dwos_mesh* bad = nullptr;
    expect(dwos_remesh(3, V.data(), (int64_t)V.size() / 3, T.data(), (int64_t)T.size() / 3, nullptr, -1.0, 5, &bad) ==
               DWOS_EINVAL, "remesh error path");
    std::printf("%s\n", fails ? "sanitize_host: failures" : "sanitize_host: ok");
    return fails ? 1 : 0;
}
