// Independent reference for the Philox4x32-10 pin: rocRAND's engine (host side).
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal uint32) from stdin and prints the
// four output words of ten rounds for each.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

// ten_rounds is a protected member of the engine; expose it.
struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 rounds(uint4 c, uint2 k) { return ten_rounds(c, k); }
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Engine eng;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 c = {c0, c1, c2, c3};
        uint2 k = {k0, k1};
        uint4 r = eng.rounds(c, k);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
