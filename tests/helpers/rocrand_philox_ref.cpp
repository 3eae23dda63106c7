// Independent Philox4x32-10 reference for the oracle's generator: rocRAND's
// header-only engine, compiled for the host.  Reads lines "c0 c1 c2 c3 k0 k1"
// on stdin and prints the four 32-bit outputs of ten rounds for each.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

struct Engine : rocrand_device::philox4x32_10_engine {
    using rocrand_device::philox4x32_10_engine::ten_rounds;
};

int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    Engine eng;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = eng.ten_rounds(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
