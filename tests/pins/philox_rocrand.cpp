// Independent Philox4x32-10 reference for the tests: rocRAND's host-callable
// engine (its ten_rounds() is protected, so a derived struct exposes it).
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) from stdin and prints the four
// output words per line.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

struct Engine : rocrand_device::philox4x32_10_engine {
    uint4 block(uint4 ctr, uint2 key) { return ten_rounds(ctr, key); }
};

int main() {
    Engine e;
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = e.block(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
