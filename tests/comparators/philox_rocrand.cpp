// Test comparator: raw Philox4x32-10 blocks from rocRAND's open-source header.
// Reads lines "c0 c1 c2 c3 k0 k1" (decimal) and prints the four output words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct probe : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    probe p;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint4 r = p.run(uint4{c0, c1, c2, c3}, uint2{k0, k1});
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
