// Test comparator: raw Philox4x32-10 blocks from PyTorch's open-source
// PhiloxRNGEngine.h.  The engine's key is the 64-bit seed, counter words 2,3
// are the subsequence and words 0,1 the offset; four calls return one block.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>
int main() {
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
        uint64_t sub = (uint64_t)c2 | ((uint64_t)c3 << 32);
        uint64_t off = (uint64_t)c0 | ((uint64_t)c1 << 32);
        at::philox_engine e(seed, sub, off);
        unsigned r0 = e(), r1 = e(), r2 = e(), r3 = e();
        std::printf("%u %u %u %u\n", r0, r1, r2, r3);
    }
    return 0;
}
