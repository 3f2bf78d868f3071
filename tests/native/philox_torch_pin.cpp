// Independent Philox4x32-10 implementation for a test pin: PyTorch's
// at::philox_engine (a header-only implementation of the same published
// generator).  Reads lines "c0 c1 c2 c3 k0 k1" on stdin and prints the four
// output words of the block at that counter and key.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
    unsigned long long c0, c1, c2, c3, k0, k1;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        uint64_t seed = (k1 << 32) | k0;
        at::philox_engine eng(seed, (c3 << 32) | c2, 0);
        eng.set_offset((c1 << 32) | c0);
        uint32_t w[4];
        for (int i = 0; i < 4; ++i) w[i] = eng();
        std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
