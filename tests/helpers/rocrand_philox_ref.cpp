// Independent reference for the oracle's Philox-4x32-10: runs the generator
// that ships with ROCm's rocRAND (its header-only engine, on the host).
// Input lines: "k0 k1 c0 c1 c2 c3" (decimal); output: the 4 output words.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long k0, k1, c0, c1, c2, c3;
    while (std::scanf("%llu %llu %llu %llu %llu %llu", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        const unsigned long long seed = k0 | (k1 << 32);
        const unsigned long long subsequence = c2 | (c3 << 32);
        const unsigned long long offset = 4ull * (c0 | (c1 << 32));
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
        const uint4 r = eng.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
