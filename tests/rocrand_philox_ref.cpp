// Host-side reference for the Philox4x32-10 pin: reads "seed c0 c1 c2 c3"
// lines and prints the four output words of rocRAND's philox4x32_10 engine
// for that key and counter.  rocRAND keys the engine with (lo32(seed),
// hi32(seed)) and starts its counter at (offset/4 as 64 bits in words 0-1,
// subsequence as 64 bits in words 2-3), so the counter is set exactly.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>

int main() {
    unsigned long long seed;
    unsigned c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long subsequence = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long block = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 0);
        // skip 4 * block outputs in four steps of block outputs each, so the
        // 64-bit offset cannot overflow
        for (int r = 0; r < 4; ++r) eng.discard(block);
        unsigned o0 = eng(), o1 = eng(), o2 = eng(), o3 = eng();
        std::printf("%u %u %u %u\n", o0, o1, o2, o3);
    }
    return 0;
}
