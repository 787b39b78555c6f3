// Host build of the GPU library's random-stream header, for comparison with
// the CPU oracle.  Prints the sample keys and K-means++ words of a few points,
// then an xor-fold over a strided range.
#include <cstdio>
#include <cstdlib>

#include "../paper_2204_07485_amd/csrc/bm_rng.h"

int main(int argc, char** argv) {
  const long n = argc > 1 ? std::atol(argv[1]) : 1000000;
  const unsigned long long seed = argc > 2 ? std::strtoull(argv[2], nullptr, 10) : 1;
  const unsigned t = 7;
  auto key = [&](long i) {
    uint64_t e, o;
    bm::sample_key_pair(seed, t, static_cast<unsigned long long>(i) >> 1, e, o);
    return (i & 1) ? o : e;
  };
  const long spots[4] = {0, 1, n - 1, n / 2 + 1};
  for (long i : spots) std::printf("%llu\n", static_cast<unsigned long long>(key(i)));
  for (long q : spots) std::printf("%llu\n", static_cast<unsigned long long>(bm::seed_draw(seed, t, static_cast<uint64_t>(q))));
  uint64_t fold = 0;
  for (long i = 0; i < n; i += 997) fold ^= key(i) ^ bm::seed_draw(seed, t, static_cast<unsigned long long>(i));
  std::printf("%llu\n", static_cast<unsigned long long>(fold));
  return 0;
}
