// Prints Philox4x32-10 blocks computed by rocRAND's host-callable engine, an
// implementation developed independently of this repository. Input lines:
// "k0 k1 c0 c1 c2 c3" (decimal uint32); output lines: four uint32 words.
// Used by the oracle's generator test as a known-answer source.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdio>

int main() {
  unsigned k0, k1, c0, c1, c2, c3;
  while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long subsequence = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long offset = 4ull * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
    uint4 r = eng.next4();
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
