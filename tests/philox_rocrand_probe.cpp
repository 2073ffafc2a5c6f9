// Host-only probe: Philox4x32-10 outputs from rocRAND's engine, used as an
// independent library reference for the oracle's Philox. Reads lines
// "c0 c1 c2 c3 k0 k1" (decimal) from stdin and prints the four output words.
// rocRAND's engine(seed, subsequence, offset) starts at counter
// (offset/4 low, offset/4 high, subsequence low, subsequence high) with key
// (seed low, seed high).
#include <rocrand/rocrand_kernel.h>

#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    const unsigned long long seed = k0 | (k1 << 32);
    const unsigned long long sub = c2 | (c3 << 32);
    const unsigned long long offset = 4ull * (c0 | (c1 << 32));
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, sub, offset, &st);
    const uint4 r = rocrand4(&st);
    std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
  }
  return 0;
}
