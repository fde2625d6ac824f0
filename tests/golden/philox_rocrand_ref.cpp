// Independent reference for Philox4x32-10: AMD's open-source rocRAND engine
// (rocrand/rocrand_philox4x32_10.h), run on the host.  Reads lines
// "key c0 c1 c2 c3" and prints the four output words for that counter.  The
// engine addresses counter (c0, c1, c2, c3) as subsequence c2 | c3 << 32 plus
// an offset of 4 * (c0 | c1 << 32) numbers, applied in pieces that fit 64 bits.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main() {
  unsigned long long key; unsigned c0, c1, c2, c3;
  while (scanf("%llu %u %u %u %u", &key, &c0, &c1, &c2, &c3) == 5) {
    unsigned long long sub = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long x = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
    rocrand_device::philox4x32_10_engine e(key, sub, 0ull);
    for (int q = 0; q < 4; ++q) e.discard(4ull * (x >> 2));
    e.discard(4ull * (x & 3ull));
    unsigned a = e(), b = e(), c = e(), d = e();
    printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
