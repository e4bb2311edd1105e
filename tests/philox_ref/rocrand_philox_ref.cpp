// Prints raw Philox4x32-10 blocks from ROCm's rocRAND engine (a library call),
// used to pin the oracle's Philox.  Reads lines "seed c0 c1 c2 c3" on stdin and
// writes "w0 w1 w2 w3".  The counter maps onto rocRAND's (subsequence, offset)
// as counter = (offset/4 low, offset/4 high, subsequence low, subsequence high).
#include <cstdio>
#include <cstdint>
#include <rocrand/rocrand_kernel.h>

int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    const unsigned long long subsequence = c2 | (c3 << 32);
    const unsigned long long offset = 4ull * (c0 | (c1 << 32));
    rocrand_device::philox4x32_10_engine eng(seed, subsequence, offset);
    unsigned w[4];
    for (int i = 0; i < 4; ++i) w[i] = eng();
    std::printf("%u %u %u %u\n", w[0], w[1], w[2], w[3]);
  }
  return 0;
}
