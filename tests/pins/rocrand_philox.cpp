// Independent Philox4x32-10 for pinning the oracle: rocRAND's header
// implementation, run on the host.  Reads lines "c0 c1 c2 c3 k0 k1" (uint32)
// from stdin and prints the four output words of the block at that counter
// under that key.  rocRAND's state maps (seed, subsequence, offset) to
// key = seed, counter = (offset / 4, subsequence), so c1 must stay below
// 2^30 for the offset to fit in 64 bits.
#include <rocrand/rocrand_kernel.h>
#include <cstdio>
#include <cstdint>

int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (std::scanf("%u %u %u %u %u %u", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
    unsigned long long subseq = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
    unsigned long long offset = 4ULL * ((unsigned long long)c0 | ((unsigned long long)c1 << 32));
    rocrand_state_philox4x32_10 st;
    rocrand_init(seed, subseq, offset, &st);
    unsigned a = rocrand(&st), b = rocrand(&st), c = rocrand(&st), d = rocrand(&st);
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
