// Reads lines "seed c0 c1 c2 c3" on stdin and prints the four words of
// Philox-4x32-10 at that counter and key, computed by rocRAND's host-callable
// engine.  Used only to pin the oracle's own Philox implementation.
#include <rocrand/rocrand_philox4x32_10.h>

#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    // rocRAND: key = seed; counter words 2,3 = subsequence; words 0,1 =
    // offset / 4 with the offset counted in 32-bit outputs.
    unsigned long long subseq = c2 | (c3 << 32);
    unsigned long long offset = 4ull * (c0 | (c1 << 32));
    rocrand_device::philox4x32_10_engine e(seed, subseq, offset);
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
