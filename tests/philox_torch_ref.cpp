// Black-box known-answer helper: drives PyTorch's own Philox4x32-10 engine
// (ATen/core/PhiloxRNGEngine.h, a third-party implementation of the same
// published generator) so the tests can compare the oracle's generator
// against it.  Reads "c0 c1 c2 c3 k0 k1" lines (decimal) and prints the four
// output words of each block.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    // the engine's state maps key = seed, counter = (offset, subsequence)
    const uint64_t seed = (uint64_t)k0 | ((uint64_t)k1 << 32);
    const uint64_t subsequence = (uint64_t)c2 | ((uint64_t)c3 << 32);
    const uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
    at::philox_engine eng(seed, subsequence, offset);
    uint32_t o[4];
    for (int i = 0; i < 4; ++i) o[i] = eng();
    std::printf("%u %u %u %u\n", o[0], o[1], o[2], o[3]);
  }
  return 0;
}
