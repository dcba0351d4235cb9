// Prints Philox4x32-10 words from PyTorch's own header-only engine
// (at::philox_engine), an implementation independent of this repository.
// Input lines: seed ctr0 ctr1 ctr2 ctr3 (decimal); output: four words.
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long seed, c0, c1, c2, c3;
  while (std::scanf("%llu %llu %llu %llu %llu", &seed, &c0, &c1, &c2, &c3) == 5) {
    // the engine's counter is {offset_lo, offset_hi, subsequence_lo, subsequence_hi}
    uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
    uint64_t subseq = (uint64_t)c2 | ((uint64_t)c3 << 32);
    at::philox_engine eng(seed, subseq, offset);
    unsigned w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
  return 0;
}
