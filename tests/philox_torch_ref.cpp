// Outside reference for Philox4x32-10: PyTorch's philox engine, used through
// its public interface only.  Reads lines "key c0 c1 c2 c3" on stdin and
// prints the four output words of that block.
#include <ATen/core/PhiloxRNGEngine.h>

#include <cstdint>
#include <cstdio>

int main() {
  unsigned long long key;
  unsigned c0, c1, c2, c3;
  while (std::scanf("%llu %u %u %u %u", &key, &c0, &c1, &c2, &c3) == 5) {
    // engine(seed, subsequence, offset): key = seed, counter = (offset, subsequence)
    uint64_t offset = (uint64_t)c0 | ((uint64_t)c1 << 32);
    uint64_t subsequence = (uint64_t)c2 | ((uint64_t)c3 << 32);
    at::Philox4_32 engine(key, subsequence, offset);
    uint32_t a = engine(), b = engine(), c = engine(), d = engine();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
  return 0;
}
