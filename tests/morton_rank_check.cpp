// Host check of morton_rank (lpr_dev.h, a host-and-device function): every
// cell of random grids gets the rank of its Morton code among the grid's
// codes, found here by sorting all codes.
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "lpr_dev.h"

static uint64_t interleave(uint64_t x, uint64_t y, uint64_t z) {
  uint64_t m = 0;
  for (int b = 0; b < 21; ++b)
    m |= ((x >> b) & 1u) << (3 * b) | ((y >> b) & 1u) << (3 * b + 1) | ((z >> b) & 1u) << (3 * b + 2);
  return m;
}

int main() {
  std::mt19937 g(7);
  for (int t = 0; t < 200; ++t) {
    int32_t n[3] = {1 + (int32_t)(g() % 40), 1 + (int32_t)(g() % 40), 1 + (int32_t)(g() % 24)};
    if (t % 10 == 0) n[0] = 1 + (int32_t)(g() % 300);
    std::vector<uint64_t> codes;
    for (int z = 0; z < n[2]; ++z)
      for (int y = 0; y < n[1]; ++y)
        for (int x = 0; x < n[0]; ++x) codes.push_back(interleave(x, y, z));
    std::vector<uint64_t> sorted = codes;
    std::sort(sorted.begin(), sorted.end());
    size_t q = 0;
    for (int z = 0; z < n[2]; ++z)
      for (int y = 0; y < n[1]; ++y)
        for (int x = 0; x < n[0]; ++x, ++q) {
          const int32_t c[3] = {x, y, z};
          const uint64_t want = (uint64_t)(std::lower_bound(sorted.begin(), sorted.end(), codes[q]) - sorted.begin());
          const uint64_t got = lpr::morton_rank(c, n);
          if (got != want) {
            std::printf("grid %d %d %d cell %d %d %d: %llu, want %llu\n", n[0], n[1], n[2], x, y, z,
                        (unsigned long long)got, (unsigned long long)want);
            return 1;
          }
        }
  }
  std::printf("ok\n");
  return 0;
}
