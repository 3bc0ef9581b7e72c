// Host check of the multiply-shift division used by the kernels for lattice
// coordinates: floor(n / d) for every divisor 1..70000 against many
// numerators (edge values and random ones), every numerator below 2^31 for
// small divisors (sampled with a stride for the rest), and a few very large
// divisors.  Prints "ok" and exits 0 when every quotient matches.
#include <cstdint>
#include <cstdio>
#include <random>

#include "kernel_api.hpp"

int main() {
  using feod::fastdiv;
  using feod::make_fastdiv;
  std::mt19937_64 rng(12345);
  long bad = 0, checks = 0;
  auto check = [&](uint32_t n, uint32_t d, const feod::FastDiv& f) {
    ++checks;
    if (fastdiv(n, f) != n / d) {
      if (bad < 5) std::printf("mismatch: %u / %u\n", n, d);
      ++bad;
    }
  };
  for (uint32_t d = 1; d <= 70000; ++d) {
    const feod::FastDiv f = make_fastdiv(d);
    for (uint32_t i = 0; i < 64; ++i) {
      check(0x7fffffffu - i, d, f);
      const uint64_t m = (uint64_t)i * d + (d - 1);
      if (m <= 0x7fffffffu) check((uint32_t)m, d, f);
      check((uint32_t)(rng() & 0x7fffffffu), d, f);
    }
  }
  for (uint32_t d : {1u, 2u, 3u, 5u, 7u}) {
    const feod::FastDiv f = make_fastdiv(d);
    for (uint64_t n = 0; n <= 0x7fffffffull; n += 1 + 6 * (d > 3)) check((uint32_t)n, d, f);
  }
  for (uint32_t d : {97u, 129u, 193u, 257u, 513u, 1025u, 4097u}) {
    const feod::FastDiv f = make_fastdiv(d);
    for (uint64_t n = 0; n <= 0x7fffffffull; n += 997) check((uint32_t)n, d, f);
  }
  for (uint32_t d : {0x7fffffffu, 0x80000000u, 0x40000001u, 12345679u}) {
    const feod::FastDiv f = make_fastdiv(d);
    for (int i = 0; i < 200000; ++i) check((uint32_t)(rng() & 0x7fffffffu), d, f);
  }
  std::printf("%s: %ld checks, %ld mismatches\n", bad ? "FAILED" : "ok", checks, bad);
  return bad != 0;
}
