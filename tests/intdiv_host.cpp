// Host check of hom::divmod62 (hom_intdiv.h, __host__ __device__; the start-point kernel's 64-bit
// quotients) against the compiler's exact 64-bit division.  Compiled for the host only and run
// by tests/test_intdiv_host.py.  Output: "checks <count> bad <count>".
#include <cstdint>
#include <cstdio>
#include <initializer_list>
#include <random>

#include "hom_intdiv.h"

int main(int argc, char **argv) {
  const long rounds = argc > 1 ? std::atol(argv[1]) : 1000000;
  std::mt19937_64 g(62);
  long bad = 0, n = 0;
  auto check = [&](int64_t q, int64_t d) {
    int64_t r;
    const int64_t t = hom::divmod62(q, d, 1.0 / (double)d, r);
    ++n;
    if (t != q / d || r != q % d) {
      if (bad < 5) std::printf("# q=%lld d=%lld t=%lld r=%lld\n", (long long)q, (long long)d,
                               (long long)t, (long long)r);
      ++bad;
    }
  };
  const int64_t qmax = ((int64_t)1 << 62) - 1, dmax = ((int64_t)1 << 31) - 1;
  // edges: the largest dividend, powers of two around 2^53, divisors 1, 2, small, 2^30, 2^31 - 1
  for (int64_t d : std::initializer_list<int64_t>{1, 2, 3, 7, 10, 32, 3881632, (int64_t)1 << 30,
                                                   ((int64_t)1 << 30) + 1, dmax - 1, dmax})
    for (int64_t q : std::initializer_list<int64_t>{0, 1, d - 1, d, d + 1, qmax, qmax - 1, qmax - d,
                                                     (int64_t)1 << 53, ((int64_t)1 << 53) + 1,
                                                     ((int64_t)1 << 53) - 1})
      if (q >= 0 && q <= qmax) check(q, d);
  for (long k = 0; k < rounds; ++k) {
    const int64_t d = 1 + (int64_t)(g() % (uint64_t)dmax);
    check((int64_t)(g() & (uint64_t)qmax) >> (g() % 63), d);  // dividends of every magnitude
    const int64_t a = (int64_t)(g() % (uint64_t)d), b = (int64_t)(g() % (uint64_t)d);
    check(a * b, d);  // products of two residues, as the kernel reduces them
  }
  std::printf("checks %ld bad %ld\n", n, bad);
  return bad != 0;
}
