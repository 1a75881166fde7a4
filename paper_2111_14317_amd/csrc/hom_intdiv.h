// 64-bit quotients by small divisors without the compiler's 64-bit division routine (a long
// software sequence on the GPU): an FP64 estimate of the quotient, corrected twice in int64.
// __host__ __device__, so the host test (tests/intdiv_host.cpp) runs the same source.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace hom {

// q = t d + r with 0 <= r < d; returns t.  For 0 <= q < 2^62 and 1 <= d < 2^31, inv = 1/d
// rounded to double.  The FP64 estimate of q/d is within 1537 of it (q, 1/d and their product
// each carry a relative rounding error of at most 2^-53, and q/d < 2^62), so the remainder it
// leaves is below 2^42 in magnitude and exact in FP64; that remainder's quotient estimate is then
// within one, which the last step fixes.
__host__ __device__ __forceinline__ int64_t divmod62(int64_t q, int64_t d, double inv, int64_t &r) {
  int64_t t = (int64_t)((double)q * inv);
  int64_t e = q - t * d;
  const int64_t t2 = (int64_t)floor((double)e * inv);
  t += t2;
  e -= t2 * d;
  if (e < 0) {
    e += d;
    --t;
  } else if (e >= d) {
    e -= d;
    ++t;
  }
  r = e;
  return t;
}

}  // namespace hom
