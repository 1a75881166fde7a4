// Host-side accuracy check of the FP64 exponential and sine/cosine that the evaluation kernels use
// for their terms (hom_device.h: exp_eval, sincos_turns; both are __host__ __device__).  Compiled
// for the host only and run by tests/test_device_math_host.py.
//
// References: long double (64-bit significand) expl, sinl, cosl.  For sin and cos of 2 pi t the
// reference first removes the nearest quarter turn, t = q/4 + f (exact in binary arithmetic), and
// evaluates sinl / cosl of 2 pi f, rotated by q quarter turns; near the zeros of sin(2 pi t) a
// direct sinl(2 pi t) would carry an absolute error far above one ulp of the result.
//
// Output: one line "exp_max_ulp <v> exp_subnormal_max_abs <v> sin_max_ulp <v> cos_max_ulp <v>
// special_ok <0|1>".
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>

#include "hom_device.h"

static double ulp_err(double got, long double ref) {
  if (ref == 0.0L) return got == 0.0 ? 0.0 : INFINITY;
  const double r = (double)ref;
  const int e = std::ilogb(r);
  const long double ulp = std::ldexp(1.0L, (e < DBL_MIN_EXP - 1 ? DBL_MIN_EXP - 1 : e) - 52);
  return (double)(std::fabs((long double)got - ref) / ulp);
}

int main(int argc, char **argv) {
  const long count = argc > 1 ? std::atol(argv[1]) : 4000000;
  std::mt19937_64 gen(20211129);
  const long double two_pi = 6.283185307179586476925286766559005768L;

  double exp_max = 0.0, sub_abs = 0.0;
  std::uniform_real_distribution<double> dx(-708.0, 300.0), dsub(-745.0, -708.0);
  for (long i = 0; i < count; ++i) {
    const double x = i % 8 == 0 ? dx(gen) * 1e-3 : dx(gen);  // also dense near 0
    const double u = ulp_err(hom::exp_eval(x), ::expl((long double)x));
    if (u > exp_max) exp_max = u;
  }
  for (long i = 0; i < count / 16; ++i) {  // subnormal results: absolute error
    const double x = dsub(gen);
    const long double d = std::fabs((long double)hom::exp_eval(x) - ::expl((long double)x));
    if ((double)d > sub_abs) sub_abs = (double)d;
  }

  double sin_max = 0.0, cos_max = 0.0;
  std::uniform_real_distribution<double> dt(-0.5, 0.5);
  for (long i = 0; i < count; ++i) {
    double t = dt(gen);
    if (i % 4 == 1) t = std::ldexp(t, -(int)(i % 40));  // tiny phases
    if (i % 4 == 2) {                                     // next to quarter turns
      const double q = std::rint(4.0 * t) / 4.0;
      t = q + std::ldexp(dt(gen), -(int)(i % 45));
      if (t > 0.5 || t < -0.5) t = q;
    }
    double s, c;
    hom::sincos_turns(t, s, c);
    const long double q = std::rint(4.0L * t);
    const long double f = (long double)t - q / 4.0L;  // exact
    const long double sf = ::sinl(two_pi * f), cf = ::cosl(two_pi * f);
    const int qi = ((int)q % 4 + 4) % 4;
    long double rs, rc;
    switch (qi) {
      case 0: rs = sf; rc = cf; break;
      case 1: rs = cf; rc = -sf; break;
      case 2: rs = -sf; rc = -cf; break;
      default: rs = -cf; rc = sf; break;
    }
    const double us = ulp_err(s, rs), uc = ulp_err(c, rc);
    if (us > sin_max) sin_max = us;
    if (uc > cos_max) cos_max = uc;
  }

  // special arguments: exact quarter turns, e^0, NaN in -> NaN out, deep underflow -> 0
  double s0, c0, s1, c1, s2, c2;
  hom::sincos_turns(0.0, s0, c0);
  hom::sincos_turns(0.25, s1, c1);
  hom::sincos_turns(-0.5, s2, c2);
  double sn, cn;
  hom::sincos_turns(NAN, sn, cn);
  const bool special = s0 == 0.0 && c0 == 1.0 && s1 == 1.0 && c1 == 0.0 && s2 == 0.0 &&
                       c2 == -1.0 && hom::exp_eval(0.0) == 1.0 && std::isnan(hom::exp_eval(NAN)) &&
                       std::isnan(sn) && std::isnan(cn) && hom::exp_eval(-800.0) == 0.0;
  std::printf("exp_max_ulp %.4f exp_subnormal_max_abs %.3e sin_max_ulp %.4f cos_max_ulp %.4f "
              "special_ok %d\n",
              exp_max, sub_abs, sin_max, cos_max, special ? 1 : 0);
  return 0;
}
