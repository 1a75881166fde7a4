// Internal declarations shared by the C ABI and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "hom_device.h"

namespace hom {

// Compiled group sizes; a system with n unknowns runs on the smallest N >= n.
constexpr int kSizes[] = {2, 3, 4, 5, 6, 7, 8, 10, 12, 16, 20, 24, 32};
int bucket_for(int n);   // smallest compiled N >= n, or 0
int table_ld(int N);     // TableLD<N>::value at run time

struct System {
  int n = 0, N = 0, mmax = 0, M = 0;
  int device = 0;
  double *dT = nullptr;     // device [mmax][n][LD] exponent table + lifting
  int32_t *dmk = nullptr;   // device [n]
  int32_t *doff = nullptr;  // device [n]
  int32_t *dA = nullptr;    // device [M][n] exponents as int32 (adjoint kernel)
  size_t lds_bytes = 0;     // LDS image of the tables
  SysDev dev() const { return SysDev{n, mmax, M, dT, dmk, doff}; }
};

// Tracker constants as the kernels see them.
struct TrackDev {
  double ds0, ds_max, ds_min, tol_polish, tol_track, tol_end, res_tol, div_re, sing_ratio;
  int max_polish, max_newton, max_end, max_steps, max_iters;
  int exact_shift;
};

// internal path statuses between the mixed pass and the FP64 pass of one hom_track call:
// reached s = 0 in the mixed form, FP64 endgame still to run
constexpr int kPendingEnd = 3;
// the mixed form failed after an accepted point: (z, s) is that point, continue in FP64
constexpr int kHandoff = 4;

void set_error(const std::string &msg);

// Kernel timing: when profiling is on for this thread, prof_begin/prof_end record a pair of
// events around a launch (no-ops otherwise).
// prof_units returns a zeroed device counter for the launch's work units (nullptr when off).
void prof_begin(hipStream_t stream);
unsigned long long *prof_units(hipStream_t stream);
void prof_end(hipStream_t stream, const char *label);

// launchers (return a hipError_t)
hipError_t launch_eval(const System &S, const double *c, int64_t P, const double *z,
                       const double *s, double *G, double *logscale, int flags,
                       hipStream_t stream);
hipError_t launch_step(const System &S, const double *c, int64_t P, const double *z,
                       const double *s, double *dE, double *dN, int32_t *status, int precision,
                       hipStream_t stream);
hipError_t launch_track(const System &S, const double *c, int64_t P, double *z, double *s,
                        double *ds, int32_t *status, int32_t *counters, const TrackDev &pr,
                        bool mixed, unsigned long long *queue, hipStream_t stream);
hipError_t launch_grad(const System &S, const double *c, int64_t P, const double *z_end,
                       const double *grad_x, double *grad_c, int precision, double *work,
                       size_t work_elems, hipStream_t stream);
size_t grad_work_elems(const System &S, int64_t P);

// number of compute units of the current device (cached)
int num_cus();

}  // namespace hom
