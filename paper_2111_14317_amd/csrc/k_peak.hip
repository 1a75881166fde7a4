// Peak probes: the rates of the units the kernels are bound by, measured on the device they run
// on (the denominators of the rooflines, beside the published figures).  Each probe is one
// bounded kernel timed with hipEvents over a few launches after a warm-up; every result is
// written out so that the compiler keeps the work.
//   HBM read / write : a 4 GiB buffer streamed with 32-byte accesses per lane
//   FP64 / FP32 FMA  : 8 independent FMA chains per lane
//   FP32 exp2        : 8 independent chains of v_exp_f32
//   MFMA             : 4 independent accumulators of 16x16x4 f64 / 16x16x32 bf16
//   exp_eval, sincos_turns : the library's FP64 exponential and sine/cosine of the terms
#include <hip/hip_runtime.h>

#include "hom_internal.h"

namespace hom {

namespace {

typedef __bf16 pk_bf16x8_t __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float pk_f32x4_t __attribute__((__vector_size__(4 * sizeof(float))));
typedef double pk_f64x4_t __attribute__((__vector_size__(4 * sizeof(double))));

constexpr int kPeakBlock = 256;

__global__ void __launch_bounds__(kPeakBlock)
    k_peak_read(const double4 *__restrict__ p, int64_t n, double *__restrict__ out) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double4 v = p[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  if (acc == -1.0) out[blockIdx.x] = acc;  // never true for the buffer written below
}

__global__ void __launch_bounds__(kPeakBlock)
    k_peak_write(double4 *__restrict__ p, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = double4{v, v, v, v};
}

template <typename T>
__global__ void __launch_bounds__(kPeakBlock)
    k_peak_fma(T *__restrict__ out, int iters, T a, T b) {
  T x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = (T)(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = fma(x[k], a, b);
  }
  T s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kPeakBlock)
    k_peak_exp2f(float *__restrict__ out, int iters, float c) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = -0.001f * (float)(threadIdx.x + k);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_exp2f(x[k]) * c;  // stays in (-1, 0)
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kPeakBlock)
    k_peak_mfma_f64(double *__restrict__ out, int iters, double a) {
  pk_f64x4_t acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = pk_f64x4_t{0.0, 0.0, 0.0, 0.0};
  const double b = a * (double)(threadIdx.x & 63);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kPeakBlock)
    k_peak_mfma_bf16(float *__restrict__ out, int iters, float a) {
  pk_f32x4_t acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = pk_f32x4_t{0.f, 0.f, 0.f, 0.f};
  pk_bf16x8_t va, vb;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    va[e] = (__bf16)(a * (float)e);
    vb[e] = (__bf16)(a * (float)(threadIdx.x & 7));
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, acc[k], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// evaluations of the library's FP64 exp (SIN = false) or sin/cos pair (SIN = true) on
// independent arguments in the range the terms use
template <bool SIN>
__global__ void __launch_bounds__(kPeakBlock)
    k_peak_poly(double *__restrict__ out, int iters) {
  double acc = 0.0;
  const double x0 = -1e-3 * (double)(threadIdx.x & 255);
  for (int it = 0; it < iters; ++it) {
    const double x = x0 - 1e-4 * (double)it;
    if constexpr (SIN) {
      double sn, cs;
      sincos_turns(fma(0.37, x, 0.1), sn, cs);  // |t| <= 1/2
      acc += sn + cs;
    } else {
      acc += exp_eval(x);
    }
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// mean duration (ms) of `reps` launches after one warm-up launch
template <class F>
hipError_t time_launches(hipStream_t st, int reps, F launch, double *ms) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  launch();
  e = hipEventRecord(e0, st);
  for (int i = 0; i < reps && e == hipSuccess; ++i) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  *ms = (double)t / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return e;
}

}  // namespace

hipError_t peak_probe(int kind, double *rate, hipStream_t st) {
  const int blocks = num_cus() * 8;
  const int64_t threads = (int64_t)blocks * kPeakBlock;
  const int reps = 5;
  double ms = 0.0;
  hipError_t e = hipSuccess;
  if (kind == HOM_PEAK_HBM_READ || kind == HOM_PEAK_HBM_WRITE) {
    const int64_t bytes = (int64_t)4 << 30, n = bytes / 32;
    void *buf = nullptr, *out = nullptr;
    e = hipMalloc(&buf, bytes);
    if (e == hipSuccess) e = hipMalloc(&out, (size_t)blocks * 8);
    if (e == hipSuccess) {
      double4 *p = static_cast<double4 *>(buf);
      hipLaunchKernelGGL(k_peak_write, dim3(blocks), dim3(kPeakBlock), 0, st, p, n, 1.0);
      e = hipGetLastError();
      if (e == hipSuccess && kind == HOM_PEAK_HBM_READ)
        e = time_launches(st, reps, [&] {
          hipLaunchKernelGGL(k_peak_read, dim3(blocks), dim3(kPeakBlock), 0, st, p, n,
                             static_cast<double *>(out));
        }, &ms);
      else if (e == hipSuccess)
        e = time_launches(st, reps, [&] {
          hipLaunchKernelGGL(k_peak_write, dim3(blocks), dim3(kPeakBlock), 0, st, p, n, 2.0);
        }, &ms);
      if (e == hipSuccess) *rate = (double)bytes / (ms * 1e-3) / 1e9;  // GB/s
    }
    hipError_t e2 = hipStreamSynchronize(st);
    if (buf) (void)hipFree(buf);
    if (out) (void)hipFree(out);
    return e != hipSuccess ? e : e2;
  }
  void *out = nullptr;
  e = hipMalloc(&out, (size_t)threads * 8);
  if (e != hipSuccess) return e;
  const int iters = 4096;
  double work = 0.0, unit = 1e12;  // per launch: flops (TFLOP/s) or evaluations (G/s)
  switch (kind) {
    case HOM_PEAK_FP64_FMA:
      e = time_launches(st, reps, [&] {
        hipLaunchKernelGGL(k_peak_fma<double>, dim3(blocks), dim3(kPeakBlock), 0, st,
                           static_cast<double *>(out), iters, 0.999999, 1e-7);
      }, &ms);
      work = 2.0 * 8 * iters * (double)threads;
      break;
    case HOM_PEAK_FP32_FMA:
      e = time_launches(st, reps, [&] {
        hipLaunchKernelGGL(k_peak_fma<float>, dim3(blocks), dim3(kPeakBlock), 0, st,
                           static_cast<float *>(out), iters, 0.9999f, 1e-5f);
      }, &ms);
      work = 2.0 * 8 * iters * (double)threads;
      break;
    case HOM_PEAK_FP32_EXP2:
      e = time_launches(st, reps, [&] {
        hipLaunchKernelGGL(k_peak_exp2f, dim3(blocks), dim3(kPeakBlock), 0, st,
                           static_cast<float *>(out), iters / 4, -0.5f);
      }, &ms);
      work = 8.0 * (iters / 4) * (double)threads;
      unit = 1e9;
      break;
    case HOM_PEAK_MFMA_F64:
      e = time_launches(st, reps, [&] {
        hipLaunchKernelGGL(k_peak_mfma_f64, dim3(blocks), dim3(kPeakBlock), 0, st,
                           static_cast<double *>(out), iters / 16, 1e-3);
      }, &ms);
      work = 2.0 * 16 * 16 * 4 * 4 * (iters / 16) * (double)(threads / 64);
      break;
    case HOM_PEAK_MFMA_BF16:
      e = time_launches(st, reps, [&] {
        hipLaunchKernelGGL(k_peak_mfma_bf16, dim3(blocks), dim3(kPeakBlock), 0, st,
                           static_cast<float *>(out), iters / 4, 1e-3f);
      }, &ms);
      work = 2.0 * 16 * 16 * 32 * 4 * (iters / 4) * (double)(threads / 64);
      break;
    case HOM_PEAK_EXP_F64:
      e = time_launches(st, reps, [&] {
        hipLaunchKernelGGL(k_peak_poly<false>, dim3(blocks), dim3(kPeakBlock), 0, st,
                           static_cast<double *>(out), iters / 16);
      }, &ms);
      work = (double)(iters / 16) * (double)threads;
      unit = 1e9;
      break;
    case HOM_PEAK_SINCOS_F64:
      e = time_launches(st, reps, [&] {
        hipLaunchKernelGGL(k_peak_poly<true>, dim3(blocks), dim3(kPeakBlock), 0, st,
                           static_cast<double *>(out), iters / 16);
      }, &ms);
      work = (double)(iters / 16) * (double)threads;
      unit = 1e9;
      break;
    default:
      e = hipErrorInvalidValue;
  }
  if (e == hipSuccess) *rate = work / (ms * 1e-3) / unit;
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(out);
  return e != hipSuccess ? e : e2;
}

}  // namespace hom
