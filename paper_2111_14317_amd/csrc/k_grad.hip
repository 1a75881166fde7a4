// Adjoint endpoint gradient (A9).
//
// For a real loss L on endpoints x* (t = 1), with upstream g = dL/dRe x + i dL/dIm x, the
// implicit function theorem (the argument behind the Davidenko equation, Sec. 2.3) gives
//   dL = Re(nu^H dF/dc dc),   J_x^H nu = -g,
// and, since J_x = J_z diag(e^{-z}), J_z^H nu = -conj(x) .* g.  The rows of the evaluated
// Jacobian carry the scale e^{-M_k}, so the kernel solves Js^H mu = -conj(x) .* g with
// Js = diag(e^{-M}) J_z and nu = e^{-M} mu.  The coefficient gradient is
//   grad c_{k,a} = sum_p nu_{p,k} conj(x_p^a) = sum_p mu_{p,k} conj(e^{<a, z_p> - M_{p,k}}).
// Per path: one evaluation (lane k owns equation k), a transpose of J_z through LDS so that lane
// j owns row j of Js^H, the same group LU as the tracker, then lane k writes the contributions
// of its monomials.  Paths are summed per monomial in a fixed order by two reduction kernels,
// so the result is bitwise reproducible.
#include <stdio.h>

#include "hom_internal.h"

namespace hom {

// mu = -(Js^H)^{-1} b for one path, in precision T: evaluate J_z at t = 1 (lane r: row r),
// transpose it through the group's LDS tile so that lane j holds row j of Js^H, then the group LU.
// Returns the singular flag; ratio is the pivot ratio, Mr the row shift.  Every lane of the wave
// must call it (it shuffles).
template <int N, typename T>
__device__ __forceinline__ bool adjoint_solve(const SysLds<N> &S, const Geo<N> &geo, int n,
                                              const double (&zr)[N], const double (&zi)[N],
                                              Cx<double> b, Cx<T> *tile, Cx<double> &mu,
                                              double &ratio, double &Mr) {
  const int r = geo.r;
  Cx<T> row[N + 2];
  T absum;
  eval_row_exact<N, T>(S, r, zr, zi, 0.0, row, Mr, absum);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // earlier reads of the tile are done
  __builtin_amdgcn_wave_barrier();
  if (geo.valid) {
#pragma unroll
    for (int j = 0; j < N; ++j) tile[r * N + j] = row[j];
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  Cx<T> rh[N + 2];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const Cx<T> v = geo.valid ? tile[j * N + r] : Cx<T>{T(j == r), T(0)};
    rh[j] = {v.x, -v.y};
  }
  rh[N] = {(T)b.x, (T)b.y};
  rh[N + 1] = {T(0), T(0)};
  Cx<T> m, unused;
  double nE, nN;
  T rt;
  bool sing = lu_solve2<N, T>(rh, r, geo.base, n, m, unused, nE, nN, rt);
  sing |= !(nE <= INFINITY);
  mu = {(double)m.x, (double)m.y};
  ratio = (double)rt;
  return sing;
}

// The mixed form solves in FP32 and redoes in FP64 the paths whose FP32 pivot ratio is below
// this (or that are singular in FP32), as the mixed step does: near a singular endpoint the FP32
// solve would carry an error of about kappa * 6e-8 into the gradient.
constexpr double kGradRedoRatio = 1e-4;
// A path whose (final) pivot ratio is below this is singular and contributes nothing, as in
// hom_step.
constexpr double kGradSingRatio = 1e-14;

template <int N, bool MIXED, bool GT>
__global__ void __launch_bounds__(64) k_grad_paths(SysDev sd, const double *__restrict__ c,
                                                   int64_t P0, int64_t Pc,
                                                   const double *__restrict__ z,
                                                   const double *__restrict__ gx,
                                                   double *__restrict__ work, size_t table_bytes,
                                                   double sing_ratio) {
  constexpr int LD = TableLD<N>::value;
  extern __shared__ __align__(16) char smem[];
  const SysLds<N> S = stage_tables<N, GT>(smem, sd, c);
  const Geo<N> geo;
  const int n = sd.n, r = geo.r, M = sd.M;
  // the group's transpose tile, sized for FP64 (the mixed form's redo uses it too)
  char *tile_b = smem + table_bytes + (size_t)(geo.valid ? geo.g : 0) * N * N * sizeof(Cx<double>);
  const int64_t p_loc = (int64_t)blockIdx.x * Geo<N>::G + geo.g;
  const bool act = geo.valid && p_loc < Pc;
  const int64_t p = P0 + (act ? p_loc : 0);
  double zr[N], zi[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    zr[j] = j < n ? z[2 * (p * n + j)] : 0.0;
    zi[j] = j < n ? z[2 * (p * n + j) + 1] : 0.0;
  }
  // right-hand side conj(x_r) g_r (zero on padding unknowns)
  Cx<double> b = {0.0, 0.0};
  if (act && r < n) {
    const double mag = exp(z[2 * (p * n + r)]);
    double sn, cs;
    sincos(-z[2 * (p * n + r) + 1], &sn, &cs);
    const Cx<double> xc = {mag * cs, mag * sn};  // conj(x_r)
    const Cx<double> g = {gx[2 * (p * n + r)], gx[2 * (p * n + r) + 1]};
    b = cmul(xc, g);
  }
  Cx<double> mu;
  double ratio, Mr;
  bool sing;
  if constexpr (MIXED) {
    sing = adjoint_solve<N, float>(S, geo, n, zr, zi, b, reinterpret_cast<Cx<float> *>(tile_b), mu,
                                   ratio, Mr);
    const bool redo = sing || !(ratio >= kGradRedoRatio);  // uniform within a group
    if (__any(redo)) {  // the whole wave runs the FP64 solve; only the flagged groups keep it
      Cx<double> mu64;
      double ratio64, Mr64;
      const bool sing64 = adjoint_solve<N, double>(S, geo, n, zr, zi, b,
                                                   reinterpret_cast<Cx<double> *>(tile_b), mu64,
                                                   ratio64, Mr64);
      if (redo) {
        mu = mu64;
        ratio = ratio64;
        Mr = Mr64;
        sing = sing64;
      }
    }
  } else {
    sing = adjoint_solve<N, double>(S, geo, n, zr, zi, b, reinterpret_cast<Cx<double> *>(tile_b), mu,
                                    ratio, Mr);
  }
  // mu = -(Js^H)^{-1} b.  Contributions of equation r's monomials.
  if (!act || r >= n) return;
  const bool ok = !sing && ratio >= sing_ratio;
  const int mr = S.mk[r];
  double *out = work + 2 * (p_loc * (int64_t)M);
  for (int i = 0; i < mr; ++i) {
    const double *t = S.T + (i * n + r) * LD;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      re = fma(t[j], zr[j], re);
      im = fma(t[j], zi[j], im);
    }
    double turns = im * kInv2Pi;
    turns -= rint(turns);
    Cx<double> E;  // conj(e^{u - M})
    if constexpr (MIXED) {
      const float mag = __builtin_amdgcn_exp2f((float)((re - Mr) * kLog2e));
      const float tf = (float)turns;
      E = {(double)(mag * __builtin_amdgcn_cosf(tf)), -(double)(mag * __builtin_amdgcn_sinf(tf))};
    } else {
      const double mag = exp_eval(re - Mr);
      double sn, cs;
      sincos_turns(turns, sn, cs);
      E = {mag * cs, -mag * sn};
    }
    Cx<double> v = ok ? cmul(mu, E) : Cx<double>{0.0, 0.0};
    const int q = sd.off[r] + i;
    out[2 * q] = v.x;
    out[2 * q + 1] = v.y;
  }
}

// part[t][q] = sum over rows p = t, t + T, t + 2T, ... of work[p][q] (fixed order)
__global__ void k_grad_red1(const double *__restrict__ work, int64_t Pc, int M, int T,
                            double *__restrict__ part) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (q >= M) return;
  double ax = 0.0, ay = 0.0;
  for (int64_t p = t; p < Pc; p += T) {
    ax += work[2 * (p * M + q)];
    ay += work[2 * (p * M + q) + 1];
  }
  part[2 * ((int64_t)t * M + q)] = ax;
  part[2 * ((int64_t)t * M + q) + 1] = ay;
}

// grad[q] (+)= sum_t part[t][q] in order
__global__ void k_grad_red2(const double *__restrict__ part, int M, int T, int accumulate,
                            double *__restrict__ grad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= M) return;
  double ax = accumulate ? grad[2 * q] : 0.0, ay = accumulate ? grad[2 * q + 1] : 0.0;
  double sx = 0.0, sy = 0.0;
  for (int t = 0; t < T; ++t) {
    sx += part[2 * ((int64_t)t * M + q)];
    sy += part[2 * ((int64_t)t * M + q) + 1];
  }
  grad[2 * q] = ax + sx;
  grad[2 * q + 1] = ay + sy;
}

constexpr int kRedT = 256;

size_t grad_work_elems(const System &S, int64_t P) {
  // chunk of paths whose per-path contributions fit in 256 MB, plus the partial sums
  int64_t Pc = (int64_t)((256ull << 20) / (16ull * (uint64_t)S.M));
  if (Pc < 1) Pc = 1;
  if (Pc > P) Pc = P > 0 ? P : 1;
  return (size_t)(2 * Pc * (int64_t)S.M + 2 * (int64_t)kRedT * S.M);
}

template <int N>
static hipError_t grad_n(const System &S, const void *cws, const double *c, int64_t P,
                         const double *z,
                         const double *gx, double *grad, int precision, double *work,
                         size_t work_elems, hipStream_t stream) {
  const size_t tb = (S.lds_bytes + 15) & ~(size_t)15;
  const size_t tile = (size_t)Geo<N>::G * N * N * sizeof(Cx<double>);
  const int64_t part_elems = 2 * (int64_t)kRedT * S.M;
  int64_t Pc = ((int64_t)work_elems - part_elems) / (2 * (int64_t)S.M);
  if (Pc < 1) return hipErrorInvalidValue;
  double *part = work + (work_elems - part_elems);
  if (P == 0) {
    hipLaunchKernelGGL(k_grad_red2, dim3((S.M + 255) / 256), dim3(256), 0, stream, part, S.M, 0,
                       0, grad);
    return hipGetLastError();
  }
  for (int64_t P0 = 0; P0 < P; P0 += Pc) {
    const int64_t pc = (P - P0) < Pc ? (P - P0) : Pc;
    const unsigned blocks = (unsigned)((pc + Geo<N>::G - 1) / Geo<N>::G);
    char label[64];
    snprintf(label, sizeof label, "k_grad_paths<%d,%s>", N, precision == 1 ? "mixed" : "fp64");
    prof_begin(stream);
    auto kern = precision == 1
                    ? (S.global_tables ? k_grad_paths<N, true, true> : k_grad_paths<N, true, false>)
                    : (S.global_tables ? k_grad_paths<N, false, true> : k_grad_paths<N, false, false>);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64), tb + tile, stream, S.dev(cws), c, P0, pc, z,
                       gx, work, tb, kGradSingRatio);
    prof_end(stream, label);
    hipLaunchKernelGGL(k_grad_red1, dim3((S.M + 255) / 256, kRedT), dim3(256), 0, stream, work,
                       pc, S.M, kRedT, part);
    hipLaunchKernelGGL(k_grad_red2, dim3((S.M + 255) / 256), dim3(256), 0, stream, part, S.M,
                       kRedT, P0 > 0 ? 1 : 0, grad);
  }
  return hipGetLastError();
}

#define HOM_SWITCH_G(N, CALL)            \
  switch (N) {                         \
    case 2: { constexpr int NN = 2; CALL; } \
    case 3: { constexpr int NN = 3; CALL; } \
    case 4: { constexpr int NN = 4; CALL; } \
    case 5: { constexpr int NN = 5; CALL; } \
    case 6: { constexpr int NN = 6; CALL; } \
    case 7: { constexpr int NN = 7; CALL; } \
    case 8: { constexpr int NN = 8; CALL; } \
    case 10: { constexpr int NN = 10; CALL; } \
    case 12: { constexpr int NN = 12; CALL; } \
    case 16: { constexpr int NN = 16; CALL; } \
    case 20: { constexpr int NN = 20; CALL; } \
    case 24: { constexpr int NN = 24; CALL; } \
    case 32: { constexpr int NN = 32; CALL; } \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_grad(const System &S, const void *cws, const double *c, int64_t P,
                       const double *z_end,
                       const double *grad_x, double *grad_c, int precision, double *work,
                       size_t work_elems, hipStream_t stream) {
  HOM_SWITCH_G(S.N, return grad_n<NN>(S, cws, c, P, z_end, grad_x, grad_c, precision, work,
                                      work_elems, stream))
}

}  // namespace hom
