// Batched evaluation (A1-A4) and evaluation + consolidated Euler/Newton solve (A1-A5).
//
// hom_eval : G = [J_z | H_s | H] per point, rows scaled by e^{-M_k} (Sec. 5.1-5.2; Alg. 2).
// hom_step : the same evaluation kept in registers, then one LU with partial pivoting of J_z
//            applied to both right-hand sides (Sec. 6 in its affine form; Alg. 3).
// One group of N lanes per point, grid-stride over points; tables staged once per block.
#include <stdio.h>

#include "hom_internal.h"

namespace hom {

constexpr int kBlock = 256;

template <int N>
__device__ __forceinline__ void load_point(const double *__restrict__ z, int64_t p, int n,
                                           double (&zr)[N], double (&zi)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if (j < n) {
      zr[j] = z[2 * (p * n + j)];
      zi[j] = z[2 * (p * n + j) + 1];
    } else {
      zr[j] = 0.0;
      zi[j] = 0.0;
    }
  }
}

// Per-wave LDS of k_eval: the wave's points (one complex per lane: lane r of group g holds z_r of
// the group's point) and a staging buffer through which the rows leave in contiguous 1 KiB
// stores.  A wave's output rows are consecutive in G ([P][n][n+2]), so the buffer takes them
// in chunks of whole rows and the wave writes each chunk with 16 bytes per lane.
constexpr int kEvalStageBytes = 4096;
constexpr int kEvalWaveBytes = 64 * 16 + kEvalStageBytes;

// FP32 up to 12 lanes per group: three waves per SIMD (at most 168 registers); the others need
// more and run two.
template <int N, typename T, bool GT>
__global__ void __launch_bounds__(kBlock)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && N <= 12 ? 3 : 1)))
    k_eval(SysDev sd, const double *__restrict__ c,
                                                 int64_t P, const double *__restrict__ z,
                                                 const double *__restrict__ s,
                                                 double *__restrict__ G,
                                                 double *__restrict__ logscale, int flags,
                                                 size_t table_bytes) {
  extern __shared__ __align__(16) char smem[];
  const SysLds<N> S = stage_tables<N, GT>(smem, sd, c);
  const Geo<N> geo;
  const int n = sd.n, r = geo.r, lane = geo.lane;
  char *wbuf = smem + table_bytes + (threadIdx.x >> 6) * kEvalWaveBytes;
  Cx<double> *sZ = reinterpret_cast<Cx<double> *>(wbuf);
  char *stage = wbuf + 64 * 16;
  const int64_t gpb = (kBlock / 64) * Geo<N>::G;
  const int64_t stride = (int64_t)gridDim.x * gpb;
  const int row_bytes = (n + 2) * 16;
  const int rows_per_chunk = kEvalStageBytes / row_bytes;
  // this lane's coordinate of its group's next point, loaded one iteration ahead
  auto fetch = [&](int64_t q, Cx<double> &zq, double &sq) {
    const bool ok = geo.valid && q < P;
    zq = (ok && r < n) ? reinterpret_cast<const Cx<double> *>(z)[q * n + r] : Cx<double>{0.0, 0.0};
    sq = ok ? s[q] : 0.0;
  };
  const int64_t wave0 = (int64_t)blockIdx.x * gpb + (threadIdx.x >> 6) * Geo<N>::G;
  Cx<double> zmine;
  double smine;
  fetch(wave0 + geo.g, zmine, smine);
  for (int64_t base = wave0; base < P; base += stride) {  // wave-uniform
    const int64_t p = base + geo.g;
    const bool act = geo.valid && p < P;
    if (geo.valid) sZ[lane] = zmine;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    double zr[N], zi[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const Cx<double> v = geo.valid ? sZ[geo.base + j] : Cx<double>{0.0, 0.0};
      zr[j] = j < n ? v.x : 0.0;
      zi[j] = j < n ? v.y : 0.0;
    }
    const double sp = smine;
    fetch(p + stride, zmine, smine);
    Cx<T> row[N + 2];
    double M;
    T absum;
    eval_row_exact<N, T>(S, r, zr, zi, sp, row, M, absum);
    const double scale = (flags & 1) ? exp_eval(M) : 1.0;  // HOM_UNSCALED
    const double fs = (flags & 2) ? scale * exp_eval(-sp) : scale;  // HOM_AFFINE: H_t = e^{-s} H_s
    // rows of this wave's block in chunks through the staging buffer
    const int64_t left = P - base;
    const int groups = left < Geo<N>::G ? (int)left : Geo<N>::G;
    const int rows = groups * n;
    const int q = geo.g * n + r;  // this lane's row within the block
    const bool owner = act && r < n;
    double *Gw = G + 2 * (base * n) * (n + 2);
    for (int c0 = 0; c0 < rows; c0 += rows_per_chunk) {
      if (owner && q >= c0 && q < c0 + rows_per_chunk) {
        Cx<double> *dst = reinterpret_cast<Cx<double> *>(stage + (q - c0) * row_bytes);
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j < n) dst[j] = Cx<double>{(double)row[j].x * scale, (double)row[j].y * scale};
        dst[n] = Cx<double>{(double)row[N].x * fs, (double)row[N].y * fs};
        dst[n + 1] = Cx<double>{(double)row[N + 1].x * scale, (double)row[N + 1].y * scale};
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      const int nrow = rows - c0 < rows_per_chunk ? rows - c0 : rows_per_chunk;
      const int pieces = nrow * (n + 2);  // 16-byte pieces of this chunk
      const double2 *src = reinterpret_cast<const double2 *>(stage);
      double2 *out = reinterpret_cast<double2 *>(Gw + 2 * (int64_t)c0 * (n + 2));
      if (flags & 2) {  // HOM_AFFINE: J_x = J_z diag(e^{-z}), on the way out
        for (int k = lane; k < pieces; k += 64) {
          const int rq = c0 + k / (n + 2), j = k - (k / (n + 2)) * (n + 2);
          double2 v = src[k];
          if (j < n) {
            const Cx<double> zj = sZ[(rq / n) * N + j];
            double t = -zj.y * kInv2Pi;  // the phase in turns, reduced to [-1/2, 1/2]
            t -= rint(t);
            double sn, cs;
            sincos_turns(t, sn, cs);
            const double mag = exp_eval(-zj.x);
            const Cx<double> w = cmul(Cx<double>{v.x, v.y}, Cx<double>{mag * cs, mag * sn});
            v.x = w.x;
            v.y = w.y;
          }
          out[k] = v;
        }
      } else {
        for (int k = lane; k < pieces; k += 64) out[k] = src[k];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();  // the buffer is read before the next chunk overwrites it
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    if (logscale && owner) logscale[p * n + r] = (flags & 1) ? 0.0 : M;
  }
}

// Evaluation + consolidated solve.  The loop over points is wave-uniform (the LU shuffles);
// groups past the end compute on a dummy point and store nothing.
// The mixed form up to 12 lanes per group: three waves per SIMD (some registers spill; 2-5%
// faster at 1M points than two waves without spills).  The FP64 form measured the same at three.
template <int N, bool MIXED, bool GT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(MIXED && N <= 12 ? 3 : 1)))
    k_step(SysDev sd, const double *__restrict__ c,
                                                 int64_t P, const double *__restrict__ z,
                                                 const double *__restrict__ s,
                                                 double *__restrict__ dE,
                                                 double *__restrict__ dN,
                                                 int32_t *__restrict__ status) {
  extern __shared__ __align__(16) char smem[];
  const SysLds<N> S = stage_tables<N, GT>(smem, sd, c);
  const Geo<N> geo;
  const int n = sd.n, r = geo.r;
  const int64_t gpb = (kBlock / 64) * Geo<N>::G;
  const int64_t stride = (int64_t)gridDim.x * gpb;
  const int64_t p0 = (int64_t)blockIdx.x * gpb + (threadIdx.x >> 6) * Geo<N>::G + geo.g;
  for (int64_t it = 0;; ++it) {
    const int64_t p = p0 + it * stride;
    const bool act = geo.valid && p < P;
    if (!__any(act)) break;
    double zr[N], zi[N];
    load_point<N>(z, act ? p : 0, act ? n : 0, zr, zi);
    const double sp = act ? s[p] : 0.0;
    double M, nE, nN;
    Cx<double> e, q;
    bool sing;
    double ratio;
    if constexpr (MIXED) {
      Cx<float> row[N + 2], ef, qf;
      float absum, rf;
      eval_row_exact<N, float>(S, r, zr, zi, sp, row, M, absum);
      sing = lu_solve2<N, float>(row, r, geo.base, n, ef, qf, nE, nN, rf);
      e = {ef.x, ef.y};
      q = {qf.x, qf.y};
      ratio = rf;
      // near-singular in FP32: redo this point's evaluation and LU in FP64
      const bool redo = act && (sing || !(rf >= 1e-4f));
      if (__any(redo)) {
        Cx<double> rowd[N + 2], ed, qd;
        double ad, rd, nEd, nNd;
        eval_row_exact<N, double>(S, r, zr, zi, sp, rowd, M, ad);
        const bool sd2 = lu_solve2<N, double>(rowd, r, geo.base, n, ed, qd, nEd, nNd, rd);
        if (redo) {
          e = ed;
          q = qd;
          sing = sd2;
          ratio = rd;
        }
      }
    } else {
      Cx<double> row[N + 2];
      double absum;
      eval_row_exact<N, double>(S, r, zr, zi, sp, row, M, absum);
      sing = lu_solve2<N, double>(row, r, geo.base, n, e, q, nE, nN, ratio);
    }
    if (act) {
      if (r < n) {
        dE[2 * (p * n + r)] = e.x;
        dE[2 * (p * n + r) + 1] = e.y;
        dN[2 * (p * n + r)] = q.x;
        dN[2 * (p * n + r) + 1] = q.y;
      }
      if (r == 0) status[p] = (sing || !(ratio >= 1e-14)) ? -1 : 0;
    }
  }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
static int grid_for(int64_t P, int groups_per_block) {
  const int64_t need = (P + groups_per_block - 1) / groups_per_block;
  const int64_t cap = (int64_t)num_cus() * 8;
  return (int)(need < cap ? (need > 0 ? need : 1) : cap);
}

#define HOM_SWITCH(N, CALL)            \
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

// Table-order coefficients and their moduli [mmax][n] for a system whose tables stay in global
// memory (the same arrays stage_tables builds in LDS otherwise).
__global__ void k_coeff_tables(SysDev sd, const double *__restrict__ c, Cx<double> *__restrict__ C,
                               double *__restrict__ Cabs) {
  const int total = sd.mmax * sd.n;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const int i = idx / sd.n, r = idx - i * sd.n;
    Cx<double> v = {0.0, 0.0};
    if (i < sd.mk[r]) {
      const int q = sd.off[r] + i;
      v.x = c[2 * q];
      v.y = c[2 * q + 1];
    }
    C[idx] = v;
    Cabs[idx] = sqrt(v.x * v.x + v.y * v.y);
  }
}

hipError_t launch_coeff_tables(const System &S, const double *c, void *cws, hipStream_t stream) {
  const SysDev sd = S.dev(cws);
  const int total = S.mmax * S.n;
  hipLaunchKernelGGL(k_coeff_tables, dim3((total + 255) / 256), dim3(256), 0, stream, sd, c,
                     const_cast<Cx<double> *>(sd.Cg), const_cast<double *>(sd.Cabs_g));
  return hipGetLastError();
}

template <int N>
static hipError_t eval_n(const System &S, const void *cws, const double *c, int64_t P,
                         const double *z, const double *s, double *G, double *logscale, int flags,
                         hipStream_t stream) {
  const int gpb = (kBlock / 64) * Geo<N>::G;
  char label[64];
  snprintf(label, sizeof label, "k_eval<%d,%s>", N, (flags & 4) ? "fp32" : "fp64");
  prof_begin(stream);
  auto kern = (flags & 4) ? (S.global_tables ? k_eval<N, float, true> : k_eval<N, float, false>)
                          : (S.global_tables ? k_eval<N, double, true> : k_eval<N, double, false>);
  const size_t tb = (S.lds_bytes + 15) & ~(size_t)15;
  const size_t lds = tb + (kBlock / 64) * kEvalWaveBytes;
  hipLaunchKernelGGL(kern, dim3(grid_for(P, gpb)), dim3(kBlock), lds, stream, S.dev(cws), c, P, z,
                     s, G, logscale, flags, tb);
  prof_end(stream, label);
  return hipGetLastError();
}

template <int N>
static hipError_t step_n(const System &S, const void *cws, const double *c, int64_t P,
                         const double *z, const double *s, double *dE, double *dN,
                         int32_t *status, int precision, hipStream_t stream) {
  const int gpb = (kBlock / 64) * Geo<N>::G;
  char label[64];
  snprintf(label, sizeof label, "k_step<%d,%s>", N, precision == 1 ? "mixed" : "fp64");
  prof_begin(stream);
  auto kern = precision == 1 ? (S.global_tables ? k_step<N, true, true> : k_step<N, true, false>)
                             : (S.global_tables ? k_step<N, false, true> : k_step<N, false, false>);
  hipLaunchKernelGGL(kern, dim3(grid_for(P, gpb)), dim3(kBlock), S.lds_bytes, stream, S.dev(cws), c,
                     P, z, s, dE, dN, status);
  prof_end(stream, label);
  return hipGetLastError();
}

hipError_t launch_eval(const System &S, const void *cws, const double *c, int64_t P,
                       const double *z, const double *s, double *G, double *logscale, int flags,
                       hipStream_t stream) {
  HOM_SWITCH(S.N, return eval_n<NN>(S, cws, c, P, z, s, G, logscale, flags, stream))
}

hipError_t launch_step(const System &S, const void *cws, const double *c, int64_t P,
                       const double *z, const double *s, double *dE, double *dN,
                       int32_t *status, int precision, hipStream_t stream) {
  HOM_SWITCH(S.N, return step_n<NN>(S, cws, c, P, z, s, dE, dN, status, precision, stream))
}

}  // namespace hom
