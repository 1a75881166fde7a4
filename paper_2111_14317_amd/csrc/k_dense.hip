// Dense-support evaluation on the matrix cores (large m_k, e.g. n = 32 with 128 monomials per
// equation).  Per equation k and per tile of 16 points:
//
//   A1  u = [A_k | w_k] [z; s]          MFMA, rows = monomials, columns = points (Sec. 5.1, the
//                                       exponent product e^{Z A})
//   A2  V = c exp(u - M_k)              vector units, in the MFMA result layout
//   A3  [J_z | H_s | H]_k = V C_k       MFMA with V as the A operand straight from the A1 result
//                                       registers (Sec. 5.1, the per-equation product with B_k);
//                                       the w and 1 columns (H_s, H) are summed on the vector units
//
// Two engines:
//   FP64    16x16x4 f64 MFMA; phase in turns (z's imaginary parts divided by 2 pi and reduced
//           before the product), exponential and sine/cosine in FP64.
//   BF16x3  16x16x32 bf16 MFMA with FP32 accumulation.  Re z is split into three bf16 parts
//           (hi + mid + lo, one accumulator); Im z / 2 pi is written as three signed base-512
//           digits, each product summed in its own accumulator, so the phase is formed exactly
//           modulo one turn from integer sums.  exp2/sin/cos on the FP32 transcendental unit; V
//           (FP32) is split into three bf16 parts whose sum is exact for A3.
//
// The row shift M_k is the row maximum of the hi-part product plus w s (an approximation is
// enough: any shift gives the same directions, and the true maximum term stays within e^{0.1}).
#include <stdio.h>

#include <type_traits>

#include "hom_internal.h"

namespace hom {

typedef __bf16 bf16x8_t __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x4_t __attribute__((__vector_size__(4 * sizeof(float))));
typedef double f64x4_t __attribute__((__vector_size__(4 * sizeof(double))));

constexpr int kDenseBlock = 256;       // 4 waves; each owns one 16-point tile at a time
// points per evaluation + LU round of hom_step: 4096 tiles, enough blocks for every CU; the FP32
// rows of a round take 570 MB at n = 32
constexpr int64_t kDenseChunk = 65536;
constexpr int32_t kDenseRedo = 2;  // internal status between the FP32 LU and its FP64 pass

__device__ __forceinline__ bf16x8_t as_bf16x8(uint4 v) { return __builtin_bit_cast(bf16x8_t, v); }

__device__ __forceinline__ bf16x8_t pack8(const uint32_t (&w)[4]) {
  return __builtin_bit_cast(bf16x8_t, uint4{w[0], w[1], w[2], w[3]});
}

// two bf16-valued floats (low 16 bits zero) -> one packed register, a in the low half
__device__ __forceinline__ uint32_t pack2(float a, float b) {
  return (__float_as_uint(a) >> 16) | (__float_as_uint(b) & 0xffff0000u);
}

// round a float to its 8 most significant bits (nearest, ties to even; finite inputs)
__device__ __forceinline__ float bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// x ~ h + m + l, each exactly a bf16, residual below 2^-24 |x|
__device__ __forceinline__ void split3_rne(double x, float &h, float &m, float &l) {
  h = bf16_rne((float)x);
  const double r = x - (double)h;
  m = bf16_rne((float)r);
  l = bf16_rne((float)(r - (double)m));
}

// v = h + m + l exactly (24 significant bits in three 8-bit pieces, by truncation)
__device__ __forceinline__ void split3_exact(float v, float &h, float &m, float &l) {
  h = __uint_as_float(__float_as_uint(v) & 0xffff0000u);
  const float r = v - h;
  m = __uint_as_float(__float_as_uint(r) & 0xffff0000u);
  l = r - m;
}

// Im z / (2 pi), reduced to [-1/2, 1/2], as d1/512 + d2/512^2 + d3/512^3 with integer digits
// |d| <= 256 (exact bf16 values); the dropped remainder is below 2^-28 turns.
__device__ __forceinline__ void turn_digits(double im, float &d1, float &d2, float &d3) {
  double t = im * kInv2Pi;
  t -= rint(t);
  const double t1 = t * 512.0;
  const double r1 = rint(t1);
  const double t2 = (t1 - r1) * 512.0;
  const double r2 = rint(t2);
  const double r3 = rint((t2 - r2) * 512.0);
  d1 = (float)r1;
  d2 = (float)r2;
  d3 = (float)r3;
}

// Result layouts of the two 16x16 MFMA shapes: lane l holds column l % 16; its four result
// registers r hold rows 4 (l / 16) + r (f32, 16x16x32 bf16) and 4 r + l / 16 (f64, 16x16x4 f64).
__device__ __forceinline__ int row_f32(int q, int r) { return 4 * q + r; }
__device__ __forceinline__ int row_f64(int q, int r) { return 4 * r + q; }

__device__ __forceinline__ f32x4_t mfma_bf16(bf16x8_t a, bf16x8_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f64x4_t mfma_f64(double a, double b, f64x4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Coordinates of this lane's point in the bf16 B-operand layout (coordinates 8q .. 8q+7):
// hi part of Re z only (the row-maximum pass).
__device__ __forceinline__ void load_hi(const double *__restrict__ z, int64_t p, bool valid, int n,
                                        int q, uint32_t (&zh)[4]) {
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    float h[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int j = 8 * q + e + u;
      const double x = (valid && j < n) ? z[2 * (p * n + j)] : 0.0;
      h[u] = bf16_rne((float)x);
    }
    zh[e / 2] = pack2(h[0], h[1]);
  }
}

// Row maximum (pass 1) of equation tiles [t0, t1) for this lane's point, reduced over the wave's
// four lane quarters (the same point).
__device__ __forceinline__ float row_max(const DenseDev &D, int t0, int t1, int lane, int q,
                                         const bf16x8_t zh, float sf) {
  float m = -INFINITY;
  const f32x4_t zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1  // (a loop holding an MFMA is not unrolled with a remainder)
  for (int t = t0; t < t1; ++t) {
    const f32x4_t d = mfma_bf16(as_bf16x8(D.EAb[t * 64 + lane]), zh, zero);
#pragma unroll
    for (int r = 0; r < 4; ++r) m = fmaxf(m, fmaf((float)D.W[t * 16 + row_f32(q, r)], sf, d[r]));
  }
  m = fmaxf(m, __shfl_xor(m, 16));
  m = fmaxf(m, __shfl_xor(m, 32));
  return m;
}

// Writes one equation's row block of a 16-point tile from the MFMA accumulators (row layout of
// the FP64 or the FP32 result), the H_s and H columns, and the row's logscale: the column scale
// e^{M} (HOM_UNSCALED) is formed once per lane and passed by shuffle, and the e^{-z_j} factors of
// HOM_AFFINE one (row, column tile) at a time with the polynomial exp and sin/cos, so that the
// store stays small next to the contraction's registers.
template <typename OutT, int NCT, class Coef, typename AccT = f64x4_t, bool F64 = true>
__device__ __forceinline__ void store_row_lean(OutT *__restrict__ G, double *__restrict__ logscale,
                                               int flags, int64_t p0, int64_t pb, int64_t p1,
                                               int n, int k, int q, int c16,
                                               const AccT (&aR)[2], const AccT (&aI)[2],
                                               Cx<double> H, Cx<double> Hs, double m, double sp,
                                               const double *__restrict__ z, Coef kc) {
  const int ld = n + 2;
  const double own = (flags & 1) ? exp_eval(m, kc) : 1.0;  // e^{M} of this lane's point
#pragma unroll 1
  for (int rc = 0; rc < 4 * NCT; ++rc) {
    const int r = rc / NCT, ct = rc % NCT;
    const int pr = F64 ? row_f64(q, r) : row_f32(q, r);
    const int64_t p = pb + pr;
    const double scale = __shfl(own, pr);
    const int col = 16 * ct + c16;
    double vr = (double)aR[0][0], vi = (double)aI[0][0];
#pragma unroll
    for (int u = 0; u < 4 * NCT; ++u)
      if (u == rc) {
        vr = (double)aR[u % NCT][u / NCT];
        vi = (double)aI[u % NCT][u / NCT];
      }
    if (p < p1 && col < n) {
      Cx<double> v = {vr * scale, vi * scale};
      if (flags & 2) {  // times e^{-z_col}
        const double *zp = z + 2 * (p * n + col);
        double t = -zp[1] * kInv2Pi;
        t -= rint(t);
        double sn, cs;
        sincos_turns(t, sn, cs, kc);
        const double mag = exp_eval(-zp[0], kc);
        v = cmul(v, Cx<double>{mag * cs, mag * sn});
      }
      OutT *g = G + 2 * (((p - p0) * n + k) * ld + col);
      g[0] = (OutT)v.x;
      g[1] = (OutT)v.y;
    }
  }
  const int64_t p = pb + c16;
  if (q == 0 && p < p1) {
    const double fs = (flags & 2) ? own * exp_eval(-sp, kc) : own;  // H_t = e^{-s} H_s
    OutT *g = G + 2 * (((p - p0) * n + k) * ld + n);
    g[0] = (OutT)(Hs.x * fs);
    g[1] = (OutT)(Hs.y * fs);
    g[2] = (OutT)(H.x * own);
    g[3] = (OutT)(H.y * own);
    if (logscale) logscale[p * n + k] = (flags & 1) ? 0.0 : m;
  }
}


// ------------------------------------------------------------------------------------------
// BF16x3 engine
// ------------------------------------------------------------------------------------------
// LW: the liftings and the FP32 coefficients are staged in LDS once per block, when they fit
// kDenseLdsBytes; else read from global memory per term.  WF: every lifting is exactly a float
// (integers below 2^24, as the method's liftings usually are; the handle records it), so they are
// staged as float: 12 bytes per monomial instead of 16, 48 KiB at n = 32, m = 128, which lets
// three blocks (three waves per SIMD) onto a CU instead of two.
constexpr size_t kDenseLdsBytes = 64 * 1024;
constexpr size_t kCuLdsBytes = 160 * 1024;  // LDS of one CU

#ifndef HOM_BF16_WAVES
#define HOM_BF16_WAVES 4  // waves per block (they share the block's staged tables)
#endif
#ifndef HOM_BF16_EU
#define HOM_BF16_EU 3  // waves per SIMD the register budget is set for
#endif
constexpr int kBf16Block = 64 * HOM_BF16_WAVES;
// byte offset of the staged coefficients, after the Md liftings (float or double; 8-byte aligned)
template <bool WF>
__host__ __device__ constexpr size_t bf16_stage_c_offset(int Md) {
  return WF ? ((size_t)Md * 4 + 7) / 8 * 8 : (size_t)Md * 8;
}
template <typename OutT, bool LW, int NCT, bool WF>
__global__ void __launch_bounds__(kBf16Block) __attribute__((amdgpu_waves_per_eu(HOM_BF16_EU)))
    k_dense_bf16(DenseDev D, const Cx<float> *__restrict__ Cf, int64_t p0, int64_t p1,
                 const double *__restrict__ z, const double *__restrict__ s, OutT *__restrict__ G,
                 double *__restrict__ logscale, int flags, unsigned long long *units) {
  extern __shared__ __align__(16) char smem[];
  __shared__ double sK[kCoefCount];  // the polynomial constants of exp and sin/cos (the store)
  stage_coefficients(sK);
  const double *Wt = D.W;
  const float *Wf = nullptr;
  const Cx<float> *Ct = Cf;
  if constexpr (LW) {
    using WT = typename std::conditional<WF, float, double>::type;
    WT *sW = reinterpret_cast<WT *>(smem);
    Cx<float> *sC = reinterpret_cast<Cx<float> *>(smem + bf16_stage_c_offset<WF>(D.Md));
    for (int i = threadIdx.x; i < D.Md; i += blockDim.x) {
      sW[i] = (WT)D.W[i];
      sC[i] = Cf[i];
    }
    if constexpr (WF) Wf = reinterpret_cast<const float *>(sW);
    else Wt = reinterpret_cast<const double *>(sW);
    Ct = sC;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, q = lane >> 4, c16 = lane & 15;
  const int n = D.n;  // NCT = D.nct
  const int64_t ntile = (p1 - p0 + 15) >> 4;
  const f32x4_t zero = {0.f, 0.f, 0.f, 0.f};
  for (int64_t tile = (int64_t)blockIdx.x * HOM_BF16_WAVES + (threadIdx.x >> 6); tile < ntile;
       tile += (int64_t)gridDim.x * HOM_BF16_WAVES) {
    const int64_t pb = p0 + tile * 16, pl = pb + c16;
    const bool lv = pl < p1;
    // B operands: lane (c16, q) holds coordinates 8q .. 8q+7 of point c16
    uint32_t zh[4], zm[4], zl[4], th[4], tm[4], tl[4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      float h[2], m[2], l[2], a[2], b[2], c[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int j = 8 * q + e + u;
        double xr = 0.0, xi = 0.0;
        if (lv && j < n) {
          xr = z[2 * (pl * n + j)];
          xi = z[2 * (pl * n + j) + 1];
        }
        split3_rne(xr, h[u], m[u], l[u]);
        turn_digits(xi, a[u], b[u], c[u]);
      }
      zh[e / 2] = pack2(h[0], h[1]);
      zm[e / 2] = pack2(m[0], m[1]);
      zl[e / 2] = pack2(l[0], l[1]);
      th[e / 2] = pack2(a[0], a[1]);
      tm[e / 2] = pack2(b[0], b[1]);
      tl[e / 2] = pack2(c[0], c[1]);
    }
    const bf16x8_t Bzh = pack8(zh), Bzm = pack8(zm), Bzl = pack8(zl);
    const bf16x8_t Bth = pack8(th), Btm = pack8(tm), Btl = pack8(tl);
    const double sp = lv ? s[pl] : 0.0;
    const float sf = (float)sp;

    for (int k = 0; k < n; ++k) {
      const int t0 = D.tile0[k], t1 = D.tile0[k + 1];
      const float mk = row_max(D, t0, t1, lane, q, Bzh, sf);
      const double Mk = (double)mk;
      f32x4_t aR[2] = {zero, zero}, aI[2] = {zero, zero};
      float hr = 0.f, hi = 0.f, sr = 0.f, si = 0.f;
      // the MFMA operand tables of the next 32 monomials are loaded one chunk ahead
      const int ch0 = t0 >> 1, ch1 = t1 >> 1;
      uint4 eaN[2], cbN[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        eaN[u] = D.EAb[(2 * ch0 + u) * 64 + lane];
        cbN[u] = u < NCT ? D.CBb[(ch0 * 2 + u) * 64 + lane] : uint4{0, 0, 0, 0};
      }
#pragma unroll 1
      for (int ch = ch0; ch < ch1; ++ch) {
        uint32_t vr[3][4], vi[3][4];  // bf16 parts hi / mid / lo of V, packed in pairs
        const uint4 eaC[2] = {eaN[0], eaN[1]}, cbC[2] = {cbN[0], cbN[1]};
        if (ch + 1 < ch1) {
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            eaN[u] = D.EAb[(2 * (ch + 1) + u) * 64 + lane];
            if (u < NCT) cbN[u] = D.CBb[((ch + 1) * 2 + u) * 64 + lane];
          }
        }
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int t = 2 * ch + hh;
          const bf16x8_t ea = as_bf16x8(eaC[hh]);
          f32x4_t dr = mfma_bf16(ea, Bzl, zero);
          dr = mfma_bf16(ea, Bzm, dr);
          dr = mfma_bf16(ea, Bzh, dr);
          const f32x4_t d1 = mfma_bf16(ea, Bth, zero);
          const f32x4_t d2 = mfma_bf16(ea, Btm, zero);
          const f32x4_t d3 = mfma_bf16(ea, Btl, zero);
          float Vr[4], Vi[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = t * 16 + row_f32(q, r);
            const double w = (LW && WF) ? (double)Wf[i] : Wt[i];
            const float e = dr[r] + (float)fma(w, sp, -Mk);
            const float mag = __builtin_amdgcn_exp2f(e * (float)kLog2e);
            // phase in turns from the exact digit sums: fract(d1/512 + d2/512^2) + d3/512^3
            float ph = __builtin_amdgcn_fractf(d1[r] * (1.0f / 512.0f));
            ph = __builtin_amdgcn_fractf(fmaf(d2[r], 1.0f / 262144.0f, ph));
            ph = fmaf(d3[r], 1.0f / 134217728.0f, ph);
            const float sn = __builtin_amdgcn_sinf(ph), cs = __builtin_amdgcn_cosf(ph);
            const Cx<float> cc = Ct[i];
            const float cr = cc.x * mag, ci = cc.y * mag;
            Vr[r] = cr * cs - ci * sn;
            Vi[r] = cr * sn + ci * cs;
            const float wf = (float)w;
            hr += Vr[r];
            hi += Vi[r];
            sr = fmaf(wf, Vr[r], sr);
            si = fmaf(wf, Vi[r], si);
          }
#pragma unroll
          for (int r = 0; r < 4; r += 2) {
            float a0, b0, c0, a1, b1, c1;
            split3_exact(Vr[r], a0, b0, c0);
            split3_exact(Vr[r + 1], a1, b1, c1);
            vr[0][2 * hh + r / 2] = pack2(a0, a1);
            vr[1][2 * hh + r / 2] = pack2(b0, b1);
            vr[2][2 * hh + r / 2] = pack2(c0, c1);
            split3_exact(Vi[r], a0, b0, c0);
            split3_exact(Vi[r + 1], a1, b1, c1);
            vi[0][2 * hh + r / 2] = pack2(a0, a1);
            vi[1][2 * hh + r / 2] = pack2(b0, b1);
            vi[2][2 * hh + r / 2] = pack2(c0, c1);
          }
        }
        const bf16x8_t r0 = pack8(vr[0]), r1 = pack8(vr[1]), r2 = pack8(vr[2]);
        const bf16x8_t i0 = pack8(vi[0]), i1 = pack8(vi[1]), i2 = pack8(vi[2]);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const bf16x8_t cb = as_bf16x8(cbC[ct]);
          aR[ct] = mfma_bf16(r2, cb, aR[ct]);
          aR[ct] = mfma_bf16(r1, cb, aR[ct]);
          aR[ct] = mfma_bf16(r0, cb, aR[ct]);
          aI[ct] = mfma_bf16(i2, cb, aI[ct]);
          aI[ct] = mfma_bf16(i1, cb, aI[ct]);
          aI[ct] = mfma_bf16(i0, cb, aI[ct]);
        }
      }
      hr += __shfl_xor(hr, 16);
      hr += __shfl_xor(hr, 32);
      hi += __shfl_xor(hi, 16);
      hi += __shfl_xor(hi, 32);
      sr += __shfl_xor(sr, 16);
      sr += __shfl_xor(sr, 32);
      si += __shfl_xor(si, 16);
      si += __shfl_xor(si, 32);
      store_row_lean<OutT, NCT, CoefLds, f32x4_t, false>(
          G, logscale, flags, p0, pb, p1, n, k, q, c16, aR, aI, Cx<double>{hr, hi},
          Cx<double>{sr, si}, Mk, sp, z, CoefLds{sK, PointLds{}.fresh()});
    }
    if (units && lane == 0) {
      const int64_t cnt = p1 - pb < 16 ? p1 - pb : 16;
      atomicAdd(units, (unsigned long long)cnt);
    }
  }
}

// ------------------------------------------------------------------------------------------
// FP64 engine
// ------------------------------------------------------------------------------------------
#ifndef HOM_DENSE_F64_WAVES
#define HOM_DENSE_F64_WAVES 2
#endif
#ifndef HOM_DENSE_F64_KLDS
#define HOM_DENSE_F64_KLDS 0
#endif
template <typename OutT, int NCT>
__global__ void __launch_bounds__(kDenseBlock) __attribute__((amdgpu_waves_per_eu(HOM_DENSE_F64_WAVES)))
    k_dense_f64(DenseDev D, const Cx<double> *__restrict__ Cd, int64_t p0, int64_t p1,
                const double *__restrict__ z, const double *__restrict__ s, OutT *__restrict__ G,
                double *__restrict__ logscale, int flags, unsigned long long *units) {
  __shared__ double sK[kCoefCount];  // the polynomial constants of exp and sin/cos
  const int lane = threadIdx.x & 63, q = lane >> 4, c16 = lane & 15;
  const int n = D.n, nks = D.nks;  // NCT = D.nct
  stage_coefficients(sK);
  __syncthreads();
  const int64_t ntile = (p1 - p0 + 15) >> 4;
  const f64x4_t zero = {0.0, 0.0, 0.0, 0.0};
  for (int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); tile < ntile;
       tile += (int64_t)gridDim.x * 4) {
    const int64_t pb = p0 + tile * 16, pl = pb + c16;
    const bool lv = pl < p1;
    uint32_t zh[4];
    load_hi(z, pl, lv, n, q, zh);
    const bf16x8_t Bzh = pack8(zh);
    // FP64 B operands: lane (c16, q) holds coordinate q + 4 ks of point c16; Im as turns
    double zr[8], zt[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int j = q + 4 * ks;
      double xr = 0.0, t = 0.0;
      if (lv && j < n) {
        xr = z[2 * (pl * n + j)];
        t = z[2 * (pl * n + j) + 1] * kInv2Pi;
        t -= rint(t);
      }
      zr[ks] = xr;
      zt[ks] = t;
    }
    const double sp = lv ? s[pl] : 0.0;
    const float sf = (float)sp;

    for (int k = 0; k < n; ++k) {
      const int t0 = D.tile0[k], t1 = D.tile0[k + 1];
      const double Mk = (double)row_max(D, t0, t1, lane, q, Bzh, sf);
      f64x4_t aR[2] = {zero, zero}, aI[2] = {zero, zero};
      Cx<double> H = {0.0, 0.0}, Hs = {0.0, 0.0};
#ifndef HOM_DENSE_F64_PF
#define HOM_DENSE_F64_PF 1
#endif
      // the operand tables of the next tile are loaded while this one is processed
      double eaN[8], cbN[8];
      if (HOM_DENSE_F64_PF) {
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) eaN[ks] = ks < nks ? D.EAd[(t0 * 8 + ks) * 64 + lane] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          cbN[u] = (u & 1) < NCT ? D.CBd[((t0 * 4 + (u >> 1)) * 2 + (u & 1)) * 64 + lane] : 0.0;
      }
#pragma unroll 1
      for (int t = t0; t < t1; ++t) {
        double eaC[8], cbC[8];
        if (HOM_DENSE_F64_PF) {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            eaC[u] = eaN[u];
            cbC[u] = cbN[u];
          }
          if (t + 1 < t1) {
#pragma unroll
            for (int ks = 0; ks < 8; ++ks)
              if (ks < nks) eaN[ks] = D.EAd[((t + 1) * 8 + ks) * 64 + lane];
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if ((u & 1) < NCT) cbN[u] = D.CBd[(((t + 1) * 4 + (u >> 1)) * 2 + (u & 1)) * 64 + lane];
          }
        }
        // two accumulator chains per product (even / odd K steps) so that consecutive MFMAs
        // do not wait for each other's results
        f64x4_t dr0 = zero, di0 = zero, dr1 = zero, di1 = zero;
#pragma unroll
        for (int ks = 0; ks < 8; ks += 2) {
          if (ks < nks) {
            const double ea = HOM_DENSE_F64_PF ? eaC[ks] : D.EAd[(t * 8 + ks) * 64 + lane];
            dr0 = mfma_f64(ea, zr[ks], dr0);
            di0 = mfma_f64(ea, zt[ks], di0);
          }
          if (ks + 1 < nks) {
            const double ea = HOM_DENSE_F64_PF ? eaC[ks + 1] : D.EAd[(t * 8 + ks + 1) * 64 + lane];
            dr1 = mfma_f64(ea, zr[ks + 1], dr1);
            di1 = mfma_f64(ea, zt[ks + 1], di1);
          }
        }
        const f64x4_t dr = dr0 + dr1, di = di0 + di1;
#ifndef HOM_DENSE_F64_UNROLL
#define HOM_DENSE_F64_UNROLL 1
#endif
#pragma unroll HOM_DENSE_F64_UNROLL
        for (int r = 0; r < 4; ++r) {
          const int i = t * 16 + row_f64(q, r);
          const double w = D.W[i];
#if HOM_DENSE_F64_KLDS
          const CoefLds kc{sK, PointLds{}.fresh()};  // constants read at their use
#else
          const CoefConst kc{};
#endif
          const double mag = exp_eval(fma(w, sp, dr[r] - Mk), kc);
          const double ph = di[r] - rint(di[r]);
          double sn, cs;
          sincos_turns(ph, sn, cs, kc);
          const Cx<double> cc = Cd[i];
          const double cr = cc.x * mag, ci = cc.y * mag;
          const double vr = cr * cs - ci * sn, vi = cr * sn + ci * cs;
          H.x += vr;
          H.y += vi;
          Hs.x = fma(w, vr, Hs.x);
          Hs.y = fma(w, vi, Hs.y);
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            const double cb =
                HOM_DENSE_F64_PF ? cbC[2 * r + ct] : D.CBd[((t * 4 + r) * 2 + ct) * 64 + lane];
            aR[ct] = mfma_f64(vr, cb, aR[ct]);
            aI[ct] = mfma_f64(vi, cb, aI[ct]);
          }
        }
      }
      H.x += __shfl_xor(H.x, 16);
      H.x += __shfl_xor(H.x, 32);
      H.y += __shfl_xor(H.y, 16);
      H.y += __shfl_xor(H.y, 32);
      Hs.x += __shfl_xor(Hs.x, 16);
      Hs.x += __shfl_xor(Hs.x, 32);
      Hs.y += __shfl_xor(Hs.y, 16);
      Hs.y += __shfl_xor(Hs.y, 32);
      store_row_lean<OutT, NCT>(G, logscale, flags, p0, pb, p1, n, k, q, c16, aR, aI, H, Hs, Mk,
                                sp, z, CoefLds{sK, PointLds{}.fresh()});
    }
    if (units && lane == 0) {
      const int64_t cnt = p1 - pb < 16 ? p1 - pb : 16;
      atomicAdd(units, (unsigned long long)cnt);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Common-support FP64 engine (Sec. 5.1's unmixed case): a block of four waves per tile of 16
// points.
//   A1  u = A z + w s for the common monomials   FP64 MFMA (equation 0's tables: all alike)
//   A2  E = e^{u - M}, one shift M per point      FP64 vector units, once for all equations;
//                                                 the four waves split the monomial tiles and
//                                                 leave E in LDS
//   A3  per equation k: V = c_k . E, then V [a | w | 1] on the matrix cores (J_z) and the
//       vector units (H_s, H), as in the per-equation engine; the waves split the equations.
// The exponentials are formed once per (point, monomial) instead of once per (point, monomial,
// equation); the LDS tile of E is shared by the four waves, so that a CU holds enough waves to
// hide the latency of the contraction.
// ------------------------------------------------------------------------------------------
constexpr int kUnionWaves = 4;
constexpr int kUnionBlock = 64 * kUnionWaves;
constexpr size_t kUnionCoefBytes = (kCoefCount * 8 + 15) / 16 * 16;
#ifndef HOM_UNION_WAVES
#define HOM_UNION_WAVES 3
#endif

template <typename OutT, int NCT>
__global__ void __launch_bounds__(kUnionBlock) __attribute__((amdgpu_waves_per_eu(HOM_UNION_WAVES)))
    k_union_f64(DenseDev D, const Cx<double> *__restrict__ Cd, int64_t p0, int64_t p1,
                const double *__restrict__ z, const double *__restrict__ s, OutT *__restrict__ G,
                double *__restrict__ logscale, int flags, unsigned long long *units) {
  extern __shared__ __align__(16) char smem[];
  double *sK = reinterpret_cast<double *>(smem);  // the polynomial constants of exp and sin/cos
  Cx<double> *sE = reinterpret_cast<Cx<double> *>(smem + kUnionCoefBytes);  // [tiles][4][64]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, q = lane >> 4, c16 = lane & 15;
  const int n = D.n, nks = D.nks;  // NCT = D.nct
  const int t0 = D.tile0[0], t1 = D.tile0[1];  // the common support's 16-monomial tiles
  const int64_t ntile = (p1 - p0 + 15) >> 4;
  const f64x4_t zero = {0.0, 0.0, 0.0, 0.0};
  stage_coefficients(sK);
  __syncthreads();
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t pb = p0 + tile * 16, pl = pb + c16;
    const bool lv = pl < p1;
    uint32_t zh[4];
    load_hi(z, pl, lv, n, q, zh);
    const bf16x8_t Bzh = pack8(zh);
    double zr[8], zt[8];
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int j = q + 4 * ks;
      double xr = 0.0, t = 0.0;
      if (lv && j < n) {
        xr = z[2 * (pl * n + j)];
        t = z[2 * (pl * n + j) + 1] * kInv2Pi;
        t -= rint(t);
      }
      zr[ks] = xr;
      zt[ks] = t;
    }
    const double sp = lv ? s[pl] : 0.0;
    const float sf = (float)sp;
    // one shift per point: the support's row maximum (hi parts of Re z, + w s); every wave forms
    // it from the same operands in the same order, so the four copies agree bit for bit
    const double Mp = (double)row_max(D, t0, t1, lane, q, Bzh, sf);
    // ---- A1 + A2 once, this wave's share of the tiles ----
#pragma unroll 1
    for (int t = t0 + wv; t < t1; t += kUnionWaves) {
      f64x4_t dr0 = zero, di0 = zero, dr1 = zero, di1 = zero;
#pragma unroll
      for (int ks = 0; ks < 8; ks += 2) {
        if (ks < nks) {
          const double ea = D.EAd[(t * 8 + ks) * 64 + lane];
          dr0 = mfma_f64(ea, zr[ks], dr0);
          di0 = mfma_f64(ea, zt[ks], di0);
        }
        if (ks + 1 < nks) {
          const double ea = D.EAd[(t * 8 + ks + 1) * 64 + lane];
          dr1 = mfma_f64(ea, zr[ks + 1], dr1);
          di1 = mfma_f64(ea, zt[ks + 1], di1);
        }
      }
      const f64x4_t dr = dr0 + dr1, di = di0 + di1;
#pragma unroll 2
      for (int r = 0; r < 4; ++r) {
        const int i = t * 16 + row_f64(q, r);
        const CoefLds kc{sK, PointLds{}.fresh()};  // constants read at their use, not hoisted
        const double mag = exp_eval(fma(D.W[i], sp, dr[r] - Mp), kc);
        const double ph = di[r] - rint(di[r]);
        double sn, cs;
        sincos_turns(ph, sn, cs, kc);
        sE[((t - t0) * 4 + r) * 64 + lane] = Cx<double>{mag * cs, mag * sn};
      }
    }
    __syncthreads();
    // ---- A3, this wave's equations ----
    for (int k = wv; k < n; k += kUnionWaves) {
      const int ck = D.tile0[k] * 16 - t0 * 16;  // equation k's slots, relative to the support
      f64x4_t aR[2] = {zero, zero}, aI[2] = {zero, zero};
      Cx<double> H = {0.0, 0.0}, Hs = {0.0, 0.0};
#pragma unroll 1
      for (int t = t0; t < t1; ++t) {
        Cx<double> e[4], cc[4];
        double cb[8], w[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {  // every operand of the tile first, then the arithmetic
          const int i = t * 16 + row_f64(q, r);
          e[r] = sE[((t - t0) * 4 + r) * 64 + lane];
          cc[r] = Cd[ck + i];
          w[r] = D.W[i];
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) cb[2 * r + ct] = D.CBd[((t * 4 + r) * 2 + ct) * 64 + lane];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const Cx<double> v = cmul(cc[r], e[r]);
          H.x += v.x;
          H.y += v.y;
          Hs.x = fma(w[r], v.x, Hs.x);
          Hs.y = fma(w[r], v.y, Hs.y);
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            aR[ct] = mfma_f64(v.x, cb[2 * r + ct], aR[ct]);
            aI[ct] = mfma_f64(v.y, cb[2 * r + ct], aI[ct]);
          }
        }
      }
      H.x += __shfl_xor(H.x, 16);
      H.x += __shfl_xor(H.x, 32);
      H.y += __shfl_xor(H.y, 16);
      H.y += __shfl_xor(H.y, 32);
      Hs.x += __shfl_xor(Hs.x, 16);
      Hs.x += __shfl_xor(Hs.x, 32);
      Hs.y += __shfl_xor(Hs.y, 16);
      Hs.y += __shfl_xor(Hs.y, 32);
      store_row_lean<OutT, NCT>(G, logscale, flags, p0, pb, p1, n, k, q, c16, aR, aI, H, Hs, Mp,
                                sp, z, CoefLds{sK, PointLds{}.fresh()});
    }
    __syncthreads();  // E of this tile is read by every wave before the next tile overwrites it
    if (units && threadIdx.x == 0) {
      const int64_t cnt = p1 - pb < 16 ? p1 - pb : 16;
      atomicAdd(units, (unsigned long long)cnt);
    }
  }
}

// Coefficients in the padded dense order (padding monomials get 0), FP64 and FP32 copies.
__global__ void k_dense_coeffs(DenseDev D, const double *__restrict__ c, Cx<double> *__restrict__ Cd,
                               Cx<float> *__restrict__ Cf) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < D.Md; i += gridDim.x * blockDim.x) {
    const int q = D.src[i];
    Cx<double> v = {0.0, 0.0};
    if (q >= 0) v = {c[2 * q], c[2 * q + 1]};
    Cd[i] = v;
    Cf[i] = {(float)v.x, (float)v.y};
  }
}

// ------------------------------------------------------------------------------------------
// A5 after a dense evaluation: the consolidated LU on rows read back from the chunk workspace.
// Mixed form: FP32 rows and LU; a point whose FP32 pivot ratio is below 1e-4 (or singular) is
// evaluated again on the vector units in FP64 and solved in FP64, as in the fused step.
// ------------------------------------------------------------------------------------------
template <int N, bool MIXED, bool GT>
__global__ void __launch_bounds__(kDenseBlock) __attribute__((amdgpu_waves_per_eu(MIXED && N <= 20 ? 3 : 1)))
    k_dense_lu(SysDev sd, const double *__restrict__ c, int64_t p0, int64_t p1,
               const void *__restrict__ Gws, const double *__restrict__ z,
               const double *__restrict__ s, double *__restrict__ dE, double *__restrict__ dN,
               int32_t *__restrict__ status) {
  using T = typename std::conditional<MIXED, float, double>::type;
  const T *Gw = static_cast<const T *>(Gws);
  const Geo<N> geo;
  const int n = sd.n, r = geo.r, ld = n + 2;
  const int64_t gpb = (kDenseBlock / 64) * Geo<N>::G;
  const int64_t stride = (int64_t)gridDim.x * gpb;
  const int64_t q0 = p0 + (int64_t)blockIdx.x * gpb + (threadIdx.x >> 6) * Geo<N>::G + geo.g;
  for (int64_t it = 0;; ++it) {
    const int64_t p = q0 + it * stride;
    const bool act = geo.valid && p < p1;
    if (!__any(act)) break;
    Cx<T> row[N + 2];
#pragma unroll
    for (int j = 0; j < N + 2; ++j) row[j] = {T(0), T(0)};
    if (act && r < n) {
      const T *g = Gw + 2 * ((p - p0) * n + r) * ld;
#pragma unroll
      for (int j = 0; j < N; ++j)
        if (j < n) row[j] = {g[2 * j], g[2 * j + 1]};
      row[N] = {g[2 * n], g[2 * n + 1]};
      row[N + 1] = {g[2 * n + 2], g[2 * n + 3]};
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j)
        if (j == r) row[j].x = T(1);
    }
    Cx<T> ef, qf;
    double nE, nN;
    T rf;
    bool sing = lu_solve2<N, T>(row, r, geo.base, n, ef, qf, nE, nN, rf);
    Cx<double> e = {(double)ef.x, (double)ef.y}, qv = {(double)qf.x, (double)qf.y};
    double ratio = (double)rf;
    // mixed form: a point the FP32 LU cannot resolve is marked for the FP64 pass that follows
    // (k_dense_redo), which keeps the FP64 evaluation's registers out of this kernel
    const bool redo = MIXED && (sing || !(rf >= T(1e-4)));
    if (act) {
      if (r < n) {
        dE[2 * (p * n + r)] = e.x;
        dE[2 * (p * n + r) + 1] = e.y;
        dN[2 * (p * n + r)] = qv.x;
        dN[2 * (p * n + r) + 1] = qv.y;
      }
      if (r == 0) status[p] = redo ? kDenseRedo : ((sing || !(ratio >= 1e-14)) ? -1 : 0);
    }
  }
}

// FP64 evaluation and LU of the points the mixed form's FP32 LU marked (status kDenseRedo).
template <int N, bool GT>
__global__ void __launch_bounds__(kDenseBlock)
    k_dense_redo(SysDev sd, const double *__restrict__ c, int64_t p0, int64_t p1,
                 const double *__restrict__ z, const double *__restrict__ s,
                 double *__restrict__ dE, double *__restrict__ dN, int32_t *__restrict__ status) {
  extern __shared__ __align__(16) char smem[];
  const SysLds<N> S = stage_tables<N, GT>(smem, sd, c);
  const Geo<N> geo;
  const int n = sd.n, r = geo.r;
  const int64_t gpb = (kDenseBlock / 64) * Geo<N>::G;
  const int64_t stride = (int64_t)gridDim.x * gpb;
  const int64_t q0 = p0 + (int64_t)blockIdx.x * gpb + (threadIdx.x >> 6) * Geo<N>::G + geo.g;
  for (int64_t it = 0;; ++it) {
    const int64_t p = q0 + it * stride;
    const bool inside = geo.valid && p < p1;
    if (!__any(inside)) break;
    const bool act = inside && status[p] == kDenseRedo;
    if (!__any(act)) continue;
    double zr[N], zi[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      zr[j] = (act && j < n) ? z[2 * (p * n + j)] : 0.0;
      zi[j] = (act && j < n) ? z[2 * (p * n + j) + 1] : 0.0;
    }
    const double sp = act ? s[p] : 0.0;
    Cx<double> row[N + 2], e, q;
    double M, absum, ratio, nE, nN;
    eval_row_exact<N, double>(S, r, zr, zi, sp, row, M, absum);
    const bool sing = lu_solve2<N, double>(row, r, geo.base, n, e, q, nE, nN, ratio);
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
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t dense_ws_bytes(const System &S, int64_t P, bool step, int engine) {
  size_t b = align256((size_t)S.Md * 16) + align256((size_t)S.Md * 8);
  if (step) {
    const int64_t pc = P < kDenseChunk ? P : kDenseChunk;
    b += align256((size_t)pc * S.n * (S.n + 2) * (engine == 1 ? 8 : 16));
  }
  return b;
}

static int dense_grid(int64_t npts) {
  const int64_t tiles = (npts + 15) / 16;
  const int64_t need = (tiles + 3) / 4;
  const int64_t cap = (int64_t)num_cus() * 8;
  return (int)(need < cap ? (need > 0 ? need : 1) : cap);
}

static hipError_t dense_coeffs(const System &S, const double *c, void *dws, Cx<double> **Cd,
                               Cx<float> **Cf, hipStream_t stream) {
  char *base = static_cast<char *>(dws);
  *Cd = reinterpret_cast<Cx<double> *>(base);
  *Cf = reinterpret_cast<Cx<float> *>(base + align256((size_t)S.Md * 16));
  hipLaunchKernelGGL(k_dense_coeffs, dim3((S.Md + 255) / 256), dim3(256), 0, stream, S.dense, c,
                     *Cd, *Cf);
  return hipGetLastError();
}

template <typename OutT>
static void dense_launch(const System &S, int engine, const Cx<double> *Cd, const Cx<float> *Cf,
                         int64_t p0, int64_t p1, const double *z, const double *s, OutT *G,
                         double *logscale, int flags, hipStream_t stream) {
  prof_begin(stream);
  unsigned long long *units = prof_units(stream);
  const dim3 grid(dense_grid(p1 - p0)), block(kDenseBlock);
  const bool wf = S.dense.w_f32 != 0;
  const size_t lw = (wf ? bf16_stage_c_offset<true>(S.Md) : bf16_stage_c_offset<false>(S.Md)) +
                    (size_t)S.Md * 8;
  if (engine == 1) {
    const int64_t tiles = (p1 - p0 + 15) / 16, need = (tiles + HOM_BF16_WAVES - 1) / HOM_BF16_WAVES;
    const dim3 bb(kBf16Block);
    if (lw <= kDenseLdsBytes) {  // the blocks that fit a CU's LDS hold the staged tables
      const int64_t per = (int64_t)(kCuLdsBytes / lw) < 8 ? (int64_t)(kCuLdsBytes / lw) : 8;
      const int64_t cap = per * (int64_t)num_cus();
      const dim3 g2((unsigned)(need < cap ? (need > 0 ? need : 1) : cap));
      auto kern = S.dense.nct == 1 ? (wf ? k_dense_bf16<OutT, true, 1, true> : k_dense_bf16<OutT, true, 1, false>)
                                   : (wf ? k_dense_bf16<OutT, true, 2, true> : k_dense_bf16<OutT, true, 2, false>);
      hipLaunchKernelGGL(kern, g2, bb, lw, stream, S.dense, Cf, p0, p1, z, s, G, logscale, flags,
                         units);
    } else {
      const int64_t cap = (int64_t)num_cus() * 8;
      const dim3 g1((unsigned)(need < cap ? (need > 0 ? need : 1) : cap));
      if (S.dense.nct == 1)
        hipLaunchKernelGGL((k_dense_bf16<OutT, false, 1, false>), g1, bb, 0, stream, S.dense, Cf, p0,
                           p1, z, s, G, logscale, flags, units);
      else
        hipLaunchKernelGGL((k_dense_bf16<OutT, false, 2, false>), g1, bb, 0, stream, S.dense, Cf, p0,
                           p1, z, s, G, logscale, flags, units);
    }
  } else if (S.union_support) {  // common support: the exponentials once per point
    const size_t lds = kUnionCoefBytes + (size_t)S.union_tiles * 4 * 64 * 16;
    const int64_t tiles = (p1 - p0 + 15) / 16;
    // exactly the blocks that are resident at once (registers or LDS, whichever binds): every
    // block strides over the same number of tiles, and none waits for a slot
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, S.dense.nct == 1 ? k_union_f64<OutT, 1> : k_union_f64<OutT, 2>, kUnionBlock,
            lds) != hipSuccess || per_cu < 1)
      per_cu = 1;
    const int64_t cap = (int64_t)num_cus() * per_cu;
    const dim3 gu((unsigned)(tiles < cap ? (tiles > 0 ? tiles : 1) : cap));
    if (S.dense.nct == 1)
      hipLaunchKernelGGL((k_union_f64<OutT, 1>), gu, dim3(kUnionBlock), lds, stream, S.dense, Cd,
                         p0, p1, z, s, G, logscale, flags, units);
    else
      hipLaunchKernelGGL((k_union_f64<OutT, 2>), gu, dim3(kUnionBlock), lds, stream, S.dense, Cd,
                         p0, p1, z, s, G, logscale, flags, units);
  } else if (S.dense.nct == 1)
    hipLaunchKernelGGL((k_dense_f64<OutT, 1>), grid, block, 0, stream, S.dense, Cd, p0, p1, z, s,
                       G, logscale, flags, units);
  else
    hipLaunchKernelGGL((k_dense_f64<OutT, 2>), grid, block, 0, stream, S.dense, Cd, p0, p1, z, s,
                       G, logscale, flags, units);
  prof_end(stream, engine == 1 ? "k_dense<bf16x3>"
                               : (S.union_support ? "k_union<fp64>" : "k_dense<fp64>"));
}

hipError_t launch_dense_eval(const System &S, const double *c, int64_t P, const double *z,
                             const double *s, double *G, double *logscale, int flags, int engine,
                             void *dws, hipStream_t stream) {
  Cx<double> *Cd;
  Cx<float> *Cf;
  hipError_t e = dense_coeffs(S, c, dws, &Cd, &Cf, stream);
  if (e != hipSuccess) return e;
  dense_launch<double>(S, engine, Cd, Cf, 0, P, z, s, G, logscale, flags, stream);
  return hipGetLastError();
}

template <int N>
static hipError_t dense_lu_n(const System &S, const void *cws, const double *c, int64_t p0,
                             int64_t p1, const void *Gws, const double *z, const double *s,
                             double *dE, double *dN, int32_t *status, bool mixed,
                             hipStream_t stream) {
  const int gpb = (kDenseBlock / 64) * Geo<N>::G;
  const int64_t need = (p1 - p0 + gpb - 1) / gpb;
  const int64_t cap = (int64_t)num_cus() * 8;
  const dim3 grid((unsigned)(need < cap ? need : cap)), block(kDenseBlock);
  char label[64];
  snprintf(label, sizeof label, "k_dense_lu<%d,%s>", N, mixed ? "mixed" : "fp64");
  prof_begin(stream);
  const size_t tb = mixed ? (S.lds_bytes + 15) & ~(size_t)15 : 0;
  auto kern = mixed ? (S.global_tables ? k_dense_lu<N, true, true> : k_dense_lu<N, true, false>)
                    : k_dense_lu<N, false, false>;
  hipLaunchKernelGGL(kern, grid, block, 0, stream, S.dev(cws), c, p0, p1, Gws, z, s, dE, dN,
                     status);
  prof_end(stream, label);
  if (mixed) {
    snprintf(label, sizeof label, "k_dense_redo<%d>", N);
    prof_begin(stream);
    auto kr = S.global_tables ? k_dense_redo<N, true> : k_dense_redo<N, false>;
    hipLaunchKernelGGL(kr, grid, block, tb, stream, S.dev(cws), c, p0, p1, z, s, dE, dN, status);
    prof_end(stream, label);
  }
  return hipGetLastError();
}

#define HOM_SWITCH_D(N, CALL)                  \
  switch (N) {                                 \
    case 2: { constexpr int NN = 2; CALL; }    \
    case 3: { constexpr int NN = 3; CALL; }    \
    case 4: { constexpr int NN = 4; CALL; }    \
    case 5: { constexpr int NN = 5; CALL; }    \
    case 6: { constexpr int NN = 6; CALL; }    \
    case 7: { constexpr int NN = 7; CALL; }    \
    case 8: { constexpr int NN = 8; CALL; }    \
    case 10: { constexpr int NN = 10; CALL; }  \
    case 12: { constexpr int NN = 12; CALL; }  \
    case 16: { constexpr int NN = 16; CALL; }  \
    case 20: { constexpr int NN = 20; CALL; }  \
    case 24: { constexpr int NN = 24; CALL; }  \
    case 32: { constexpr int NN = 32; CALL; }  \
    default: return hipErrorInvalidValue;      \
  }

hipError_t launch_dense_step(const System &S, const void *cws, const double *c, int64_t P,
                             const double *z, const double *s, double *dE, double *dN,
                             int32_t *status, int precision, void *dws, hipStream_t stream) {
  const bool mixed = precision == 1;
  const int engine = mixed ? 1 : 0;
  Cx<double> *Cd;
  Cx<float> *Cf;
  hipError_t e = dense_coeffs(S, c, dws, &Cd, &Cf, stream);
  if (e != hipSuccess) return e;
  char *Gws = static_cast<char *>(dws) + align256((size_t)S.Md * 16) + align256((size_t)S.Md * 8);
  for (int64_t p0 = 0; p0 < P; p0 += kDenseChunk) {
    const int64_t p1 = P - p0 < kDenseChunk ? P : p0 + kDenseChunk;
    if (mixed)
      dense_launch<float>(S, engine, Cd, Cf, p0, p1, z, s, reinterpret_cast<float *>(Gws), nullptr,
                          0, stream);
    else
      dense_launch<double>(S, engine, Cd, Cf, p0, p1, z, s, reinterpret_cast<double *>(Gws),
                           nullptr, 0, stream);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    HOM_SWITCH_D(S.N, e = dense_lu_n<NN>(S, cws, c, p0, p1, Gws, z, s, dE, dN, status, mixed,
                                         stream);
                 break)
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace hom
