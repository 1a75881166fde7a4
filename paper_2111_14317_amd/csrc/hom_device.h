// Device building blocks of the homotopy hot path for gfx950 (wave64).
//
// Work mapping.  A path (or point) is owned by a group of N consecutive lanes of a wave, N = the
// system's n rounded up to a compiled size; lane r of the group owns equation r.  A wave holds
// G = 64 / N groups.  Lanes r >= n of a group are padding: they produce an identity row, so the
// padded unknowns solve to zero.
//
//  * eval_row   (A1-A3, Sec. 5.1-5.2): lane r forms, for each monomial i of equation r, the
//    exponent u = <a_i, z> + w_i s (a real x complex contraction over the exponent table), the
//    row maximum M_r of Re u, the shifted term V_i = c_i exp(u - M_r), and accumulates
//    V_i * [a_i | w_i | 1] into row r of the extended Jacobian [J_z | H_s | H].  All of this is
//    lane-local: no cross-lane traffic during the evaluation.
//  * lu_solve2  (A5, Sec. 6 in its affine form): LU with partial pivoting of J_z on the augmented
//    rows, both right-hand sides (H_s, H) at once.  Rows stay in registers; the pivot search is a
//    rotation-doubling max of packed (magnitude, row) keys across the group and the pivot row is
//    broadcast with ds_bpermute.  Back substitution is column oriented, so every solution entry
//    is broadcast once.
//
// The exponent table in LDS is laid out [i][r][LD] (monomial, equation, exponent) with the
// lifting w in slot N and LD odd, so the n lanes of a group reading monomial i of their own
// equations hit distinct LDS banks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hom {

constexpr double kInv2Pi = 0.159154943091895335768883763372514362;  // 1 / (2 pi)
constexpr double kLog2e = 1.44269504088896340735992468100189214;

template <typename T>
struct Cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// a - l * b
template <typename T>
__device__ __forceinline__ Cx<T> cfnms(Cx<T> a, Cx<T> l, Cx<T> b) {
  Cx<T> r;
  r.x = fma(-l.x, b.x, fma(l.y, b.y, a.x));
  r.y = fma(-l.x, b.y, fma(-l.y, b.x, a.y));
  return r;
}

// a + l * b
template <typename T>
__device__ __forceinline__ Cx<T> cfma(Cx<T> a, Cx<T> l, Cx<T> b) {
  Cx<T> r;
  r.x = fma(l.x, b.x, fma(-l.y, b.y, a.x));
  r.y = fma(l.x, b.y, fma(l.y, b.x, a.y));
  return r;
}

// 1/x: hardware reciprocal estimate refined by Newton steps (two in FP64: ~1 ulp), instead of the
// IEEE division sequence.
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ float fast_rcp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// ------------------------------------------------------------------------------------------
// FP64 exponential and sine/cosine of the evaluation's terms (A2)
// ------------------------------------------------------------------------------------------
// The library routines accept every input (infinities, huge arguments, denormal results) at
// several times the cost.  The terms' arguments are bounded: the shifted exponent Re u - M (at
// most the lag margin above 0; below about -745 the term underflows to 0) and a phase already
// reduced to [-1/2, 1/2] turns.  On those ranges both functions are accurate to a few ulp; a
// non-finite argument gives NaN.
//
// e^x: Cody-Waite reduction x = k ln 2 + r, |r| <= ln 2 / 2, with ln 2 split into a head whose
// low 21 bits are zero (k * head is exact for |k| < 2^21) and a tail; the Taylor polynomial of
// e^r to degree 13 (truncation error below 2^-57 relative); the result scaled by 2^k.
// sin and cos of 2 pi t for |t| <= 1/2: quadrant q = rint(4 t), f = t - q/4 (exact), the angle
// 2 pi f in [-pi/4, pi/4] through the Taylor polynomials of sin (degree 17) and cos (degree 16),
// whose truncation errors stay below 2^-53 there, then the rotation by q quarter turns.
//
// The coefficients sit in one compile-time table: 1/k! for e^r (k = 13 down to 0), the sine's
// (odd k = 17 down to 1, alternating signs), the cosine's (even k = 16 down to 0), then ln 2
// (head, tail) and 2 pi.
enum : int { kCoefExp = 0, kCoefSin = 14, kCoefCos = 23, kCoefLn2Hi = 32, kCoefLn2Lo = 33,
             kCoefTwoPi = 34, kCoefCount = 35 };
#define HOM_FP64_COEFFICIENTS                                                                     \
  1.0 / 6227020800.0, 1.0 / 479001600.0, 1.0 / 39916800.0, 1.0 / 3628800.0, 1.0 / 362880.0,      \
      1.0 / 40320.0, 1.0 / 5040.0, 1.0 / 720.0, 1.0 / 120.0, 1.0 / 24.0, 1.0 / 6.0, 0.5, 1.0, 1.0, \
      1.0 / 355687428096000.0, -1.0 / 1307674368000.0, 1.0 / 6227020800.0, -1.0 / 39916800.0,     \
      1.0 / 362880.0, -1.0 / 5040.0, 1.0 / 120.0, -1.0 / 6.0, 1.0,                                \
      1.0 / 20922789888000.0, -1.0 / 87178291200.0, 1.0 / 479001600.0, -1.0 / 3628800.0,          \
      1.0 / 40320.0, -1.0 / 720.0, 1.0 / 24.0, -0.5, 1.0,                                         \
      0.6931471803691238 /* ln 2, low 21 bits cleared */,                                         \
      1.9082149292705877e-10 /* ln 2 minus the head */, 6.283185307179586
struct CoefConst {
  __host__ __device__ constexpr double operator()(int k) const {
    constexpr double c[kCoefCount] = {HOM_FP64_COEFFICIENTS};
    return c[k];
  }
  __host__ __device__ constexpr CoefConst at(int) const { return *this; }
};
// The same table in LDS (staged by the block), read at each use: a kernel whose registers cannot
// also hold 35 FP64 constants takes them from there.  `off` is an opaque zero produced inside the
// caller's loop, so that the reads stay next to their uses instead of being hoisted.
struct CoefLds {
  const double *K;
  int off = 0;
  __device__ double operator()(int k) const { return K[off + k]; }
  __device__ CoefLds at(int o) const { return CoefLds{K, o}; }
};
__device__ __forceinline__ void stage_coefficients(double *sK) {  // visible after a barrier
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kCoefCount; ++i) sK[i] = CoefConst{}(i);
  }
}

template <class Coef = CoefConst>
__host__ __device__ __forceinline__ double exp_eval(double x, Coef c = Coef{}) {
  const double k = rint(x * kLog2e);
  double r = fma(-k, c(kCoefLn2Hi), x);
  r = fma(-k, c(kCoefLn2Lo), r);
  double p = c(kCoefExp);
#pragma unroll
  for (int i = 1; i < 14; ++i) p = fma(p, r, c(kCoefExp + i));
  return ldexp(p, (int)k);
}

template <class Coef = CoefConst>
__host__ __device__ __forceinline__ void sincos_turns(double t, double &sn, double &cs,
                                                      Coef c = Coef{}) {
  const double q = rint(4.0 * t);
  const double th = fma(-0.25, q, t) * c(kCoefTwoPi);
  const double t2 = th * th;
  double ps = c(kCoefSin);
#pragma unroll
  for (int i = 1; i < 9; ++i) ps = fma(ps, t2, c(kCoefSin + i));
  const double s0 = th * ps;
  double pc = c(kCoefCos);
#pragma unroll
  for (int i = 1; i < 9; ++i) pc = fma(pc, t2, c(kCoefCos + i));
  const double c0 = pc;
  const int qi = (int)q & 3;  // the angle is 2 pi f + qi pi/2
  const double a = (qi & 1) ? c0 : s0, b = (qi & 1) ? s0 : c0;
  sn = (qi & 2) ? -a : a;
  cs = ((qi + 1) & 2) ? -b : b;
}

template <typename T>
__device__ __forceinline__ Cx<T> shfl_cx(Cx<T> v, int src) {
  return {__shfl(v.x, src, 64), __shfl(v.y, src, 64)};
}

// Stride of one (monomial, equation) record in the exponent table: N exponents, the lifting, and
// one pad slot when needed to make the stride odd (conflict-free LDS reads across a group).
template <int N>
struct TableLD {
  static constexpr int value = ((N + 1) & 1) ? (N + 1) : (N + 2);
};

template <int N>
struct Geo {
  static constexpr int G = 64 / N;  // groups per wave
  int lane, g, r, base;
  bool valid;  // lane belongs to a full group
  __device__ __forceinline__ Geo() {
    lane = threadIdx.x & 63;
    g = lane / N;
    r = lane - g * N;
    base = g * N;
    valid = g < G;
  }
};

// Pivot-search key: the top 32 bits of a non-negative magnitude (monotone in the value), with the
// low 6 bits replaced by 63 - r, so that an unsigned max over the group returns the largest
// magnitude (to ~14 significant bits) and, among equal keys, the lowest row.  Rows already used
// as pivots get key 0, below every candidate.
__device__ __forceinline__ uint32_t pivot_key(double mag, int r) {
  const uint32_t hi = (uint32_t)(__double_as_longlong(mag) >> 32);
  return (hi & ~63u) | (uint32_t)(63 - r);
}
__device__ __forceinline__ uint32_t pivot_key(float mag, int r) {
  return ((uint32_t)__float_as_uint(mag) & ~63u) | (uint32_t)(63 - r);
}

template <int N>
__device__ __forceinline__ uint32_t group_max_u32(uint32_t v, int r, int base) {
#pragma unroll
  for (int off = 1; off < N; off <<= 1) {
    int t = r + off;
    t = t >= N ? t - N : t;
    const uint32_t o = (uint32_t)__shfl((int)v, base + t, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Maximum over the group (every lane ends with it); NaN propagates.
template <int N, typename T>
__device__ __forceinline__ T group_max(T v, int r, int base) {
#pragma unroll
  for (int off = 1; off < N; off <<= 1) {
    int t = r + off;
    t = t >= N ? t - N : t;
    const T o = __shfl(v, base + t, 64);
    v = (o > v || o != o) ? o : v;  // propagates NaN
  }
  return v;
}

// Maximum over the group of a value that is >= +0 or NaN: an unsigned maximum of the bit
// patterns, which is monotone on non-negative floats and puts every NaN above +inf.
template <int N>
__device__ __forceinline__ float group_max_nonneg(float v, int r, int base) {
  return __uint_as_float(group_max_u32<N>(__float_as_uint(v), r, base));
}

// Bitwise OR over the group (every lane ends with it).
template <int N>
__device__ __forceinline__ uint32_t group_or_u32(uint32_t v, int r, int base) {
#pragma unroll
  for (int off = 1; off < N; off <<= 1) {
    int t = r + off;
    t = t >= N ? t - N : t;
    v |= (uint32_t)__shfl((int)v, base + t, 64);
  }
  return v;
}

// ------------------------------------------------------------------------------------------
// tables staged in LDS
// ------------------------------------------------------------------------------------------
struct SysDev {
  int n;              // true number of equations / unknowns
  int mmax;           // largest m_k
  int M;              // total monomials
  const double *T;    // [mmax][n][LD] exponents (as doubles, zero padded to N) + lifting
  const int32_t *mk;  // [n]
  const int32_t *off; // [n] offset of equation k in the equation-major arrays
  // Tables too large for LDS stay in global memory: then Cg / Cabs_g hold this call's
  // coefficients and their moduli in table order [mmax][n] (built by a prologue kernel),
  // otherwise both are null and the block stages everything into LDS.
  const Cx<double> *Cg;
  const double *Cabs_g;
};

// LDS image of a system: exponent table, coefficients in table order, |c|, m_k.
template <int N>
struct SysLds {
  const double *T;
  const Cx<double> *C;
  const double *Cabs;
  const int32_t *mk;
  int n, mmax;
};

template <int N>
__host__ __device__ constexpr size_t lds_table_bytes(int n, int mmax) {
  return (size_t)mmax * n * TableLD<N>::value * 8 + (size_t)mmax * n * (16 + 8) + 4 * 32 + 64;
}

// Cooperative copy of the tables into LDS (whole block).  c: complex128 [M] equation-major.
// GT (tables in global memory): only return the global pointers.  A compile-time choice, so
// that the evaluation's table reads compile to LDS instructions when the tables are staged.
template <int N, bool GT>
__device__ SysLds<N> stage_tables(char *smem, const SysDev &sd, const double *__restrict__ c) {
  if constexpr (GT) return SysLds<N>{sd.T, sd.Cg, sd.Cabs_g, sd.mk, sd.n, sd.mmax};
  constexpr int LD = TableLD<N>::value;
  const int n = sd.n, mmax = sd.mmax;
  double *sT = reinterpret_cast<double *>(smem);
  const int nT = mmax * n * LD;
  Cx<double> *sC = reinterpret_cast<Cx<double> *>(sT + nT);
  double *sA = reinterpret_cast<double *>(sC + mmax * n);
  int32_t *sM = reinterpret_cast<int32_t *>(sA + mmax * n);
  for (int idx = threadIdx.x; idx < nT; idx += blockDim.x) sT[idx] = sd.T[idx];
  for (int idx = threadIdx.x; idx < mmax * n; idx += blockDim.x) {
    const int i = idx / n, r = idx - (idx / n) * n;
    Cx<double> v = {0.0, 0.0};
    if (i < sd.mk[r]) {
      const int q = sd.off[r] + i;
      v.x = c[2 * q];
      v.y = c[2 * q + 1];
    }
    sC[idx] = v;
    sA[idx] = sqrt(v.x * v.x + v.y * v.y);
  }
  for (int idx = threadIdx.x; idx < n; idx += blockDim.x) sM[idx] = sd.mk[idx];
  __syncthreads();
  return SysLds<N>{sT, sC, sA, sM, n, mmax};
}

// Tables of the FP32 evaluation (the mixed form), staged beside the FP64 ones: the exponents as
// f16 (exact: |a| <= 127), H16<N> halves per (monomial, equation) record, which the row
// accumulation feeds to mixed f16 x f32 FMAs without conversions, and {Re c, Im c, |c|, w} as
// float.  Null pointers: the evaluation converts the FP64 tables instead.
template <int N>
struct H16 {
  static constexpr int value = (N + 3) / 4 * 4;  // 8-byte records: conflict-free for N <= 12
};
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
template <int N>
struct F32Tables {
  const half4_t *Th;  // [mmax][n][H16 / 4]
  const float4 *Cf;   // [mmax][n]
};
template <int N>
__host__ __device__ constexpr size_t lds_f32_bytes(int n, int mmax) {
  return (size_t)mmax * n * (H16<N>::value * 2 + 16);
}

// Stage the FP32 tables at `dst` (16-byte aligned, lds_f32_bytes) from the staged FP64 tables
// (which must be visible: call after stage_tables); ends with a barrier.
template <int N>
__device__ F32Tables<N> stage_f32_tables(char *dst, const SysLds<N> &S) {
  constexpr int LD = TableLD<N>::value, H = H16<N>::value;
  const int n = S.n, recs = S.mmax * S.n;
  float4 *Cf = reinterpret_cast<float4 *>(dst);
  _Float16 *Th = reinterpret_cast<_Float16 *>(Cf + recs);
  for (int idx = threadIdx.x; idx < recs; idx += blockDim.x) {
    const double *t = S.T + idx * LD;  // record (i, r) = idx: the same order
    const Cx<double> cc = S.C[idx];
    Cf[idx] = make_float4((float)cc.x, (float)cc.y, (float)S.Cabs[idx], (float)t[N]);
#pragma unroll
    for (int j = 0; j < H; ++j) Th[idx * H + j] = (_Float16)(j < N ? (float)t[j] : 0.0f);
  }
  (void)n;
  __syncthreads();
  return F32Tables<N>{reinterpret_cast<const half4_t *>(Th), Cf};
}

// ------------------------------------------------------------------------------------------
// A1-A3: one row of [J_z | H_s | H] at (z, s), scaled by e^{-M_r}
// ------------------------------------------------------------------------------------------
// row[j], j < N: dh_r/dz_j;  row[N]: dh_r/ds;  row[N+1]: h_r.  logM = M_r; absum = sum |V_i|.
// T is the precision of the exponentials and of the contraction (double, or float for the
// mixed form).  The exponent sums u are always formed in FP64.
//
// Row shift.  With `exact` the shift is the row maximum of Re u (a first pass over the
// monomials).  Otherwise the shift is the caller's `Mlag` (the previous evaluation's maximum at a
// nearby point); the exact maximum of this evaluation is returned in `Mlag` either way.  Any shift
// gives the same directions (row scaling), so the lag only has to keep the terms in range: the
// function returns false when the maximum moved further than the type's safe margin, and the
// caller must then discard the row and evaluate again with `exact`.
template <typename T>
struct ShiftMargin {
  static constexpr double value = sizeof(T) == 8 ? 300.0 : 40.0;
};

// Where A1 reads the point: replicated registers, or the group's LDS copy read at each use (an
// opaque zero offset, produced inside the monomial loop, keeps those reads from being hoisted
// back into registers; the FP64 tracker trades LDS reads for the registers).
template <int N>
struct PointRegs {
  const double (&zr)[N];
  const double (&zi)[N];
  __device__ __forceinline__ int fresh() const { return 0; }
  __device__ __forceinline__ Cx<double> at(int j, int) const { return {zr[j], zi[j]}; }
};
struct PointLds {
  const Cx<double> *z;
  __device__ __forceinline__ int fresh() const {
    int zero;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
    return zero;
  }
  __device__ __forceinline__ Cx<double> at(int j, int off) const { return z[off + j]; }
};

template <int N, typename T, class Pt, class Coef = CoefConst>
__device__ __forceinline__ bool eval_row_at(const SysLds<N> &S, int r, const Pt &pt, double s,
                                            Cx<T> (&row)[N + 2], double &logM, T &absum,
                                            double &Mlag, bool exact, Coef kc = Coef{},
                                            const F32Tables<N> *ft = nullptr) {
  constexpr int LD = TableLD<N>::value;
#pragma unroll
  for (int j = 0; j < N + 2; ++j) row[j] = {T(0), T(0)};
  absum = T(0);
  logM = 0.0;
  if (r >= S.n) {  // padding lane: identity row for unknown r
#pragma unroll
    for (int j = 0; j < N; ++j)
      if (j == r) row[j].x = T(1);
    absum = T(1);
    return true;
  }
  const int n = S.n, mr = S.mk[r];
  double M = Mlag;
  if (exact) {  // pass 1: row maximum of Re u
    M = -INFINITY;
#pragma unroll 1
    for (int i = 0; i < mr; ++i) {
      const double *t = S.T + (i * n + r) * LD;
      const int off = pt.fresh();
      double e = t[N] * s;
#pragma unroll
      for (int j = 0; j < N; ++j) e = fma(t[j], pt.at(j, off).x, e);
      M = fmax(M, e);
    }
  }
  logM = M;
  double Mnew = -INFINITY;
  // pass 2: shifted exponentials and the contraction with [a | w | 1]
#pragma unroll 1
  for (int i = 0; i < mr; ++i) {
    const double *t = S.T + (i * n + r) * LD;
    const int off = pt.fresh();
    double re = t[N] * s, im = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const Cx<double> zj = pt.at(j, off);
      re = fma(t[j], zj.x, re);
      im = fma(t[j], zj.y, im);
    }
    Mnew = re > Mnew ? re : Mnew;  // (ignores a NaN like fmax, without its canonicalisation)
    double turns = im * kInv2Pi;
    turns -= rint(turns);  // phase in turns, [-1/2, 1/2]
    const Cx<double> cc = S.C[i * n + r];
    Cx<T> v;
    T mag;
    if constexpr (sizeof(T) == 8) {
      const auto kci = kc.at(off);
      mag = exp_eval(re - M, kci);
      double sn, cs;
      sincos_turns(turns, sn, cs, kci);
      v.x = mag * (cc.x * cs - cc.y * sn);
      v.y = mag * (cc.x * sn + cc.y * cs);
      absum += mag * S.Cabs[i * n + r];
    } else {
      mag = __builtin_amdgcn_exp2f((float)((re - M) * kLog2e));
      const float tf = (float)turns;
      const float sn = __builtin_amdgcn_sinf(tf), cs = __builtin_amdgcn_cosf(tf);
      if (ft) {  // FP32 tables: no conversions
        const float4 cw = ft->Cf[i * n + r];
        v.x = mag * (cw.x * cs - cw.y * sn);
        v.y = mag * (cw.x * sn + cw.y * cs);
        absum += mag * cw.z;
      } else {
        const float cx = (float)cc.x, cy = (float)cc.y;
        v.x = mag * (cx * cs - cy * sn);
        v.y = mag * (cx * sn + cy * cs);
        absum += mag * (float)S.Cabs[i * n + r];
      }
    }
    if (sizeof(T) == 4 && ft) {
      const half4_t *th = ft->Th + (i * n + r) * (H16<N>::value / 4);
#pragma unroll
      for (int q = 0; q < H16<N>::value / 4; ++q) {
        const half4_t a4 = th[q];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = 4 * q + e;
          if (j < N) {
            row[j].x = fmaf((float)a4[e], (float)v.x, (float)row[j].x);
            row[j].y = fmaf((float)a4[e], (float)v.y, (float)row[j].y);
          }
        }
      }
      const float wv = ft->Cf[i * n + r].w;
      row[N].x = fma((T)wv, v.x, row[N].x);
      row[N].y = fma((T)wv, v.y, row[N].y);
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const T a = (T)t[j];
        row[j].x = fma(a, v.x, row[j].x);
        row[j].y = fma(a, v.y, row[j].y);
      }
      const T wv = (T)t[N];
      row[N].x = fma(wv, v.x, row[N].x);
      row[N].y = fma(wv, v.y, row[N].y);
    }
    row[N + 1].x += v.x;
    row[N + 1].y += v.y;
  }
  Mlag = Mnew;
  // an exact shift is always accepted (also when NaN inputs make every sum NaN), so a caller that
  // retries with `exact` cannot loop
  const double d = Mnew - M;
  return exact || (d <= ShiftMargin<T>::value && d >= -ShiftMargin<T>::value);
}

template <int N, typename T>
__device__ __forceinline__ bool eval_row(const SysLds<N> &S, int r, const double (&zr)[N],
                                         const double (&zi)[N], double s, Cx<T> (&row)[N + 2],
                                         double &logM, T &absum, double &Mlag, bool exact,
                                         const F32Tables<N> *ft = nullptr) {
  return eval_row_at<N, T>(S, r, PointRegs<N>{zr, zi}, s, row, logM, absum, Mlag, exact,
                           CoefConst{}, ft);
}

// One evaluation with the exact row maximum as the shift.
template <int N, typename T>
__device__ __forceinline__ void eval_row_exact(const SysLds<N> &S, int r, const double (&zr)[N],
                                               const double (&zi)[N], double s,
                                               Cx<T> (&row)[N + 2], double &logM, T &absum) {
  double Ml = 0.0;
  eval_row<N, T>(S, r, zr, zi, s, row, logM, absum, Ml, true);
}

// ------------------------------------------------------------------------------------------
// A5: LU with partial pivoting across the group, two right-hand sides
// ------------------------------------------------------------------------------------------
// On return myE / myN hold entry r of dE = -J^{-1} H_s and dN = -J^{-1} H, nrmE / nrmN the
// max-modulus norms of dE and dN over the true unknowns (identical in every lane; NaN
// propagates), ratio = min|pivot| / max|pivot| over the true columns.  Returns true when a
// pivot is zero or not finite.  Every lane of the wave must call this (it shuffles).
//
// Elimination: column j's pivot row is found with a packed-key max over the rows not used yet,
// broadcast entry by entry, and every other unused row subtracts its multiple of it.  Such a row
// also clears its own entry j (it is zero in exact arithmetic), so in the back substitution every
// row can apply x_j without a mask: rows pivoted after column j hold zeros there, and the rows
// that consume x_j are exactly the ones pivoted before it.
template <int N, typename T>
__device__ __forceinline__ bool lu_solve2(Cx<T> (&row)[N + 2], int r, int base, int n, Cx<T> &myE,
                                          Cx<T> &myN, double &nrmE, double &nrmN, T &ratio) {
  bool used = false;
  Cx<T> ninv_mine = {T(0), T(0)};  // minus the inverse of this row's pivot
  int pl[N];
  T pmin2 = T(INFINITY), pmax2 = T(0);
  bool sing = false;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const T mine = row[j].x * row[j].x + row[j].y * row[j].y;
    uint32_t key = used ? 0u : pivot_key(mine, r);
    key = group_max_u32<N>(key, r, base);
    const int idx = 63 - (int)(key & 63u);
    pl[j] = idx;
    const int src = base + idx;
    const Cx<T> pv = shfl_cx(row[j], src);
    const T mag = pv.x * pv.x + pv.y * pv.y;
    sing |= !(mag > T(0) && mag < T(INFINITY));
    if (j < n) {
      if constexpr (sizeof(T) == 4) {  // non-negative (NaN is caught by `sing`): integer order
        pmin2 = __uint_as_float(min(__float_as_uint(pmin2), __float_as_uint(mag)));
        pmax2 = __uint_as_float(max(__float_as_uint(pmax2), __float_as_uint(mag)));
      } else {
        pmin2 = fmin(pmin2, mag);
        pmax2 = fmax(pmax2, mag);
      }
    }
    const T nid = -fast_rcp(mag);
    const Cx<T> ninv = {pv.x * nid, -(pv.y * nid)};  // -1 / pivot
    const bool me = (r == idx);
    const bool elim = !used && !me;
    Cx<T> l = {T(0), T(0)};  // minus the multiplier
    if (elim) {
      l = cmul(row[j], ninv);
      row[j] = {T(0), T(0)};
    }
    if (me) {
      used = true;
      ninv_mine = ninv;
    }
#pragma unroll
    for (int col = j + 1; col < N + 2; ++col) {
      const Cx<T> pc = shfl_cx(row[col], src);
      row[col] = cfma(row[col], l, pc);
    }
  }
  // back substitution, column oriented: at step j the pivot row of column j has its final
  // right-hand sides and broadcasts the two unknowns, negated (which is what dE and dN hold)
  myE = {T(0), T(0)};
  myN = {T(0), T(0)};
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    const int src = base + pl[j];
    const Cx<T> e = cmul(row[N], ninv_mine), q = cmul(row[N + 1], ninv_mine);
    const Cx<T> xe = shfl_cx(e, src), xq = shfl_cx(q, src);
    row[N] = cfma(row[N], row[j], xe);
    row[N + 1] = cfma(row[N + 1], row[j], xq);
    // lane j keeps unknown j: selects, not a branch (a branch per column costs more than the
    // four selects in exec-mask bookkeeping)
    const bool mine = r == j;
    myE.x = mine ? xe.x : myE.x;
    myE.y = mine ? xe.y : myE.y;
    myN.x = mine ? xq.x : myN.x;
    myN.y = mine ? xq.y : myN.y;
  }
  // norms over the true unknowns: squared moduli, a group maximum, one square root
  const T ae = r < n ? myE.x * myE.x + myE.y * myE.y : T(0);
  const T aq = r < n ? myN.x * myN.x + myN.y * myN.y : T(0);
  if constexpr (sizeof(T) == 8) {
    nrmE = sqrt(group_max<N, double>(ae, r, base));
    nrmN = sqrt(group_max<N, double>(aq, r, base));
  } else {
    nrmE = (double)sqrtf(group_max_nonneg<N>(ae, r, base));
    nrmN = (double)sqrtf(group_max_nonneg<N>(aq, r, base));
  }
  ratio = sqrt(pmin2 / pmax2);
  return sing;
}

// Value of a replicated register array at a runtime index (select chain, no scratch).
template <int N>
__device__ __forceinline__ double pick(const double (&a)[N], int r) {
  double v = a[0];
#pragma unroll
  for (int j = 1; j < N; ++j) v = (j == r) ? a[j] : v;
  return v;
}

}  // namespace hom
