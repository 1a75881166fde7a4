// Projective step (Sec. 2.2, eq. (3)-(5); Sec. 6; Sec. 7, Alg. 2 and Alg. 3): the Euler and
// Newton directions in homogeneous coordinates y in C^{n+1}, from the null space of the unified
// system
//   J = [ dH~/dy  dH~/ds  H~ ]      (n + 1) x (n + 3),
//       [  y^*      0      0 ]
// whose null space is spanned by (dE, 1, 0) and (dN, 0, 1).
//
// One group of N lanes per point, N a power of two with N >= n + 3.  Lane k < n evaluates row k of
// the homogenised system in log coordinates z = log y (A1-A3 of the affine evaluation, with the
// homogenising exponent as the (n+1)-th coordinate), then the y-coordinate epilogue of Alg. 2
// (column j times e^{-z_j} = 1 / y_j); lane n holds the row y^*; the other lanes carry identity
// rows of padding unknowns (they leave the null space unchanged: it gains zero entries there).
//
// The null space comes from Householder reflections (the QR decomposition of J^T of Sec. 6,
// written as an LQ decomposition of J): for i = 0..n, the reflector of row i's trailing entries
// (columns i..) zeroes them past the diagonal; every lower row applies it.  The reflectors go to
// LDS, and the two null vectors Q e_{N} and Q e_{N+1} (Q the product of the reflectors) are
// formed by applying them in reverse order to the two unit vectors, held one entry per lane.
// The row reduction of Alg. 3 (the rightmost 2 x 2 block of the two vectors made the identity)
// then gives dE and dN.
#include <stdio.h>

#include "hom_internal.h"

namespace hom {

// Four waves per block up to 16-lane groups (the tables are shared by more waves); two for 32.
template <int N>
__host__ __device__ constexpr int proj_block() {
  return N <= 16 ? 256 : 128;
}

// Columns kept per row: the n + 1 unknowns and the s and H columns (the padding unknowns' columns
// are zero in every real row), compressed as k <= n -> column k, k = n+1 -> column N (d/ds),
// k = n+2 -> column N+1 (H).
template <int N>
__host__ __device__ constexpr size_t proj_group_bytes(int n) {
  return (size_t)N * 16                        /* z_j, then 1/y_j (two passes over the same slots) */
         + (size_t)N * 16                      /* y_j */
         + (size_t)(n + 1) * (n + 3) * 16      /* reflectors W[i][k], i <= n, k <= n + 2 */
         + ((size_t)(n + 2) * 8 + 15) / 16 * 16;  /* beta_i, then |L_ii|; 16-byte multiple */
}

// v from another lane of the same row of 16 by a DPP pattern (two 32-bit moves, no LDS)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// sum over an aligned group of N lanes (N a power of two), the same value in every lane: pairs
// within quads (lane ^ 1, lane ^ 2), then quads mirrored within 8 lanes, then halves mirrored
// within 16 (DPP), then the two rows of 16 of a 32-lane group (a shuffle).  Each step adds two
// partial sums that are equal in both lanes of a pair, so every lane rounds identically.
template <int N>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (N >= 2) v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (N >= 4) v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (N >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror
  if constexpr (N >= 16) v += dpp_f64<0x140>(v); // row_mirror
  if constexpr (N >= 32) v += __shfl_xor(v, 16, 64);
  static_assert(N <= 32, "groups of at most 32 lanes");
  return v;
}

__device__ __forceinline__ Cx<double> cconj(Cx<double> a) { return {a.x, -a.y}; }

// Up to 16-lane groups the registers are bounded for two waves per SIMD (a few spill; measured
// faster than one wave without spills).
template <int N, bool GT>
__global__ void __launch_bounds__(proj_block<N>()) __attribute__((amdgpu_waves_per_eu(N <= 16 ? 2 : 1)))
    k_step_proj(SysDev sd, const double *__restrict__ c, int64_t P, const double *__restrict__ y,
                const double *__restrict__ s, double *__restrict__ dE, double *__restrict__ dN,
                int32_t *__restrict__ status, size_t table_bytes) {
  static_assert((N & (N - 1)) == 0, "projective groups are powers of two");
  extern __shared__ __align__(16) char smem[];
  const SysLds<N> S = stage_tables<N, GT>(smem, sd, c);
  const Geo<N> geo;
  const int n = sd.n, nu = n + 1, r = geo.r;
  char *gb = smem + table_bytes +
             ((threadIdx.x >> 6) * Geo<N>::G + (geo.valid ? geo.g : 0)) * proj_group_bytes<N>(n);
  Cx<double> *sZ = reinterpret_cast<Cx<double> *>(gb);
  Cx<double> *sY = sZ + N;
  const int ldw = n + 3;     // compressed columns of a reflector
  Cx<double> *sW = sY + N;  // [n + 1][n + 3]
  double *sB = reinterpret_cast<double *>(sW + (n + 1) * ldw);
  const int64_t gpb = (proj_block<N>() / 64) * Geo<N>::G;
  const int64_t stride = (int64_t)gridDim.x * gpb;
  const int64_t p0 = (int64_t)blockIdx.x * gpb + (threadIdx.x >> 6) * Geo<N>::G + geo.g;
  // this lane's compressed column: k <= n unknowns, n+1 the s column, n+2 the H column
  const int kcol = r;
  for (int64_t it = 0;; ++it) {  // wave-uniform
    const int64_t p = p0 + it * stride;
    const bool act = geo.valid && p < P;
    if (!__any(act)) break;
    // ---- coordinates: lane j <= n takes y_j, its logarithm and its inverse ----
    Cx<double> yj = {0.0, 0.0};
    if (act && r < nu) yj = {y[2 * (p * nu + r)], y[2 * (p * nu + r) + 1]};
    const double a2 = yj.x * yj.x + yj.y * yj.y;
    if (geo.valid) {
      sZ[r] = r < nu ? Cx<double>{0.5 * log(a2), atan2(yj.y, yj.x)} : Cx<double>{0.0, 0.0};
      sY[r] = yj;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    double zr[N], zi[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const Cx<double> v = geo.valid ? sZ[j] : Cx<double>{0.0, 0.0};
      zr[j] = v.x;
      zi[j] = v.y;
    }
    const double sp = act ? s[p] : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // every lane has read sZ
    __builtin_amdgcn_wave_barrier();
    if (geo.valid) sZ[r] = r < nu ? Cx<double>{yj.x / a2, -yj.y / a2} : Cx<double>{0.0, 0.0};
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    // ---- A1-A3 in log coordinates, then the y-coordinate epilogue (Alg. 2) ----
    Cx<double> row[N + 2];
    double M, absum;
    eval_row_exact<N, double>(S, r, zr, zi, sp, row, M, absum);
    if (r < n) {
#pragma unroll
      for (int j = 0; j < N; ++j)
        if (j < nu) row[j] = cmul(row[j], geo.valid ? sZ[j] : Cx<double>{0.0, 0.0});
    } else if (r == n) {  // the row y^*
#pragma unroll
      for (int j = 0; j < N; ++j)
        row[j] = j < nu ? cconj(geo.valid ? sY[j] : Cx<double>{0.0, 0.0}) : Cx<double>{0.0, 0.0};
      row[N] = {0.0, 0.0};
      row[N + 1] = {0.0, 0.0};
    }
    // ---- LQ by Householder reflections, rows 0..n ----
    double lmin = INFINITY, lmax = 0.0;
#pragma unroll
    for (int i = 0; i < N - 2; ++i) {
      if (i > n) continue;  // uniform (a static trip count lets the loop unroll)
      // lane i: the reflector of its entries in columns i.. (w = conj(x) - conj(alpha) e_i)
      if (r == i && geo.valid) {
        double nrm2a = 0.0, nrm2b = 0.0;  // two partial sums: half the dependent chain
#pragma unroll
        for (int col = 0; col < N + 2; ++col) {
          if (col < i) continue;
          const double t = row[col].x * row[col].x + row[col].y * row[col].y;
          if (col & 1) nrm2b += t;
          else nrm2a += t;
        }
        const double nrm2 = nrm2a + nrm2b;
        const double nx = sqrt(nrm2);
        Cx<double> x0 = {0.0, 0.0};  // row[i] by selects: i may stay a loop counter, and a
#pragma unroll                        // runtime index would move the row to scratch memory
        for (int col = 0; col < N - 2; ++col)
          if (col == i) x0 = row[col];
        const double a0 = sqrt(x0.x * x0.x + x0.y * x0.y);
        const Cx<double> alpha = a0 > 0.0 ? Cx<double>{-x0.x / a0 * nx, -x0.y / a0 * nx}
                                          : Cx<double>{-nx, 0.0};
        const Cx<double> v0 = {x0.x - alpha.x, x0.y - alpha.y};
        const double wn2 = v0.x * v0.x + v0.y * v0.y + (nrm2 - a0 * a0);
        // compressed storage of w: k <= n, then the s and H columns
        Cx<double> *W = sW + i * ldw;
#pragma unroll
        for (int col = 0; col < N + 2; ++col) {
          if (col < i) continue;
          const int k = col < N ? col : nu + (col - N);
          if (col < N && col > n) continue;  // padding columns: zero
          W[k] = col == i ? cconj(v0) : cconj(row[col]);
        }
        sB[i] = wn2 > 0.0 ? 2.0 / wn2 : 0.0;
        sB[nu] = sqrt(alpha.x * alpha.x + alpha.y * alpha.y);  // |L_ii|, read below
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
      const double beta = geo.valid ? sB[i] : 0.0;
      const double lii = geo.valid ? sB[nu] : 0.0;
      lmin = fmin(lmin, lii);
      lmax = fmax(lmax, lii);
      if (r > i) {  // rows below apply it: row -= beta (row . w) w^H
        const Cx<double> *W = sW + i * ldw;
        Cx<double> da = {0.0, 0.0}, db = {0.0, 0.0};  // two partial sums
#pragma unroll
        for (int col = 0; col < N + 2; ++col) {
          if (col < i || (col < N && col > n)) continue;
          const int k = col < N ? col : nu + (col - N);
          const Cx<double> wk = geo.valid ? W[k] : Cx<double>{0.0, 0.0};
          if (col & 1) db = cfma(db, row[col], wk);
          else da = cfma(da, row[col], wk);
        }
        const Cx<double> f = {beta * (da.x + db.x), beta * (da.y + db.y)};
#pragma unroll
        for (int col = 0; col < N + 2; ++col) {
          if (col < i || (col < N && col > n)) continue;
          const int k = col < N ? col : nu + (col - N);
          const Cx<double> wk = geo.valid ? W[k] : Cx<double>{0.0, 0.0};
          row[col] = cfnms(row[col], f, cconj(wk));
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // sB read before it is rewritten
      __builtin_amdgcn_wave_barrier();
    }
    // ---- null vectors: Q e applied reflector by reflector, last first; lane k holds entry k ----
    Cx<double> x1 = {kcol == nu ? 1.0 : 0.0, 0.0}, x2 = {kcol == nu + 1 ? 1.0 : 0.0, 0.0};
#pragma unroll
    for (int i = N - 3; i >= 0; --i) {
      if (i > n) continue;  // uniform
      const bool mine = geo.valid && kcol <= nu + 1 && (kcol >= i || kcol > n);
      const Cx<double> wk = mine ? sW[i * ldw + kcol] : Cx<double>{0.0, 0.0};
      const double beta = geo.valid ? sB[i] : 0.0;
      // d = w^H x over the group
      const Cx<double> t1 = cmul(cconj(wk), x1), t2 = cmul(cconj(wk), x2);
      const Cx<double> d1 = {group_sum<N>(t1.x), group_sum<N>(t1.y)};
      const Cx<double> d2 = {group_sum<N>(t2.x), group_sum<N>(t2.y)};
      x1 = cfnms(x1, Cx<double>{beta * d1.x, beta * d1.y}, wk);
      x2 = cfnms(x2, Cx<double>{beta * d2.x, beta * d2.y}, wk);
    }
    // ---- row reduction: the entries of the s and H columns made the identity ----
    const int lb = geo.base;
    const Cx<double> b00 = shfl_cx(x1, lb + nu), b01 = shfl_cx(x1, lb + nu + 1);
    const Cx<double> b10 = shfl_cx(x2, lb + nu), b11 = shfl_cx(x2, lb + nu + 1);
    const Cx<double> det = cfnms(cmul(b00, b11), b01, b10);
    const double dd = det.x * det.x + det.y * det.y;
    const Cx<double> dinv = {det.x / dd, -det.y / dd};
    // B^{-1} = [[b11, -b01], [-b10, b00]] / det; (dE, 1, 0) = row 0 of B^{-1} [x1^T; x2^T]
    const Cx<double> i00 = cmul(b11, dinv), i01 = cmul(Cx<double>{-b01.x, -b01.y}, dinv);
    const Cx<double> i10 = cmul(Cx<double>{-b10.x, -b10.y}, dinv), i11 = cmul(b00, dinv);
    const Cx<double> e = cfma(cmul(i00, x1), i01, x2), q = cfma(cmul(i10, x1), i11, x2);
    const double ratio = lmin / lmax;
    const bool sing = !(ratio >= 1e-14) || !(dd > 0.0) || !(e.x - e.x == 0.0) ||
                      !(e.y - e.y == 0.0) || !(q.x - q.x == 0.0) || !(q.y - q.y == 0.0);
    const uint32_t bad = group_or_u32<N>(sing ? 1u : 0u, r, geo.base);
    if (act) {
      if (r < nu) {
        dE[2 * (p * nu + r)] = e.x;
        dE[2 * (p * nu + r) + 1] = e.y;
        dN[2 * (p * nu + r)] = q.x;
        dN[2 * (p * nu + r) + 1] = q.y;
      }
      if (r == 0) status[p] = bad ? -1 : 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // LDS reads done before the next point
    __builtin_amdgcn_wave_barrier();
  }
}

template <int N>
static hipError_t step_proj_n(const System &S, const void *cws, const double *c, int64_t P,
                              const double *y, const double *s, double *dE, double *dN,
                              int32_t *status, hipStream_t stream) {
  const size_t tb = (S.lds_bytes + 15) & ~(size_t)15;
  constexpr int block = proj_block<N>();
  const size_t lds = tb + (size_t)(block / 64) * Geo<N>::G * proj_group_bytes<N>(S.n);
  const int64_t gpb = (block / 64) * Geo<N>::G;
  const int64_t need = (P + gpb - 1) / gpb;
  const int64_t cap = (int64_t)num_cus() * 16;
  const unsigned grid = (unsigned)(need < cap ? (need > 0 ? need : 1) : cap);
  auto kern = S.global_tables ? k_step_proj<N, true> : k_step_proj<N, false>;
  char label[64];
  snprintf(label, sizeof label, "k_step_proj<%d>", N);
  prof_begin(stream);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, stream, S.dev(cws), c, P, y, s, dE,
                     dN, status, tb);
  prof_end(stream, label);
  return hipGetLastError();
}

int proj_group_size(int n) {
  const int need = n + 3;
  for (int N = 4; N <= 32; N <<= 1)
    if (N >= need) return N;
  return 0;
}

hipError_t launch_step_proj(const System &S, const void *cws, const double *c, int64_t P,
                            const double *y, const double *s, double *dE, double *dN,
                            int32_t *status, hipStream_t stream) {
  switch (S.N) {
    case 4: return step_proj_n<4>(S, cws, c, P, y, s, dE, dN, status, stream);
    case 8: return step_proj_n<8>(S, cws, c, P, y, s, dE, dN, status, stream);
    case 16: return step_proj_n<16>(S, cws, c, P, y, s, dE, dN, status, stream);
    case 32: return step_proj_n<32>(S, cws, c, P, y, s, dE, dN, status, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hom
