// Start points of polyhedral homotopy (Sec. 2): every root of the binomial start system
// x^{d_k} = beta_k of each mixed cell, planned and written on the GPU.
//
// In log coordinates D z = log(beta) + 2 pi i k (k integer).  With the Smith form U D V = S =
// diag(sigma_0 | sigma_1 | ...), U and V unimodular, the |det D| = prod sigma_l roots are
//     z = z_base + 2 pi i sum_l V[:, l] j_l / sigma_l,   0 <= j_l < sigma_l,
// z_base = D^{-1} log(beta) (principal logarithm).  Only the fractional part of the second term
// matters, so V is needed modulo the largest factor L = sigma_{n-1} (every sigma_l divides L):
// column l contributes ((V_il mod sigma_l) * (L / sigma_l) * j_l mod L) / L.
//
// k_start_plan, one wave per cell, its matrices in LDS: the Smith form by elementary operations
// on int64 with overflow checks, the lanes splitting each row and column operation, run twice
// (the second run repeats the first one's operations and carries V modulo the L the first run
// found), and z_base by an FP64 LU solve; it writes the cell's record.
// k_binomial_starts, one thread per root: the root's coordinates from its cell's record, staged
// through LDS so that the launch streams its output to HBM in contiguous pieces; for few roots,
// k_binomial_starts_coord, one thread per coordinate, with the same arithmetic.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "hom_internal.h"
#include "hom_intdiv.h"

namespace hom {

namespace {

// outcome of one cell's plan
enum : int32_t { kPlanOk = 0, kPlanSingular = 1, kPlanOverflow = 2, kPlanTooMany = 3,
                 kPlanBigFactor = 4, kPlanBadBeta = 5 };
// elimination rounds allowed per pivot position: each round either finishes the position or
// strictly lowers the smallest nonzero |entry| of the trailing block, so a round count beyond
// this means overflow-sized entries, which are refused
constexpr int kSmithRounds = 4096;

__device__ __forceinline__ bool fma_ok(int64_t &dst, int64_t f, int64_t src) {  // dst += f * src
  int64_t p, r;
  if (__builtin_mul_overflow(f, src, &p) || __builtin_add_overflow(dst, p, &r)) return false;
  dst = r;
  return true;
}
__device__ __forceinline__ int64_t mod_pos(int64_t v, int64_t m) {
  const int64_t r = v % m;
  return r < 0 ? r + m : r;
}

// Per-wave helpers of the plan: the block is one wave, so __syncthreads is the wave's barrier
// (and memory fence) and every value that steers control flow below is wave-uniform.
constexpr int kPlanMaxN = 32;

// lexicographic minimum of (key, idx) over the wave, in every lane
__device__ __forceinline__ void wave_min2(unsigned long long &key, int &idx) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const unsigned long long ok = __shfl_xor(key, off);
    const int oi = __shfl_xor(idx, off);
    if (ok < key || (ok == key && oi < idx)) {
      key = ok;
      idx = oi;
    }
  }
}
__device__ __forceinline__ unsigned long long uabs64(int64_t v) {
  return v < 0 ? 0ull - (unsigned long long)v : (unsigned long long)v;
}

// Smith form of the n x n matrix M (row-major, int64, in LDS, destroyed), one wave: the
// invariant factors in sig[0..n).  With V (n x n int32 in LDS), V is carried modulo L (column
// operations only; entries in [0, L), L < 2^31).  Per pivot position t: move the smallest nonzero
// |entry| of the trailing block (the first in row order among equals) to (t, t); reduce the
// entries below it and right of it by their quotients; repeat until both are zero, then, if the
// pivot does not divide the whole trailing block, add the first row holding a non-multiple to
// row t and repeat.  The lanes split each row or column operation; q is n words of scratch.
__device__ int32_t smith_wave(int n, int64_t *M, int32_t *V, int64_t L, int64_t *q, int64_t *sig,
                              int lane) {
  if (V)
    for (int e = lane; e < n * n; e += 64) V[e] = (e / n == e % n) ? 1 : 0;
  __syncthreads();
  for (int t = 0; t < n; ++t) {
    const int w = n - t;  // trailing block: rows and columns t..n-1
    for (int round = 0;; ++round) {
      if (round >= kSmithRounds) return kPlanOverflow;
      unsigned long long key = ~0ull;
      int idx = INT_MAX;
      for (int e = lane; e < w * w; e += 64) {
        const int lin = (t + e / w) * n + t + e % w;  // row-major: increasing in row order
        const int64_t v = M[lin];
        if (v != 0 && uabs64(v) < key) {
          key = uabs64(v);
          idx = lin;
        }
      }
      wave_min2(key, idx);
      if (key == ~0ull) return kPlanSingular;
      const int bi = idx / n, bj = idx % n;
      if (bi != t && lane < n) {
        const int64_t a = M[t * n + lane];
        M[t * n + lane] = M[bi * n + lane];
        M[bi * n + lane] = a;
      }
      __syncthreads();
      if (bj != t && lane < n) {
        const int64_t a = M[lane * n + t];
        M[lane * n + t] = M[lane * n + bj];
        M[lane * n + bj] = a;
        if (V) {
          const int32_t b = V[lane * n + t];
          V[lane * n + t] = V[lane * n + bj];
          V[lane * n + bj] = b;
        }
      }
      __syncthreads();
      const int64_t p = M[t * n + t];
      const bool unit = p == 1 || p == -1;  // the common case: quotients without a division
      // rows below: row i -= q_i row t
      if (lane > t && lane < n) q[lane] = unit ? M[lane * n + t] * p : M[lane * n + t] / p;
      __syncthreads();
      bool ok = true;
      for (int e = lane; e < (w - 1) * n; e += 64) {
        const int i = t + 1 + e / n, j = e % n;
        if (q[i] != 0) ok = ok && fma_ok(M[i * n + j], -q[i], M[t * n + j]);
      }
      if (__syncthreads_or(!ok)) return kPlanOverflow;
      // columns right: col j -= q_j col t, and in V modulo L
      if (lane > t && lane < n) q[lane] = unit ? M[t * n + lane] * p : M[t * n + lane] / p;
      __syncthreads();
      for (int e = lane; e < (w - 1) * n; e += 64) {
        const int j = t + 1 + e / n, i = e % n;
        const int64_t qj = q[j];
        if (qj != 0) {
          ok = ok && fma_ok(M[i * n + j], -qj, M[i * n + t]);
          if (V)
            V[i * n + j] = (int32_t)(((int64_t)V[i * n + j] + mod_pos(-qj, L) * V[i * n + t]) % L);
        }
      }
      if (__syncthreads_or(!ok)) return kPlanOverflow;
      const bool rest = lane > t && lane < n && (M[lane * n + t] != 0 || M[t * n + lane] != 0);
      if (__syncthreads_or(rest)) continue;
      if (unit) break;  // a unit divides the whole trailing block
      int bad = INT_MAX;  // first row of the trailing block with an entry p does not divide
      for (int e = lane; e < (w - 1) * (w - 1); e += 64) {
        const int i = t + 1 + e / (w - 1), j = t + 1 + e % (w - 1);
        if (M[i * n + j] % p != 0 && i < bad) bad = i;
      }
      unsigned long long bk = (unsigned long long)bad;
      wave_min2(bk, bad);
      if (bad == INT_MAX) break;
      if (lane < n) ok = fma_ok(M[t * n + lane], 1, M[bad * n + lane]);  // row t += row bad
      if (__syncthreads_or(!ok)) return kPlanOverflow;
    }
    if (lane == 0) sig[t] = (int64_t)uabs64(M[t * n + t]);  // (a sign is a row operation: U only)
  }
  __syncthreads();
  return kPlanOk;
}

// x = D^{-1} b for the complex right-hand side (br, bi) in place, one wave: FP64 LU with partial
// pivoting (the largest |entry| of the column, the first among equals) on A (n x n in LDS), then
// back substitution by columns; f is n doubles of scratch.  False if D is singular.
__device__ bool solve_wave(int n, const int32_t *D, double *A, double *br, double *bi, double *f,
                           int lane) {
  for (int e = lane; e < n * n; e += 64) A[e] = (double)D[e];
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    // magnitudes are >= 0, so their bit patterns order like the values; complemented for a min
    unsigned long long key = ~0ull;
    int idx = INT_MAX;
    if (lane >= j && lane < n) {
      key = ~(unsigned long long)__double_as_longlong(fabs(A[lane * n + j]));
      idx = lane;
    }
    wave_min2(key, idx);
    if (key == ~0ull) return false;  // the whole column is zero
    if (idx != j) {
      if (lane < n) {
        const double a = A[j * n + lane];
        A[j * n + lane] = A[idx * n + lane];
        A[idx * n + lane] = a;
      }
      if (lane == 0) {
        double a = br[j];
        br[j] = br[idx];
        br[idx] = a;
        a = bi[j];
        bi[j] = bi[idx];
        bi[idx] = a;
      }
    }
    __syncthreads();
    if (lane > j && lane < n) f[lane] = A[lane * n + j] / A[j * n + j];
    __syncthreads();
    const int w = n - j;
    for (int e = lane; e < (w - 1) * w; e += 64) {
      const int i = j + 1 + e / w, k = j + e % w;
      A[i * n + k] -= f[i] * A[j * n + k];
    }
    if (lane > j && lane < n) {
      br[lane] -= f[lane] * br[j];
      bi[lane] -= f[lane] * bi[j];
    }
    __syncthreads();
  }
  for (int i = n - 1; i >= 0; --i) {
    const double d = A[i * n + i], xr = br[i] / d, xi = bi[i] / d;
    __syncthreads();
    if (lane < i) {
      br[lane] -= A[lane * n + i] * xr;
      bi[lane] -= A[lane * n + i] * xi;
    } else if (lane == i) {
      br[i] = xr;
      bi[i] = xi;
    }
    __syncthreads();
  }
  return true;
}

// One wave (block) per cell, grid-stride: status[c], det[c] and the record
// (start_record_words(n) int64 words): [0] L, [1] the number of invariant factors above one,
// then z_base (2n doubles), their radices, then their V columns (n each).  The Smith form runs
// twice: the first run finds the factors and L, the second repeats its operations (the same
// matrix, so the same choices) and carries V modulo L.
__global__ void __launch_bounds__(64)
    k_start_plan(int n, int64_t num_cells, const int32_t *__restrict__ Dall,
                 const double *__restrict__ beta_all, int64_t *__restrict__ rec_all,
                 int32_t *__restrict__ status, int64_t *__restrict__ det_out) {
  __shared__ int64_t sM[kPlanMaxN * kPlanMaxN];  // the Smith forms, then the LU (as doubles)
  __shared__ int32_t sV[kPlanMaxN * kPlanMaxN];
  __shared__ int64_t sQ[kPlanMaxN], sSig[kPlanMaxN];
  __shared__ double sB[2 * kPlanMaxN];
  const int lane = threadIdx.x;
  double *sA = reinterpret_cast<double *>(sM), *sF = reinterpret_cast<double *>(sQ);
  for (int64_t c = blockIdx.x; c < num_cells; c += gridDim.x) {
    const int32_t *D = Dall + c * n * n;
    int64_t *rec = rec_all + c * start_record_words(n);
    bool bad_beta = false;
    if (lane < n) {
      const double r = beta_all[(c * n + lane) * 2], im = beta_all[(c * n + lane) * 2 + 1];
      bad_beta = !isfinite(r) || !isfinite(im) || (r == 0.0 && im == 0.0);
      sB[lane] = log(hypot(r, im));
      sB[kPlanMaxN + lane] = atan2(im, r);
    }
    for (int e = lane; e < n * n; e += 64) sM[e] = D[e];
    int32_t st = __syncthreads_or(bad_beta) ? kPlanBadBeta : kPlanOk;
    if (st == kPlanOk) st = smith_wave(n, sM, nullptr, 1, sQ, sSig, lane);
    int64_t det = 1;
    for (int l = 0; l < n && st == kPlanOk; ++l)
      if (__builtin_mul_overflow(det, sSig[l], &det) || det >= ((int64_t)1 << 62)) st = kPlanTooMany;
    const int64_t L = st == kPlanOk ? sSig[n - 1] : 1;
    if (st == kPlanOk && L >= ((int64_t)1 << 31)) st = kPlanBigFactor;
    if (st == kPlanOk && L > 1) {  // second run, V modulo L
      __syncthreads();
      for (int e = lane; e < n * n; e += 64) sM[e] = D[e];
      st = smith_wave(n, sM, sV, L, sQ, sSig, lane);
    }
    __syncthreads();
    if (st == kPlanOk && !solve_wave(n, D, sA, sB, sB + kPlanMaxN, sF, lane)) st = kPlanSingular;
    if (st == kPlanOk) {
      int nlive = 0;
      for (int l = 0; l < n; ++l) nlive += sSig[l] > 1;
      if (lane == 0) {
        rec[0] = L;
        rec[1] = nlive;
      }
      if (lane < n) {
        rec[2 + 2 * lane] = __double_as_longlong(sB[lane]);
        rec[3 + 2 * lane] = __double_as_longlong(sB[kPlanMaxN + lane]);
      }
      int64_t *rs = rec + 2 + 2 * n, *rc = rs + nlive;
      int qn = 0;
      for (int l = 0; l < n; ++l) {
        const int64_t sg = sSig[l];
        if (sg == 1) continue;
        if (lane == 0) rs[qn] = sg;
        if (lane < n) rc[qn * n + lane] = ((int64_t)sV[lane * n + l] % sg) * (L / sg) % L;
        ++qn;
      }
    }
    if (lane == 0) {
      status[c] = st;
      det_out[c] = st == kPlanOk ? det : 0;
    }
    __syncthreads();  // the next cell reuses the LDS arrays
  }
}

// The fractional part (times L) of coordinate i of root index q of a cell: the mixed-radix
// digits of q over the cell's factors above one (first fastest; the last digit is what remains)
// times the V columns, mod L.
__device__ __forceinline__ int64_t root_num(int64_t q, int nlive, const int64_t *rs,
                                            const int64_t *rc, int n, int i, int64_t L,
                                            double inv_L) {
  int64_t acc = 0;
  for (int l = 0; l < nlive; ++l) {
    int64_t j = q;
    if (l + 1 < nlive) {
      const int64_t sg = rs[l];
      q = divmod62(q, sg, 1.0 / (double)sg, j);
    }
    int64_t t;  // j < sigma_l <= L and the column entry < L: the product is below 2^62
    divmod62(j * rc[(int64_t)l * n + i], L, inv_L, t);
    acc += t;
    if (acc >= L) acc -= L;
  }
  return acc;
}

// Im z of a coordinate: its base value plus 2 pi num / L, reduced into [-pi, pi)
__device__ __forceinline__ double root_im(double zi0, int64_t num, double inv_L) {
  const double two_pi = 6.283185307179586476925286766559;
  const double pi = 3.14159265358979323846264338327950;
  double im = zi0 + two_pi * ((double)num * inv_L) + pi;
  im -= two_pi * floor(im / two_pi);
  im -= pi;
  if (im >= pi) im -= two_pi;  // rounding at the top edge
  return im;
}

// Few roots (many small cells): one thread per (root, coordinate), so that the launch has enough
// threads; the same arithmetic as the kernel below, so the same results.
__global__ void __launch_bounds__(256)
    k_binomial_starts_coord(int n, int num_cells, const StartHdr *__restrict__ hdr,
                            const int64_t *__restrict__ rec_all, int64_t rows,
                            double *__restrict__ z) {
  const int64_t total = rows * n;
  const double inv_n = 1.0 / (double)n;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    int64_t ii;
    const int64_t row = divmod62(g, n, inv_n, ii);
    const int i = (int)ii;
    int lo = 0, hi = num_cells - 1;  // last cell with row0 <= row
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (hdr[mid].row0 <= row) lo = mid;
      else hi = mid - 1;
    }
    const StartHdr h = hdr[lo];
    const int64_t *d = rec_all + (int64_t)lo * start_record_words(n);
    const int64_t L = d[0];
    const int nlive = (int)d[1];
    const int64_t *rs = d + 2 + 2 * n, *rc = rs + nlive;
    const double inv_L = 1.0 / (double)L;
    const int64_t num = root_num(h.first + (row - h.row0), nlive, rs, rc, n, i, L, inv_L);
    reinterpret_cast<double2 *>(z)[g] =
        double2{__longlong_as_double(d[2 + 2 * i]),
                root_im(__longlong_as_double(d[3 + 2 * i]), num, inv_L)};
  }
}

// One thread per root row, 64 rows per block (one wave) per tile, grid-stride over tiles: the
// cell by binary search over the rows' starts (skipped while the row stays in the previous row's
// cell), the root index's mixed-radix digits over the cell's invariant factors above one (first
// fastest; the last digit is what remains), each coordinate's fractional part
// num_i = sum_l j_l cm[l][i] mod L, the imaginary part reduced into [-pi, pi).  In a cell with one
// factor above one (j = the root index itself), the next row of a thread is gridDim * 64 roots
// further, so num_i grows by a fixed increment mod L: one addition per coordinate instead of a
// product.  The rows go through LDS and leave in contiguous 16-byte pieces.  KN >= n.
constexpr int kStartTile = 64;
template <int KN>
__global__ void __launch_bounds__(kStartTile)
    k_binomial_starts(int n, int num_cells, const StartHdr *__restrict__ hdr,
                      const int64_t *__restrict__ rec_all, int64_t rows, double *__restrict__ z) {
  __shared__ double2 stage[kStartTile * KN];
  const int t = threadIdx.x;
  const int64_t tiles = (rows + kStartTile - 1) / kStartTile;
  const int64_t stride = (int64_t)gridDim.x * kStartTile;  // rows between a thread's rows
  int cur = -1;         // cell of this thread's previous row
  int64_t prev_q = -1;  // its root index
  int64_t num[KN], inc[KN];
#pragma unroll
  for (int i = 0; i < KN; ++i) num[i] = inc[i] = 0;
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t row = tile * kStartTile + t;
    if (row < rows) {
      int lo;
      if (cur >= 0 && row >= hdr[cur].row0 && (cur + 1 == num_cells || row < hdr[cur + 1].row0)) {
        lo = cur;
      } else {  // last cell with row0 <= row
        int a = 0, b2 = num_cells - 1;
        while (a < b2) {
          const int mid = (a + b2 + 1) >> 1;
          if (hdr[mid].row0 <= row) a = mid;
          else b2 = mid - 1;
        }
        lo = a;
      }
      const StartHdr h = hdr[lo];
      const int64_t *d = rec_all + (int64_t)lo * start_record_words(n);
      const int64_t L = d[0];
      const int nlive = (int)d[1];
      const int64_t *rs = d + 2 + 2 * n, *rc = rs + nlive;
      const double inv_L = 1.0 / (double)L;
      const int64_t q = h.first + (row - h.row0);
      if (nlive == 1 && lo == cur && q - prev_q == stride) {  // the increment, mod L
#pragma unroll
        for (int i = 0; i < KN; ++i) {
          if (i < n) {
            num[i] += inc[i];
            if (num[i] >= L) num[i] -= L;
          }
        }
      } else if (nlive == 1) {  // j = q < L; the products and, for the next rows, the increments
        int64_t sL;
        divmod62(stride, L, inv_L, sL);
#pragma unroll
        for (int i = 0; i < KN; ++i) {
          if (i < n) {
            int64_t tq;  // q and the column entry are below L < 2^31: the products below 2^62
            divmod62(q * rc[i], L, inv_L, tq);
            num[i] = tq;
            divmod62(sL * rc[i], L, inv_L, tq);
            inc[i] = tq;
          }
        }
      } else {  // several factors: every digit, every product
#pragma unroll
        for (int i = 0; i < KN; ++i)
          if (i < n) num[i] = root_num(q, nlive, rs, rc, n, i, L, inv_L);
      }
      cur = lo;
      prev_q = q;
#pragma unroll
      for (int i = 0; i < KN; ++i)
        if (i < n)
          stage[t * n + i] = double2{__longlong_as_double(d[2 + 2 * i]),
                                     root_im(__longlong_as_double(d[3 + 2 * i]), num[i], inv_L)};
    }
    __syncthreads();
    const int64_t r0 = tile * kStartTile;
    const int nrow = rows - r0 < kStartTile ? (int)(rows - r0) : kStartTile;
    double2 *out = reinterpret_cast<double2 *>(z) + r0 * n;
    for (int k = t; k < nrow * n; k += kStartTile) out[k] = stage[k];
    __syncthreads();  // the stage is read before the next tile writes it
  }
}

}  // namespace

const char *start_status_text(int32_t st) {
  switch (st) {
    case kPlanOk: return "";
    case kPlanSingular: return "D is singular (det 0)";
    case kPlanOverflow: return "an entry of the Smith form exceeds the int64 range";
    case kPlanTooMany: return "|det D| >= 2^62 roots";
    case kPlanBigFactor: return "the largest invariant factor of D is >= 2^31";
    case kPlanBadBeta: return "beta must be finite and nonzero";
    default: return "unknown plan status";
  }
}
int start_status_code(int32_t st) {
  return (st == kPlanOverflow || st == kPlanTooMany || st == kPlanBigFactor) ? HOM_EUNSUPPORTED
                                                                             : HOM_EINVAL;
}

hipError_t launch_start_plan(int n, int64_t num_cells, const int32_t *D, const double *beta,
                             int64_t *rec, int32_t *status, int64_t *det, hipStream_t stream) {
  if (n < 1 || n > kPlanMaxN) return hipErrorInvalidValue;
  prof_begin(stream);
  int64_t blocks = num_cells;
  const int64_t cap = (int64_t)num_cus() * 16;
  if (blocks > cap) blocks = cap;
  hipLaunchKernelGGL(k_start_plan, dim3((unsigned)blocks), dim3(64), 0, stream, n, num_cells, D,
                     beta, rec, status, det);
  prof_end(stream, "k_start_plan");
  return hipGetLastError();
}

hipError_t launch_binomial_starts(int n, int num_cells, const StartHdr *hdr, const int64_t *rec,
                                  int64_t rows, double *z, hipStream_t stream) {
  prof_begin(stream);
  if (rows * n <= ((int64_t)1 << 20)) {  // few roots: a thread per coordinate fills the GPU better
    int64_t blocks = (rows * n + 255) / 256;
    const int64_t cap = (int64_t)num_cus() * 16;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_binomial_starts_coord, dim3((unsigned)blocks), dim3(256), 0, stream, n,
                       num_cells, hdr, rec, rows, z);
    prof_end(stream, "k_binomial_starts");
    return hipGetLastError();
  }
  const int64_t tiles = (rows + kStartTile - 1) / kStartTile;
  int64_t blocks = tiles;
  const int64_t cap = (int64_t)num_cus() * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  const dim3 grid((unsigned)blocks), block(kStartTile);
  if (n <= 8)
    hipLaunchKernelGGL(k_binomial_starts<8>, grid, block, 0, stream, n, num_cells, hdr, rec, rows, z);
  else if (n <= 16)
    hipLaunchKernelGGL(k_binomial_starts<16>, grid, block, 0, stream, n, num_cells, hdr, rec, rows, z);
  else
    hipLaunchKernelGGL(k_binomial_starts<32>, grid, block, 0, stream, n, num_cells, hdr, rec, rows, z);
  prof_end(stream, "k_binomial_starts");
  return hipGetLastError();
}

}  // namespace hom
