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
// k_start_plan, one thread per cell: the Smith form by elementary operations on int64 with
// overflow checks, run twice (the second run repeats the first one's operations and carries V
// modulo the L the first run found), and z_base by an FP64 LU solve; it writes the cell's record.
// k_binomial_starts, one thread per (root, coordinate): the root from its record, writing
// consecutive doubles, so the launch streams its output to HBM.
#include <hip/hip_runtime.h>

#include <cmath>

#include "hom_internal.h"

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
__device__ __forceinline__ int64_t abs64(int64_t v) { return v < 0 ? -v : v; }
__device__ __forceinline__ int64_t mod_pos(int64_t v, int64_t m) {
  const int64_t r = v % m;
  return r < 0 ? r + m : r;
}

// Smith form of the n x n matrix M (row-major, int64, destroyed): the invariant factors in
// sig[0..n).  With V (n x n), V is carried modulo L (column operations only; entries in [0, L)).
__device__ int32_t smith64(int n, int64_t *M, int64_t *V, int64_t L, int64_t *sig) {
  auto at = [&](int i, int j) -> int64_t & { return M[i * n + j]; };
  if (V)
    for (int i = 0; i < n * n; ++i) V[i] = (i / n == i % n) ? mod_pos(1, L) : 0;
  for (int t = 0; t < n; ++t) {
    int round = 0;
    for (;; ++round) {
      if (round >= kSmithRounds) return kPlanOverflow;
      int bi = -1, bj = -1;  // smallest nonzero |entry| of the trailing block, first in row order
      for (int i = t; i < n; ++i)
        for (int j = t; j < n; ++j)
          if (at(i, j) != 0 && (bi < 0 || abs64(at(i, j)) < abs64(at(bi, bj)))) {
            bi = i;
            bj = j;
          }
      if (bi < 0) return kPlanSingular;
      if (bi != t)
        for (int j = 0; j < n; ++j) {
          const int64_t a = at(t, j);
          at(t, j) = at(bi, j);
          at(bi, j) = a;
        }
      if (bj != t) {
        for (int i = 0; i < n; ++i) {
          const int64_t a = at(i, t);
          at(i, t) = at(i, bj);
          at(i, bj) = a;
        }
        if (V)
          for (int i = 0; i < n; ++i) {
            const int64_t a = V[i * n + t];
            V[i * n + t] = V[i * n + bj];
            V[i * n + bj] = a;
          }
      }
      bool done = true;
      const int64_t p = at(t, t);
      for (int i = t + 1; i < n; ++i) {  // rows below: row i -= q row t
        const int64_t q = at(i, t) / p;
        if (q != 0)
          for (int j = 0; j < n; ++j)
            if (!fma_ok(at(i, j), -q, at(t, j))) return kPlanOverflow;
        if (at(i, t) != 0) done = false;
      }
      for (int j = t + 1; j < n; ++j) {  // columns right: col j -= q col t (and in V)
        const int64_t q = at(t, j) / p;
        if (q != 0) {
          for (int i = 0; i < n; ++i)
            if (!fma_ok(at(i, j), -q, at(i, t))) return kPlanOverflow;
          if (V) {
            const int64_t qm = mod_pos(-q, L);
            for (int i = 0; i < n; ++i)
              V[i * n + j] = (V[i * n + j] + qm * V[i * n + t]) % L;
          }
        }
        if (at(t, j) != 0) done = false;
      }
      if (!done) continue;
      int bad = -1;  // the pivot must divide the whole trailing block
      for (int i = t + 1; i < n && bad < 0; ++i)
        for (int j = t + 1; j < n; ++j)
          if (at(i, j) % p != 0) {
            bad = i;
            break;
          }
      if (bad < 0) break;
      for (int j = 0; j < n; ++j)  // row t += row bad
        if (!fma_ok(at(t, j), 1, at(bad, j))) return kPlanOverflow;
    }
    sig[t] = abs64(at(t, t));  // (a sign is a row operation: U only)
  }
  return kPlanOk;
}

// x = D^{-1} b for complex b (FP64 LU with partial pivoting on a copy A of D); false if singular
__device__ bool solve_complex(int n, const int32_t *D, double *A, double *br, double *bi) {
  for (int i = 0; i < n * n; ++i) A[i] = (double)D[i];
  for (int j = 0; j < n; ++j) {
    int p = j;
    for (int i = j + 1; i < n; ++i)
      if (fabs(A[i * n + j]) > fabs(A[p * n + j])) p = i;
    if (A[p * n + j] == 0.0) return false;
    if (p != j) {
      for (int k = 0; k < n; ++k) {
        const double a = A[j * n + k];
        A[j * n + k] = A[p * n + k];
        A[p * n + k] = a;
      }
      double a = br[j];
      br[j] = br[p];
      br[p] = a;
      a = bi[j];
      bi[j] = bi[p];
      bi[p] = a;
    }
    for (int i = j + 1; i < n; ++i) {
      const double f = A[i * n + j] / A[j * n + j];
      for (int k = j; k < n; ++k) A[i * n + k] -= f * A[j * n + k];
      br[i] -= f * br[j];
      bi[i] -= f * bi[j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double vr = br[i], vi = bi[i];
    for (int k = i + 1; k < n; ++k) {
      vr -= A[i * n + k] * br[k];
      vi -= A[i * n + k] * bi[k];
    }
    br[i] = vr / A[i * n + i];
    bi[i] = vi / A[i * n + i];
  }
  return true;
}

// One thread per cell of [c0, c1): status[c], det[c] and the record (start_record_words(n) int64
// words): [0] L, [1] the number of invariant factors above one, then z_base (2n doubles), their
// radices, then their V columns (n each).  ws: the thread's working arrays (start_ws_words(n)).
__global__ void __launch_bounds__(64)
    k_start_plan(int n, int64_t c0, int64_t c1, const int32_t *__restrict__ Dall,
                 const double *__restrict__ beta_all, int64_t *__restrict__ rec_all,
                 int32_t *__restrict__ status, int64_t *__restrict__ det_out,
                 int64_t *__restrict__ ws_all) {
  for (int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < c1;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int32_t *D = Dall + c * n * n;
    const double *beta = beta_all + c * 2 * n;
    int64_t *rec = rec_all + c * start_record_words(n);
    int64_t *M = ws_all + (c - c0) * start_ws_words(n);
    int64_t *V = M + n * n;
    int64_t *sig = V + n * n;
    double *A = reinterpret_cast<double *>(sig + n);
    double *br = A + n * n, *bi = br + n;
    det_out[c] = 0;
    int32_t st = kPlanOk;
    for (int k = 0; k < n; ++k) {
      const double r = beta[2 * k], im = beta[2 * k + 1];
      if (!isfinite(r) || !isfinite(im) || (r == 0.0 && im == 0.0)) st = kPlanBadBeta;
      br[k] = log(hypot(r, im));
      bi[k] = atan2(im, r);
    }
    for (int i = 0; i < n * n && st == kPlanOk; ++i) M[i] = D[i];
    if (st == kPlanOk) st = smith64(n, M, nullptr, 1, sig);
    int64_t det = 1;
    for (int l = 0; l < n && st == kPlanOk; ++l)
      if (__builtin_mul_overflow(det, sig[l], &det) || det >= ((int64_t)1 << 62)) st = kPlanTooMany;
    const int64_t L = st == kPlanOk ? sig[n - 1] : 1;
    if (st == kPlanOk && L >= ((int64_t)1 << 31)) st = kPlanBigFactor;
    if (st == kPlanOk) {  // second run: the same operations, V modulo L
      for (int i = 0; i < n * n; ++i) M[i] = D[i];
      st = smith64(n, M, V, L, sig);
    }
    if (st == kPlanOk && !solve_complex(n, D, A, br, bi)) st = kPlanSingular;
    if (st == kPlanOk) {
      int nlive = 0;
      for (int l = 0; l < n; ++l) nlive += sig[l] > 1;
      rec[0] = L;
      rec[1] = nlive;
      for (int i = 0; i < n; ++i) {
        rec[2 + 2 * i] = __double_as_longlong(br[i]);
        rec[3 + 2 * i] = __double_as_longlong(bi[i]);
      }
      int64_t *rs = rec + 2 + 2 * n, *rc = rs + nlive;
      int q = 0;
      for (int l = 0; l < n; ++l) {
        if (sig[l] == 1) continue;
        rs[q] = sig[l];
        const int64_t step = L / sig[l];
        for (int i = 0; i < n; ++i) rc[q * n + i] = (V[i * n + l] % sig[l]) * step % L;
        ++q;
      }
      det_out[c] = det;
    }
    status[c] = st;
  }
}

// One thread per (root row, coordinate): the cell by binary search over the rows' starts, the
// root index's mixed-radix digits over the cell's invariant factors above one (first fastest),
// the fractional part sum_l j_l cm[l][i] mod L, the imaginary part reduced into [-pi, pi).
__global__ void __launch_bounds__(256)
    k_binomial_starts(int n, int num_cells, const StartHdr *__restrict__ hdr,
                      const int64_t *__restrict__ rec_all, int64_t rows, double *__restrict__ z) {
  const int64_t total = rows * n;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = g / n;
    const int i = (int)(g - row * n);
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
    const double zr = __longlong_as_double(d[2 + 2 * i]), zi0 = __longlong_as_double(d[3 + 2 * i]);
    const int64_t *rs = d + 2 + 2 * n, *rc = rs + nlive;
    int64_t q = h.first + (row - h.row0), num = 0;
    for (int l = 0; l < nlive; ++l) {
      const int64_t sg = rs[l];
      const int64_t j = q % sg;
      q /= sg;
      num = (num + j * rc[(int64_t)l * n + i]) % L;
    }
    const double two_pi = 6.283185307179586476925286766559;
    double im = zi0 + two_pi * ((double)num / (double)L) + 3.14159265358979323846264338327950;
    im -= two_pi * floor(im / two_pi);
    im -= 3.14159265358979323846264338327950;
    if (im >= 3.14159265358979323846264338327950) im -= two_pi;  // rounding at the top edge
    z[2 * g] = zr;
    z[2 * g + 1] = im;
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
                             int64_t *rec, int32_t *status, int64_t *det, int64_t *ws,
                             int64_t ws_cells, hipStream_t stream) {
  prof_begin(stream);
  for (int64_t c0 = 0; c0 < num_cells; c0 += ws_cells) {
    const int64_t c1 = c0 + ws_cells < num_cells ? c0 + ws_cells : num_cells;
    const int64_t blocks = (c1 - c0 + 63) / 64;
    hipLaunchKernelGGL(k_start_plan, dim3((unsigned)blocks), dim3(64), 0, stream, n, c0, c1, D,
                       beta, rec, status, det, ws);
  }
  prof_end(stream, "k_start_plan");
  return hipGetLastError();
}

hipError_t launch_binomial_starts(int n, int num_cells, const StartHdr *hdr, const int64_t *rec,
                                  int64_t rows, double *z, hipStream_t stream) {
  prof_begin(stream);
  const int64_t total = rows * n;
  int64_t blocks = (total + 255) / 256;
  const int64_t cap = (int64_t)num_cus() * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_binomial_starts, dim3((unsigned)blocks), dim3(256), 0, stream, n,
                     num_cells, hdr, rec, rows, z);
  prof_end(stream, "k_binomial_starts");
  return hipGetLastError();
}

}  // namespace hom
