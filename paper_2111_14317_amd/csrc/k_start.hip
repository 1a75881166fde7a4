// Start points of polyhedral homotopy (Sec. 2): every root of the binomial start system
// x^{d_k} = beta_k of each mixed cell, written on the GPU.
//
// In log coordinates D z = log(beta) + 2 pi i k (k integer).  With the Smith form U D V = S =
// diag(sigma_0 | sigma_1 | ...), U and V unimodular, the |det D| = prod sigma_l roots are
//     z = z_base + 2 pi i sum_l V[:, l] j_l / sigma_l,   0 <= j_l < sigma_l,
// z_base = D^{-1} log(beta) (principal logarithm).  Only the fractional part of the second term
// matters, so V is needed modulo the largest factor L = sigma_{n-1} (every sigma_l divides L):
// column l contributes ((V_il mod sigma_l) * (L / sigma_l) * j_l mod L) / L.
//
// Host, per cell (exact): the Smith form by elementary operations on 128-bit integers, run twice
// (the second run repeats the first one's operations and carries V modulo L, which the first
// run found), and z_base by an FP64 LU solve.  GPU: one thread per (root, coordinate), writing
// consecutive doubles, so the launch streams its output to HBM.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "hom_internal.h"

namespace hom {

namespace {

typedef __int128 i128;

constexpr i128 kEntryLimit = (i128)1 << 100;

i128 iabs(i128 v) { return v < 0 ? -v : v; }

// Smith form of the n x n matrix M (row-major, modified in place).  With track_v, V is carried
// modulo `mod` (column operations only).  Returns false if an entry grows beyond kEntryLimit or
// the matrix is singular (then *singular is set).
bool smith(int n, std::vector<i128> &M, bool track_v, int64_t mod, std::vector<int64_t> &V,
           bool *singular) {
  *singular = false;
  auto at = [&](int i, int j) -> i128 & { return M[(size_t)i * n + j]; };
  auto vmod = [&](i128 v) -> int64_t {
    i128 r = v % mod;
    return (int64_t)(r < 0 ? r + mod : r);
  };
  if (track_v) {
    V.assign((size_t)n * n, 0);
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = vmod(1);
  }
  auto swap_cols = [&](int a, int b) {
    for (int i = 0; i < n; ++i) std::swap(at(i, a), at(i, b));
    if (track_v)
      for (int i = 0; i < n; ++i) std::swap(V[(size_t)i * n + a], V[(size_t)i * n + b]);
  };
  auto add_col = [&](int dst, int src, i128 f) {  // col dst += f col src
    for (int i = 0; i < n; ++i) {
      at(i, dst) += f * at(i, src);
    }
    if (track_v) {
      const i128 fm = vmod(f);
      for (int i = 0; i < n; ++i)
        V[(size_t)i * n + dst] = vmod((i128)V[(size_t)i * n + dst] + fm * V[(size_t)i * n + src]);
    }
  };
  auto add_row = [&](int dst, int src, i128 f) {  // row dst += f row src (U is not needed)
    for (int j = 0; j < n; ++j) at(dst, j) += f * at(src, j);
  };
  auto bounded = [&](int t) {
    for (int i = t; i < n; ++i)
      for (int j = t; j < n; ++j)
        if (iabs(at(i, j)) > kEntryLimit) return false;
    return true;
  };
  for (int t = 0; t < n; ++t) {
    for (;;) {
      int bi = -1, bj = -1;  // smallest nonzero |entry| of the trailing block, first in row order
      for (int i = t; i < n; ++i)
        for (int j = t; j < n; ++j)
          if (at(i, j) != 0 && (bi < 0 || iabs(at(i, j)) < iabs(at(bi, bj)))) {
            bi = i;
            bj = j;
          }
      if (bi < 0) {
        *singular = true;
        return false;
      }
      if (bi != t)
        for (int j = 0; j < n; ++j) std::swap(at(t, j), at(bi, j));
      if (bj != t) swap_cols(t, bj);
      bool done = true;
      const i128 p = at(t, t);
      for (int i = t + 1; i < n; ++i) {
        const i128 q = at(i, t) / p;
        if (q != 0) add_row(i, t, -q);
        if (at(i, t) != 0) done = false;
      }
      for (int j = t + 1; j < n; ++j) {
        const i128 q = at(t, j) / p;
        if (q != 0) add_col(j, t, -q);
        if (at(t, j) != 0) done = false;
      }
      if (!bounded(t)) return false;
      if (!done) continue;
      int bad = -1;  // the pivot must divide the whole trailing block
      for (int i = t + 1; i < n && bad < 0; ++i)
        for (int j = t + 1; j < n; ++j)
          if (at(i, j) % p != 0) {
            bad = i;
            break;
          }
      if (bad < 0) break;
      add_row(t, bad, 1);
    }
    if (at(t, t) < 0)
      for (int j = 0; j < n; ++j) at(t, j) = -at(t, j);  // a row sign: U only
  }
  return true;
}

// Solve D x = b (complex, FP64) by LU with partial pivoting; false if D is singular in FP64.
bool solve_c(int n, const int32_t *D, const std::complex<double> *b, std::complex<double> *x) {
  std::vector<double> A((size_t)n * n);
  for (int i = 0; i < n * n; ++i) A[i] = D[i];
  std::vector<std::complex<double>> r(b, b + n);
  for (int j = 0; j < n; ++j) {
    int p = j;
    for (int i = j + 1; i < n; ++i)
      if (std::fabs(A[(size_t)i * n + j]) > std::fabs(A[(size_t)p * n + j])) p = i;
    if (A[(size_t)p * n + j] == 0.0) return false;
    if (p != j) {
      for (int k = 0; k < n; ++k) std::swap(A[(size_t)j * n + k], A[(size_t)p * n + k]);
      std::swap(r[j], r[p]);
    }
    for (int i = j + 1; i < n; ++i) {
      const double f = A[(size_t)i * n + j] / A[(size_t)j * n + j];
      for (int k = j; k < n; ++k) A[(size_t)i * n + k] -= f * A[(size_t)j * n + k];
      r[i] -= f * r[j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    std::complex<double> v = r[i];
    for (int k = i + 1; k < n; ++k) v -= A[(size_t)i * n + k] * x[k];
    x[i] = v / A[(size_t)i * n + i];
  }
  return true;
}

}  // namespace

// Plan one cell: |det D|, the radices and V columns of the invariant factors above one, z_base.
// Returns an empty string or the problem (code: HOM_EINVAL or HOM_EUNSUPPORTED).
std::string start_plan(int n, const int32_t *D, const double *beta, StartPlan *out, int *code) {
  *code = HOM_EINVAL;
  for (int k = 0; k < n; ++k) {
    const double br = beta[2 * k], bi = beta[2 * k + 1];
    if (!std::isfinite(br) || !std::isfinite(bi) || (br == 0.0 && bi == 0.0))
      return "beta must be finite and nonzero";
  }
  std::vector<i128> M((size_t)n * n);
  for (int i = 0; i < n * n; ++i) M[i] = D[i];
  std::vector<int64_t> V;
  bool singular = false;
  if (!smith(n, M, false, 1, V, &singular)) {
    if (singular) return "D is singular (det 0)";
    *code = HOM_EUNSUPPORTED;
    return "an entry of the Smith form exceeds 2^100";
  }
  i128 det = 1;
  for (int l = 0; l < n; ++l) {
    det *= M[(size_t)l * n + l];
    if (det >= ((i128)1 << 62)) {
      *code = HOM_EUNSUPPORTED;
      return "|det D| >= 2^62 roots";
    }
  }
  const i128 L = M[(size_t)(n - 1) * n + (n - 1)];
  if (L >= ((i128)1 << 31)) {
    *code = HOM_EUNSUPPORTED;
    return "the largest invariant factor of D is >= 2^31";
  }
  std::vector<i128> sig(n);
  for (int l = 0; l < n; ++l) sig[l] = M[(size_t)l * n + l];
  // second run: the same operations, V modulo L
  for (int i = 0; i < n * n; ++i) M[i] = D[i];
  if (!smith(n, M, true, (int64_t)L, V, &singular)) {
    *code = HOM_EUNSUPPORTED;
    return "Smith form: second pass failed";
  }
  out->det = (int64_t)det;
  out->L = (int64_t)L;
  out->sig.clear();
  out->cm.clear();
  for (int l = 0; l < n; ++l) {
    if (sig[l] == 1) continue;
    out->sig.push_back((int64_t)sig[l]);
    const int64_t step = (int64_t)(L / sig[l]);
    for (int i = 0; i < n; ++i)
      out->cm.push_back((int64_t)(((i128)(V[(size_t)i * n + l] % (int64_t)sig[l]) * step) % L));
  }
  std::vector<std::complex<double>> b(n), x(n);
  for (int k = 0; k < n; ++k) b[k] = std::log(std::complex<double>(beta[2 * k], beta[2 * k + 1]));
  if (!solve_c(n, D, b.data(), x.data())) return "D is singular in FP64";
  out->zb.resize(2 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    out->zb[2 * i] = x[i].real();
    out->zb[2 * i + 1] = x[i].imag();
  }
  return std::string();
}

// Pack the plans into the device layout: [num_cells] headers, then each cell's data
// (z_base 2n doubles, radices, V columns as int64).
void start_pack(int n, const std::vector<StartPlan> &plans, const int64_t *first,
                const int64_t *count, std::vector<StartHdr> &hdr, std::vector<int64_t> &data,
                int64_t *rows) {
  hdr.resize(plans.size());
  data.clear();
  int64_t row = 0;
  for (size_t c = 0; c < plans.size(); ++c) {
    const StartPlan &p = plans[c];
    StartHdr &h = hdr[c];
    h.row0 = row;
    h.first = first ? first[c] : 0;
    h.count = count ? count[c] : p.det;
    h.L = p.L;
    h.nlive = (int32_t)p.sig.size();
    h.off = (int64_t)data.size();
    for (int i = 0; i < 2 * n; ++i) {
      int64_t bits;
      memcpy(&bits, &p.zb[i], 8);
      data.push_back(bits);
    }
    for (int64_t v : p.sig) data.push_back(v);
    for (int64_t v : p.cm) data.push_back(v);
    row += h.count;
  }
  *rows = row;
}

// One thread per (root row, coordinate): the cell by binary search over the rows' starts, the
// root index's mixed-radix digits over the cell's invariant factors above one (first fastest),
// the fractional part sum_l j_l cm[l][i] mod L, the imaginary part reduced into [-pi, pi).
__global__ void __launch_bounds__(256)
    k_binomial_starts(int n, int num_cells, const StartHdr *__restrict__ hdr,
                      const int64_t *__restrict__ data, int64_t rows, double *__restrict__ z) {
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
    const int64_t *d = data + h.off;
    const double zr = __longlong_as_double(d[2 * i]), zi0 = __longlong_as_double(d[2 * i + 1]);
    int64_t q = h.first + (row - h.row0), num = 0;
    for (int l = 0; l < h.nlive; ++l) {
      const int64_t sg = d[2 * n + l];
      const int64_t j = q % sg;
      q /= sg;
      num = (num + j * d[2 * n + h.nlive + (int64_t)l * n + i]) % h.L;
    }
    const double two_pi = 6.283185307179586476925286766559;
    double im = zi0 + two_pi * ((double)num / (double)h.L) + 3.14159265358979323846264338327950;
    im -= two_pi * floor(im / two_pi);
    im -= 3.14159265358979323846264338327950;
    if (im >= 3.14159265358979323846264338327950) im -= two_pi;  // rounding at the top edge
    z[2 * g] = zr;
    z[2 * g + 1] = im;
  }
}

hipError_t launch_binomial_starts(int n, int num_cells, const StartHdr *hdr, const int64_t *data,
                                  int64_t rows, double *z, hipStream_t stream) {
  prof_begin(stream);
  const int64_t total = rows * n;
  int64_t blocks = (total + 255) / 256;
  const int64_t cap = (int64_t)num_cus() * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_binomial_starts, dim3((unsigned)blocks), dim3(256), 0, stream, n,
                     num_cells, hdr, data, rows, z);
  prof_end(stream, "k_binomial_starts");
  return hipGetLastError();
}

}  // namespace hom
