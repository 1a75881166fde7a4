// C ABI (include/hom.h): argument validation, handles, workspaces, launches.
#include <string.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/hom.h"
#include "hom_internal.h"

namespace hom {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

// The library's second stream on each device (default priority, created on first use), for the
// FP64 launch that runs beside the mixed form's FP32 launch.
static constexpr int kSideBlocks = 8;  // its grid: 8 blocks of 4 waves
static hipError_t side_stream(hipStream_t *out) {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev]) {
    e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  *out = streams[dev];
  return hipSuccess;
}

// ---- kernel timing ----
struct ProfRec {
  hipEvent_t a, b;
  unsigned long long *units;  // device counter or nullptr
  char label[64];
};
static thread_local bool g_prof = false;
static thread_local std::vector<ProfRec> g_recs;
static thread_local std::vector<hipEvent_t> g_pool;
static thread_local hipEvent_t g_open = nullptr;
static thread_local unsigned long long *g_open_units = nullptr;
constexpr size_t kMaxRecs = 4096;
// one unit counter per record, allocated when profiling is switched on (no allocation between
// launches: that could order a launch on another stream behind the running one)
static thread_local unsigned long long *g_units_pool = nullptr;

static hipEvent_t pool_get() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_begin(hipStream_t stream) {
  g_open_units = nullptr;
  if (!g_prof || g_recs.size() >= kMaxRecs) return;
  g_open = pool_get();
  if (g_open) (void)hipEventRecord(g_open, stream);
}

__global__ void k_prof_zero(unsigned long long *p) { *p = 0ull; }

unsigned long long *prof_units(hipStream_t stream) {
  if (!g_prof || !g_open || !g_units_pool) return nullptr;
  unsigned long long *u = g_units_pool + g_recs.size();
  hipLaunchKernelGGL(k_prof_zero, dim3(1), dim3(1), 0, stream, u);
  g_open_units = u;
  return u;
}

void prof_end(hipStream_t stream, const char *label) {
  if (!g_prof || !g_open) return;
  hipEvent_t b = pool_get();
  if (!b) return;
  (void)hipEventRecord(b, stream);
  ProfRec r;
  r.a = g_open;
  r.b = b;
  r.units = g_open_units;
  g_open_units = nullptr;
  strncpy(r.label, label, 63);
  r.label[63] = 0;
  g_recs.push_back(r);
  g_open = nullptr;
}

int bucket_for(int n) {
  for (int N : kSizes)
    if (N >= n) return N;
  return 0;
}

int table_ld(int N) { return ((N + 1) & 1) ? (N + 1) : (N + 2); }

int num_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cached[dev] = v;
  }
  return cached[dev];
}

static size_t lds_for(int N, int n, int mmax) {
  return (size_t)mmax * n * table_ld(N) * 8 + (size_t)mmax * n * (16 + 8) + 4 * 32 + 64;
}

}  // namespace hom

using namespace hom;

struct hom_system_s {
  System s;
};

#define HOM_FAIL(code, msg)   \
  do {                        \
    set_error(msg);           \
    return code;              \
  } while (0)

#define HOM_HIP(call, what)                                                        \
  do {                                                                             \
    hipError_t _e = (call);                                                        \
    if (_e != hipSuccess) {                                                        \
      set_error(std::string(what) + ": " + hipGetErrorString(_e));                 \
      return _e == hipErrorOutOfMemory ? HOM_ENOMEM : HOM_EDEVICE;                 \
    }                                                                              \
  } while (0)

static constexpr size_t kMaxLds = 48 * 1024;  // leaves room for per-group state

// Validate one system; fills M and the largest m_k.  Returns an empty string or the problem.
static std::string validate_system(int n, const int32_t *m, const int8_t *A, const double *w,
                                   int64_t *M_out, int *mmax_out) {
  if (n < 1 || n > 32) return "n must be in [1, 32]";
  if (!m || !A || !w) return "m, A and w must be non-NULL";
  int64_t M = 0;
  int mmax = 0;
  for (int k = 0; k < n; ++k) {
    if (m[k] < 1) return "every m[k] must be >= 1";
    M += m[k];
    if (m[k] > mmax) mmax = m[k];
  }
  if (M > 65536) return "M must be <= 65536";
  for (int64_t i = 0; i < M * n; ++i)
    if (A[i] == -128) return "exponents must lie in [-127, 127]";
  for (int64_t i = 0; i < M; ++i)
    if (!std::isfinite(w[i]) || w[i] < 0) return "liftings must be finite and non-negative";
  *M_out = M;
  *mmax_out = mmax;
  return "";
}

// Exponent table [mmax][n][LD]: exponents as doubles zero padded to N, lifting in slot N.  With
// `hom` (a projective handle) slot n holds the homogenising exponent hom[monomial].
static void build_table(int n, int N, const int32_t *m, const int8_t *A, const double *w, int mmax,
                        std::vector<double> &T, std::vector<int32_t> &off,
                        const std::vector<int> *hom = nullptr) {
  const int LD = table_ld(N);
  off.assign(n, 0);
  int64_t acc = 0;
  for (int k = 0; k < n; ++k) {
    off[k] = (int32_t)acc;
    acc += m[k];
  }
  T.assign((size_t)mmax * n * LD, 0.0);
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < m[k]; ++i) {
      double *t = &T[((size_t)i * n + k) * LD];
      const int8_t *a = A + (size_t)(off[k] + i) * n;
      for (int j = 0; j < n; ++j) t[j] = (double)a[j];
      if (hom) t[n] = (double)(*hom)[off[k] + i];
      t[N] = w[off[k] + i];
    }
}

// Matrix-core tables of a dense-support system, laid out for the 16x16 MFMA operand lanes
// (lane l: row / column l % 16, K block l / 16).  Each equation's monomials are padded to a
// multiple of 32 with copies of its first monomial (the padding gets coefficient 0 per call).
struct DenseHost {
  int Md = 0;
  std::vector<int32_t> tile0, src;
  std::vector<uint16_t> EAb, CBb;  // bf16 bit patterns (small integers: exact)
  std::vector<double> EAd, CBd, W;
};

static uint16_t bf16_of_int(int v) {
  const float f = (float)v;  // |v| <= 127: exact in 8 significant bits
  uint32_t u;
  memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}

static void build_dense(int n, const int32_t *m, const int8_t *A, const double *w,
                        const std::vector<int32_t> &off, DenseHost &D) {
  std::vector<int32_t> doff(n + 1, 0);
  for (int k = 0; k < n; ++k) doff[k + 1] = doff[k] + (m[k] + 31) / 32 * 32;
  const int Md = doff[n];
  D.Md = Md;
  D.tile0.resize(n + 1);
  for (int k = 0; k <= n; ++k) D.tile0[k] = doff[k] / 16;
  D.src.assign(Md, -1);
  std::vector<int32_t> mono(Md);  // monomial whose exponents and lifting slot d carries
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < doff[k + 1] - doff[k]; ++i) {
      mono[doff[k] + i] = off[k] + (i < m[k] ? i : 0);
      if (i < m[k]) D.src[doff[k] + i] = off[k] + i;
    }
  auto a = [&](int d, int j) -> int { return j < n ? (int)A[(size_t)mono[d] * n + j] : 0; };
  const int ntile = Md / 16;
  D.EAb.assign((size_t)ntile * 64 * 8, 0);
  D.EAd.assign((size_t)ntile * 8 * 64, 0.0);
  D.CBd.assign((size_t)ntile * 4 * 2 * 64, 0.0);
  D.CBb.assign((size_t)(Md / 32) * 2 * 64 * 8, 0);
  D.W.resize(Md);
  for (int d = 0; d < Md; ++d) D.W[d] = w[mono[d]];
  for (int t = 0; t < ntile; ++t)
    for (int l = 0; l < 64; ++l) {
      for (int e = 0; e < 8; ++e)  // A1 bf16 A operand: row = monomial, K = coordinate
        D.EAb[((size_t)t * 64 + l) * 8 + e] = bf16_of_int(a(16 * t + l % 16, 8 * (l / 16) + e));
      for (int ks = 0; ks < 8; ++ks)  // A1 FP64 A operand
        D.EAd[((size_t)t * 8 + ks) * 64 + l] = a(16 * t + l % 16, 4 * ks + l / 16);
      for (int r = 0; r < 4; ++r)  // A3 FP64 B operand: K = monomial 4r + l/16 of the tile (the
        for (int ct = 0; ct < 2; ++ct)  // row that result register r of lane l holds after A1)
          D.CBd[(((size_t)t * 4 + r) * 2 + ct) * 64 + l] =
              a(16 * t + 4 * r + l / 16, 16 * ct + l % 16);
    }
  for (int ch = 0; ch < Md / 32; ++ch)  // A3 bf16 B operand: element e of K block l/16 is
    for (int ct = 0; ct < 2; ++ct)      // monomial 32 ch + 16 (e / 4) + 4 (l / 16) + e % 4
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e)
          D.CBb[(((size_t)ch * 2 + ct) * 64 + l) * 8 + e] =
              bf16_of_int(a(32 * ch + 16 * (e / 4) + 4 * (l / 16) + e % 4, 16 * ct + l % 16));
}

static void free_system(System &S) {
  (void)hipFree(S.dT);
  (void)hipFree(S.dmk);
  (void)hipFree(S.doff);
  (void)hipFree(S.dA);
  (void)hipFree(S.dBatch);
  (void)hipFree(S.dT_all);
  (void)hipFree(S.dInts_all);
  (void)hipFree(S.dDense);
}

// This call's table-order coefficients for a system whose tables stay in global memory (a
// stream-ordered workspace, freed by coeff_end); nothing for systems staged in LDS.
static hipError_t coeff_begin(const System &S, const double *c, hipStream_t st, void **cws) {
  *cws = nullptr;
  if (!S.global_tables) return hipSuccess;
  hipError_t e = hipMallocAsync(cws, S.coeff_ws_bytes(), st);
  if (e != hipSuccess) {
    *cws = nullptr;
    return e;
  }
  return launch_coeff_tables(S, c, *cws, st);
}

static hipError_t coeff_end(void *cws, hipStream_t st) {
  return cws ? hipFreeAsync(cws, st) : hipSuccess;
}

extern "C" {

const char *hom_last_error(void) { return g_err.c_str(); }

int hom_binomial_starts(int n, int num_cells, const int32_t *D, const double *beta,
                        const int64_t *first, const int64_t *count, int64_t *num_roots, double *z,
                        int64_t z_rows, hom_stream_t stream) {
  g_err.clear();
  if (n < 1 || n > 32) HOM_FAIL(HOM_EINVAL, "hom_binomial_starts: n must be in [1, 32]");
  if (num_cells < 1) HOM_FAIL(HOM_EINVAL, "hom_binomial_starts: num_cells < 1");
  if (!D || !beta || !num_roots) HOM_FAIL(HOM_EINVAL, "hom_binomial_starts: NULL array");
  if ((first == nullptr) != (count == nullptr))
    HOM_FAIL(HOM_EINVAL, "hom_binomial_starts: first and count must both be given or both NULL");
  hipStream_t st = (hipStream_t)stream;
  const int64_t cells = num_cells, rw = start_record_words(n);
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t bD = up((size_t)cells * n * n * 4), bB = up((size_t)cells * 2 * n * 8),
               bR = up((size_t)cells * rw * 8), bS = up((size_t)cells * 4), bT = up((size_t)cells * 8),
               bH = up((size_t)cells * sizeof(StartHdr));
  char *ws = nullptr;
  HOM_HIP(hipMallocAsync((void **)&ws, bD + bB + bR + bS + bT + bH, st),
          "hom_binomial_starts: workspace");
  int32_t *dD = reinterpret_cast<int32_t *>(ws);
  double *dB = reinterpret_cast<double *>(ws + bD);
  int64_t *dR = reinterpret_cast<int64_t *>(ws + bD + bB);
  int32_t *dS = reinterpret_cast<int32_t *>(ws + bD + bB + bR);
  int64_t *dT = reinterpret_cast<int64_t *>(ws + bD + bB + bR + bS);
  StartHdr *dH = reinterpret_cast<StartHdr *>(ws + bD + bB + bR + bS + bT);
  std::vector<int32_t> hs(cells);
  std::vector<StartHdr> hdr;
  // plan every cell on the GPU, then read back each cell's status and root count
  hipError_t e = hipMemcpyAsync(dD, D, (size_t)cells * n * n * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dB, beta, (size_t)cells * 2 * n * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_start_plan(n, cells, dD, dB, dR, dS, dT, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hs.data(), dS, (size_t)cells * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(num_roots, dT, (size_t)cells * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  std::string why;
  int code = HOM_OK;
  int64_t rows = 0;
  for (int64_t c = 0; c < cells && e == hipSuccess && code == HOM_OK; ++c) {
    if (hs[c] != 0) {
      code = start_status_code(hs[c]);
      why = "cell " + std::to_string(c) + ": " + start_status_text(hs[c]);
    } else if (first && (first[c] < 0 || count[c] < 0 || first[c] > num_roots[c] ||
                         count[c] > num_roots[c] - first[c])) {
      code = HOM_EINVAL;
      why = "cell " + std::to_string(c) + ": [first, first + count) outside its roots";
    }
  }
  if (e == hipSuccess && code == HOM_OK && z) {
    hdr.resize(cells);
    for (int64_t c = 0; c < cells; ++c) {
      hdr[c] = StartHdr{rows, first ? first[c] : 0, first ? count[c] : num_roots[c]};
      rows += hdr[c].count;
    }
    if (rows > z_rows) {
      code = HOM_EINVAL;
      why = "more roots than z_rows";
    } else if (rows > 0) {
      e = hipMemcpyAsync(dH, hdr.data(), (size_t)cells * sizeof(StartHdr), hipMemcpyHostToDevice,
                         st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host headers die with this call
      if (e == hipSuccess)
        e = launch_binomial_starts(n, num_cells, dH, dR, rows, z, st);
    }
  }
  hipError_t e2 = hipFreeAsync(ws, st);
  HOM_HIP(e, "hom_binomial_starts");
  HOM_HIP(e2, "hom_binomial_starts: free workspace");
  if (code != HOM_OK) HOM_FAIL(code, "hom_binomial_starts: " + why);
  return HOM_OK;
}

int hom_peak_probe(int kind, double *rate, hom_stream_t stream) {
  g_err.clear();
  if (!rate) HOM_FAIL(HOM_EINVAL, "hom_peak_probe: NULL rate");
  if (kind < HOM_PEAK_HBM_READ || kind > HOM_PEAK_SINCOS_F64)
    HOM_FAIL(HOM_EINVAL, "hom_peak_probe: unknown kind");
  HOM_HIP(peak_probe(kind, rate, (hipStream_t)stream), "hom_peak_probe");
  return HOM_OK;
}

int hom_set_profiling(int on) {
  g_err.clear();
  if (on && !g_units_pool)
    HOM_HIP(hipMalloc((void **)&g_units_pool, kMaxRecs * sizeof *g_units_pool),
            "hom_set_profiling: unit counters");
  g_prof = on != 0;
  return HOM_OK;
}

int hom_profile_read(char *names, double *ms, int64_t *units, int cap) {
  g_err.clear();
  if (cap < 0 || (cap > 0 && (!names || !ms || !units)))
    HOM_FAIL(HOM_EINVAL, "hom_profile_read: bad buffers");
  int out = 0;
  hipError_t err = hipSuccess;
  for (ProfRec &r : g_recs) {
    hipError_t e = hipEventSynchronize(r.b);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess && err == hipSuccess) err = e;
    int64_t u = -1;
    if (r.units) {
      unsigned long long hv = 0;
      if (e == hipSuccess) e = hipMemcpy(&hv, r.units, sizeof hv, hipMemcpyDeviceToHost);
      if (e != hipSuccess && err == hipSuccess) err = e;
      u = (int64_t)hv;
    }
    if (out < cap) {
      memcpy(names + 64 * out, r.label, 64);
      ms[out] = (double)t;
      units[out] = u;
      ++out;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  if (err != hipSuccess) HOM_HIP(err, "hom_profile_read");
  return out;
}

int hom_create(int n, const int32_t *m, const int8_t *A, const double *w, int flags,
               hom_system_t *out) {
  g_err.clear();
  if (!out) HOM_FAIL(HOM_EINVAL, "hom_create: out is NULL");
  *out = nullptr;
  if (flags & ~(HOM_CREATE_VALU | HOM_CREATE_PROJECTIVE | HOM_CREATE_PER_EQUATION))
    HOM_FAIL(HOM_EINVAL, "hom_create: unknown flags");
  int64_t M = 0;
  int mmax = 0;
  const std::string bad = validate_system(n, m, A, w, &M, &mmax);
  if (!bad.empty()) HOM_FAIL(HOM_EINVAL, "hom_create: " + bad);
  const bool projective = (flags & HOM_CREATE_PROJECTIVE) != 0;
  // homogenising exponents (Sec. 2.2): d_k - sum_j a_j with d_k the largest total degree of
  // equation k, so that each equation is homogeneous of degree d_k in n + 1 unknowns
  std::vector<int> hom;
  if (projective) {
    if (proj_group_size(n) == 0) HOM_FAIL(HOM_EINVAL, "hom_create: projective handles need n <= 29");
    hom.resize((size_t)M);
    int64_t o = 0;
    for (int k = 0; k < n; ++k) {
      int dk = INT_MIN;
      for (int i = 0; i < m[k]; ++i) {
        int t = 0;
        for (int j = 0; j < n; ++j) t += A[(size_t)(o + i) * n + j];
        hom[(size_t)(o + i)] = t;
        dk = std::max(dk, t);
      }
      for (int i = 0; i < m[k]; ++i) {
        hom[(size_t)(o + i)] = dk - hom[(size_t)(o + i)];
        if (hom[(size_t)(o + i)] > 127)
          HOM_FAIL(HOM_EINVAL, "hom_create: a homogenising exponent exceeds 127");
      }
      o += m[k];
    }
  }
  const int N = projective ? proj_group_size(n) : bucket_for(n);
  const size_t lds = lds_for(N, n, mmax);
  std::vector<double> T;
  std::vector<int32_t> off;
  build_table(n, N, m, A, w, mmax, T, off, projective ? &hom : nullptr);
  std::vector<int32_t> A32((size_t)M * n);
  for (size_t i = 0; i < A32.size(); ++i) A32[i] = A[i];

  hom_system_s *h = new hom_system_s();
  System &S = h->s;
  S.n = n;
  S.N = N;
  S.mmax = mmax;
  S.M = (int)M;
  // tables beyond the LDS budget stay in global memory (read through the caches)
  S.global_tables = lds > kMaxLds;
  S.lds_bytes = S.global_tables ? 0 : lds;
  S.projective = projective;
  auto fail = [&](hipError_t e, const char *what) {
    set_error(std::string("hom_create: ") + what + ": " + hipGetErrorString(e));
    free_system(S);
    delete h;
    return e == hipErrorOutOfMemory ? HOM_ENOMEM : HOM_EDEVICE;
  };
  hipError_t e;
  if ((e = hipGetDevice(&S.device)) != hipSuccess) return fail(e, "hipGetDevice");
  if ((e = hipMalloc(&S.dT, T.size() * 8)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = hipMalloc(&S.dmk, n * 4)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = hipMalloc(&S.doff, n * 4)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = hipMalloc(&S.dA, A32.size() * 4)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = hipMemcpy(S.dT, T.data(), T.size() * 8, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e, "hipMemcpy");
  if ((e = hipMemcpy(S.dmk, m, n * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e, "hipMemcpy");
  if ((e = hipMemcpy(S.doff, off.data(), n * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e, "hipMemcpy");
  if ((e = hipMemcpy(S.dA, A32.data(), A32.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e, "hipMemcpy");
  // a common support: every equation lists the same monomials in the same order, same liftings
  bool same = !projective && n > 1 && !(flags & HOM_CREATE_PER_EQUATION);
  for (int k = 1; k < n && same; ++k) {
    if (m[k] != m[0]) {
      same = false;
      break;
    }
    same = memcmp(A + (size_t)off[k] * n, A, (size_t)m[0] * n) == 0 &&
           memcmp(w + off[k], w, (size_t)m[0] * sizeof(double)) == 0;
  }
  S.union_support = same && mmax >= kDenseMinM && !(flags & HOM_CREATE_VALU) &&
                    (size_t)((m[0] + 31) / 32 * 32) * 16 * 16 <= kUnionLdsBytes;
  S.union_tiles = S.union_support ? (m[0] + 31) / 32 * 2 : 0;
  if (mmax >= kDenseMinM && !(flags & HOM_CREATE_VALU) && !projective) {
    DenseHost D;
    build_dense(n, m, A, w, off, D);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t o_tile0 = 0, o_src = o_tile0 + al(D.tile0.size() * 4);
    const size_t o_EAb = o_src + al(D.src.size() * 4), o_EAd = o_EAb + al(D.EAb.size() * 2);
    const size_t o_CBb = o_EAd + al(D.EAd.size() * 8), o_CBd = o_CBb + al(D.CBb.size() * 2);
    const size_t o_W = o_CBd + al(D.CBd.size() * 8), total = o_W + al(D.W.size() * 8);
    std::vector<char> img(total, 0);
    memcpy(img.data() + o_tile0, D.tile0.data(), D.tile0.size() * 4);
    memcpy(img.data() + o_src, D.src.data(), D.src.size() * 4);
    memcpy(img.data() + o_EAb, D.EAb.data(), D.EAb.size() * 2);
    memcpy(img.data() + o_EAd, D.EAd.data(), D.EAd.size() * 8);
    memcpy(img.data() + o_CBb, D.CBb.data(), D.CBb.size() * 2);
    memcpy(img.data() + o_CBd, D.CBd.data(), D.CBd.size() * 8);
    memcpy(img.data() + o_W, D.W.data(), D.W.size() * 8);
    if ((e = hipMalloc(&S.dDense, total)) != hipSuccess) return fail(e, "hipMalloc");
    if ((e = hipMemcpy(S.dDense, img.data(), total, hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e, "hipMemcpy");
    char *b = static_cast<char *>(S.dDense);
    S.Md = D.Md;
    S.dense = DenseDev{n,
                       (n + 15) / 16,
                       (n + 3) / 4,
                       D.Md,
                       reinterpret_cast<const int32_t *>(b + o_tile0),
                       reinterpret_cast<const int32_t *>(b + o_src),
                       reinterpret_cast<const uint4 *>(b + o_EAb),
                       reinterpret_cast<const double *>(b + o_EAd),
                       reinterpret_cast<const uint4 *>(b + o_CBb),
                       reinterpret_cast<const double *>(b + o_CBd),
                       reinterpret_cast<const double *>(b + o_W),
                       std::all_of(D.W.begin(), D.W.end(),
                                   [](double v) { return (double)(float)v == v; }) ? 1 : 0};
  }
  *out = h;
  return HOM_OK;
}

int hom_create_batch(int num_sys, const hom_sys_desc *descs, int flags, hom_system_t *out) {
  g_err.clear();
  if (!out) HOM_FAIL(HOM_EINVAL, "hom_create_batch: out is NULL");
  *out = nullptr;
  if (flags != 0) HOM_FAIL(HOM_EINVAL, "hom_create_batch: flags must be 0");
  if (num_sys < 1 || num_sys > 65536 || !descs)
    HOM_FAIL(HOM_EINVAL, "hom_create_batch: num_sys must be in [1, 65536] with descs non-NULL");
  std::vector<BatchSysDev> info(num_sys);
  std::vector<double> T_all;
  std::vector<int32_t> ints_all;
  int64_t c_acc = 0, C_acc = 0;
  int n_max = 0, mmax_all = 0;
  size_t lds_max = 0;
  for (int q = 0; q < num_sys; ++q) {
    const hom_sys_desc &d = descs[q];
    int64_t M = 0;
    int mmax = 0;
    const std::string bad = validate_system(d.n, d.m, d.A, d.w, &M, &mmax);
    if (!bad.empty())
      HOM_FAIL(HOM_EINVAL, "hom_create_batch: system " + std::to_string(q) + ": " + bad);
    const int N = bucket_for(d.n);
    std::vector<double> T;
    std::vector<int32_t> off;
    build_table(d.n, N, d.m, d.A, d.w, mmax, T, off);
    const size_t lds = lds_for(N, d.n, mmax);
    BatchSysDev &b = info[q];
    b.n = d.n;
    b.N = N;
    b.mmax = mmax;
    b.M = (int)M;
    b.T_off = (int64_t)T_all.size();
    b.ints_off = (int64_t)ints_all.size();
    b.c_off = c_acc;
    b.C_off = C_acc;
    b.lds_bytes = lds <= kMaxLds ? (int)lds : 0;
    b.pad = 0;
    if (b.lds_bytes > 0 && lds > lds_max) lds_max = lds;
    T_all.insert(T_all.end(), T.begin(), T.end());
    ints_all.insert(ints_all.end(), d.m, d.m + d.n);
    ints_all.insert(ints_all.end(), off.begin(), off.end());
    c_acc += M;
    C_acc += (int64_t)mmax * d.n;
    if (d.n > n_max) n_max = d.n;
    if (mmax > mmax_all) mmax_all = mmax;
  }
  hom_system_s *h = new hom_system_s();
  System &S = h->s;
  S.n = n_max;
  S.N = bucket_for(n_max);
  S.mmax = mmax_all;
  S.M = (int)std::min<int64_t>(c_acc, INT32_MAX);
  S.M_total = c_acc;
  S.num_sys = num_sys;
  S.C_total = C_acc;
  S.batch_lds = lds_max;
  auto fail = [&](hipError_t e, const char *what) {
    set_error(std::string("hom_create_batch: ") + what + ": " + hipGetErrorString(e));
    free_system(S);
    delete h;
    return e == hipErrorOutOfMemory ? HOM_ENOMEM : HOM_EDEVICE;
  };
  hipError_t e;
  if ((e = hipGetDevice(&S.device)) != hipSuccess) return fail(e, "hipGetDevice");
  if ((e = hipMalloc(&S.dBatch, info.size() * sizeof(BatchSysDev))) != hipSuccess)
    return fail(e, "hipMalloc");
  if ((e = hipMalloc(&S.dT_all, T_all.size() * 8)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = hipMalloc(&S.dInts_all, ints_all.size() * 4)) != hipSuccess) return fail(e, "hipMalloc");
  if ((e = hipMemcpy(S.dBatch, info.data(), info.size() * sizeof(BatchSysDev),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e, "hipMemcpy");
  if ((e = hipMemcpy(S.dT_all, T_all.data(), T_all.size() * 8, hipMemcpyHostToDevice)) !=
      hipSuccess)
    return fail(e, "hipMemcpy");
  if ((e = hipMemcpy(S.dInts_all, ints_all.data(), ints_all.size() * 4, hipMemcpyHostToDevice)) !=
      hipSuccess)
    return fail(e, "hipMemcpy");
  *out = h;
  return HOM_OK;
}

int hom_destroy(hom_system_t h) {
  g_err.clear();
  if (!h) return HOM_OK;
  (void)hipDeviceSynchronize();
  free_system(h->s);
  delete h;
  return HOM_OK;
}

int hom_system_info(hom_system_t h, int *n, int64_t *M, int *m_max, int *num_sys) {
  g_err.clear();
  if (!h) HOM_FAIL(HOM_EINVAL, "hom_system_info: NULL handle");
  if (n) *n = h->s.n;
  if (M) *M = h->s.num_sys > 0 ? h->s.M_total : h->s.M;
  if (m_max) *m_max = h->s.mmax;
  if (num_sys) *num_sys = h->s.num_sys > 0 ? h->s.num_sys : 1;
  return HOM_OK;
}

int hom_eval(hom_system_t h, const double *c, int64_t P, const double *z, const double *s,
             double *G, double *logscale, int flags, hom_stream_t stream) {
  g_err.clear();
  if (!h) HOM_FAIL(HOM_EINVAL, "hom_eval: NULL handle");
  if (h->s.projective) HOM_FAIL(HOM_EUNSUPPORTED, "hom_eval: projective handles support hom_step_proj only");
  if (h->s.num_sys > 0) HOM_FAIL(HOM_EUNSUPPORTED, "hom_eval: batch handles are supported by hom_track only");
  if (P < 0) HOM_FAIL(HOM_EINVAL, "hom_eval: P < 0");
  if (flags & ~15) HOM_FAIL(HOM_EINVAL, "hom_eval: unknown flags");
  if (P == 0) return HOM_OK;
  if (!c || !z || !s || !G) HOM_FAIL(HOM_EINVAL, "hom_eval: NULL array");
  hipStream_t st = (hipStream_t)stream;
  if (h->s.has_dense() && !(flags & HOM_EVAL_VALU)) {  // matrix-core engines
    const int engine = (flags & HOM_EVAL_FP32) ? 1 : 0;
    void *dws = nullptr;
    HOM_HIP(hipMallocAsync(&dws, dense_ws_bytes(h->s, P, false, engine), st),
            "hom_eval: workspace");
    hipError_t e = launch_dense_eval(h->s, c, P, z, s, G, logscale, flags & 3, engine, dws, st);
    hipError_t e2 = hipFreeAsync(dws, st);
    HOM_HIP(e, "hom_eval");
    HOM_HIP(e2, "hom_eval: free workspace");
    return HOM_OK;
  }
  void *cws = nullptr;
  hipError_t e = coeff_begin(h->s, c, st, &cws);
  if (e == hipSuccess) e = launch_eval(h->s, cws, c, P, z, s, G, logscale, flags & 7, st);
  hipError_t e2 = coeff_end(cws, st);
  HOM_HIP(e, "hom_eval");
  HOM_HIP(e2, "hom_eval: free workspace");
  return HOM_OK;
}

int hom_step(hom_system_t h, const double *c, int64_t P, const double *z, const double *s,
             double *dz_euler, double *dz_newton, int32_t *status, int precision,
             hom_stream_t stream) {
  g_err.clear();
  if (!h) HOM_FAIL(HOM_EINVAL, "hom_step: NULL handle");
  if (h->s.projective) HOM_FAIL(HOM_EUNSUPPORTED, "hom_step: projective handles support hom_step_proj only");
  if (h->s.num_sys > 0) HOM_FAIL(HOM_EUNSUPPORTED, "hom_step: batch handles are supported by hom_track only");
  if (P < 0) HOM_FAIL(HOM_EINVAL, "hom_step: P < 0");
  if (precision != HOM_FP64 && precision != HOM_MIXED)
    HOM_FAIL(HOM_EINVAL, "hom_step: precision must be HOM_FP64 or HOM_MIXED");
  if (P == 0) return HOM_OK;
  if (!c || !z || !s || !dz_euler || !dz_newton || !status)
    HOM_FAIL(HOM_EINVAL, "hom_step: NULL array");
  hipStream_t st = (hipStream_t)stream;
  void *cws = nullptr, *dws = nullptr;
  hipError_t e = coeff_begin(h->s, c, st, &cws);
  if (h->s.has_dense()) {  // matrix-core evaluation, then the LU on the stored rows
    if (e == hipSuccess)
      e = hipMallocAsync(&dws, dense_ws_bytes(h->s, P, true, precision == HOM_MIXED ? 1 : 0), st);
    if (e == hipSuccess)
      e = launch_dense_step(h->s, cws, c, P, z, s, dz_euler, dz_newton, status, precision, dws,
                            st);
  } else if (e == hipSuccess) {
    e = launch_step(h->s, cws, c, P, z, s, dz_euler, dz_newton, status, precision, st);
  }
  hipError_t e2 = coeff_end(cws, st);
  hipError_t e3 = dws ? hipFreeAsync(dws, st) : hipSuccess;
  HOM_HIP(e, "hom_step");
  HOM_HIP(e2, "hom_step: free workspace");
  HOM_HIP(e3, "hom_step: free workspace");
  return HOM_OK;
}

int hom_step_proj(hom_system_t h, const double *c, int64_t P, const double *y, const double *s,
                  double *dy_euler, double *dy_newton, int32_t *status, hom_stream_t stream) {
  g_err.clear();
  if (!h) HOM_FAIL(HOM_EINVAL, "hom_step_proj: NULL handle");
  if (!h->s.projective)
    HOM_FAIL(HOM_EUNSUPPORTED, "hom_step_proj: needs a handle created with HOM_CREATE_PROJECTIVE");
  if (P < 0) HOM_FAIL(HOM_EINVAL, "hom_step_proj: P < 0");
  if (P == 0) return HOM_OK;
  if (!c || !y || !s || !dy_euler || !dy_newton || !status)
    HOM_FAIL(HOM_EINVAL, "hom_step_proj: NULL array");
  hipStream_t st = (hipStream_t)stream;
  void *cws = nullptr;
  hipError_t e = coeff_begin(h->s, c, st, &cws);
  if (e == hipSuccess)
    e = launch_step_proj(h->s, cws, c, P, y, s, dy_euler, dy_newton, status, st);
  hipError_t e2 = coeff_end(cws, st);
  HOM_HIP(e, "hom_step_proj");
  HOM_HIP(e2, "hom_step_proj: free workspace");
  return HOM_OK;
}

int hom_track_params_default(hom_track_params *p, int precision) {
  g_err.clear();
  if (!p) HOM_FAIL(HOM_EINVAL, "hom_track_params_default: NULL");
  if (precision != HOM_FP64 && precision != HOM_MIXED)
    HOM_FAIL(HOM_EINVAL, "hom_track_params_default: bad precision");
  p->ds0 = 0.05;
  p->ds_max = 0.5;
  p->ds_min = 1e-10;
  p->tol_polish = 1e-12;
  p->tol_track = precision == HOM_MIXED ? 1e-5 : 1e-8;
  p->tol_end = 1e-14;
  p->res_tol = 1e-10;
  p->div_re = 40.0;
  p->sing_ratio = 1e-14;
  p->tol_predict = 1e-2;
  p->max_polish = 10;
  p->max_newton = 3;
  p->max_end = 8;
  p->max_steps = 100000;
  p->max_iters = 100000;
  p->precision = precision;
  p->flags = 0;
  p->tile = 0;
  p->predictor = HOM_PREDICT_EULER;
  return HOM_OK;
}

static TrackDev to_dev(const hom_track_params *p) {
  return TrackDev{p->ds0,        p->ds_max,     p->ds_min,  p->tol_polish, p->tol_track,
                  p->tol_end,    p->res_tol,    p->div_re,  p->sing_ratio, p->tol_predict,
                  p->max_polish,
                  p->max_newton, p->max_end,    p->max_steps, p->max_iters,
                  (p->flags & HOM_TRACK_EXACT_SHIFT) ? 1 : 0, p->tile, 3, 0, nullptr, nullptr,
                  0ull, 0, 0, 0ull, p->predictor};
}

// Checks of hom_track's arguments shared by its allocation-free variant.  Returns HOM_OK (then
// *nothing_to_do tells whether P == 0) or an error code with the message set.
static int check_track_args(const char *fn, hom_system_t h, const double *c, int64_t P,
                            const double *z, const double *s, const double *ds,
                            const int32_t *sys_idx, const hom_track_params *params,
                            const int32_t *status, const int32_t *counters, bool *nothing_to_do) {
  const std::string f(fn);
  *nothing_to_do = false;
  if (!h) HOM_FAIL(HOM_EINVAL, f + ": NULL handle");
  if (h->s.projective) HOM_FAIL(HOM_EUNSUPPORTED, f + ": projective handles support hom_step_proj only");
  if (P < 0) HOM_FAIL(HOM_EINVAL, f + ": P < 0");
  if (!params) HOM_FAIL(HOM_EINVAL, f + ": NULL params");
  const bool batch = h->s.num_sys > 0;
  if (!batch && sys_idx)
    HOM_FAIL(HOM_EINVAL, f + ": sys_idx must be NULL for a single-system handle");
  if (batch && P > 0 && !sys_idx) HOM_FAIL(HOM_EINVAL, f + ": a batch handle needs sys_idx");
  if (params->precision != HOM_FP64 && params->precision != HOM_MIXED)
    HOM_FAIL(HOM_EINVAL, f + ": bad precision");
  if (!(params->ds0 > 0) || !(params->ds_max > 0) || !(params->ds_min >= 0) ||
      !(params->tol_predict > 0) ||
      params->max_newton < 1 || params->max_end < 1 || params->max_polish < 1 ||
      params->max_steps < 0 || params->max_iters < 1 ||
      (params->flags & ~(HOM_TRACK_EXACT_SHIFT | HOM_TRACK_SERIAL | HOM_TRACK_SIDE_NOWAIT)) ||
      params->tile < 0 ||
      (params->predictor != HOM_PREDICT_EULER && params->predictor != HOM_PREDICT_HERMITE &&
       params->predictor != HOM_PREDICT_RK4))
    HOM_FAIL(HOM_EINVAL, f + ": bad params");
  if (P == 0) {
    *nothing_to_do = true;
    return HOM_OK;
  }
  if (!c || !z || !s || !ds || !status || !counters) HOM_FAIL(HOM_EINVAL, f + ": NULL array");
  return HOM_OK;
}

int hom_track(hom_system_t h, const double *c, int64_t P, double *z, double *s, double *ds,
              const int32_t *sys_idx, const hom_track_params *params, int32_t *status,
              int32_t *counters, hom_stream_t stream) {
  g_err.clear();
  bool none = false;
  const int rc = check_track_args("hom_track", h, c, P, z, s, ds, sys_idx, params, status,
                                  counters, &none);
  if (rc != HOM_OK || none) return rc;
  const bool batch = h->s.num_sys > 0;
  hipStream_t st = (hipStream_t)stream;
  const TrackDev pr = to_dev(params);
  const bool mixed = params->precision == HOM_MIXED;
  // The mixed form runs three launches: FP64 polish of the fresh paths, FP32 tracking of the
  // running paths (which parks the paths that need FP64, and every endgame), FP64 for the parked
  // paths.  The FP64 form runs one.
  TrackDev pr_pol = pr, pr32 = pr, pr64 = pr;
  pr_pol.claim = 1;
  pr_pol.polish_only = 1;
  pr32.claim = 2;
  pr64.claim = 4 | 8;
  hipError_t e = hipSuccess;
  if (batch) {
    // workspace: queue counter, per-system path and item offsets, table-order coefficients
    void *ws = nullptr;
    HOM_HIP(hipMallocAsync(&ws, track_batch_ws_bytes(h->s), st), "hom_track: workspace");
    if (!mixed) {
      e = launch_track_batch(h->s, c, P, z, s, ds, sys_idx, status, counters, pr, false, ws, st);
    } else {
      e = launch_track_batch(h->s, c, P, z, s, ds, sys_idx, status, counters, pr_pol, false, ws,
                             st);
      if (e == hipSuccess)
        e = launch_track_batch(h->s, c, P, z, s, ds, sys_idx, status, counters, pr32, true, ws, st);
      if (e == hipSuccess)
        e = launch_track_batch(h->s, c, P, z, s, ds, sys_idx, status, counters, pr64, false, ws,
                               st);
    }
    hipError_t e2 = hipFreeAsync(ws, st);
    if (e != hipSuccess) HOM_HIP(e, "hom_track");
    HOM_HIP(e2, "hom_track: free workspace");
    return HOM_OK;
  }
  // The mixed form's re-tracks run beside the FP32 launch unless asked not to or captured.
  hipStream_t side = nullptr;
  if (mixed && !(params->flags & HOM_TRACK_SERIAL)) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HOM_HIP(hipStreamIsCapturing(st, &cs), "hom_track: capture status");
    if (cs == hipStreamCaptureStatusNone) HOM_HIP(side_stream(&side), "hom_track: second stream");
  }
  // workspace: work-queue counters [0] (this stream's launches) and [1] (the side launch), the
  // park list's counters [2..5] and, with a side launch, the park list (P entries)
  const size_t ws_bytes = 256 + (side ? (size_t)P * sizeof(long long) : 0);
  unsigned long long *queue = nullptr;
  HOM_HIP(hipMallocAsync((void **)&queue, ws_bytes, st), "hom_track: workspace");
  long long *plist = side ? reinterpret_cast<long long *>(reinterpret_cast<char *>(queue) + 256)
                          : nullptr;
  void *cws = nullptr;
  e = coeff_begin(h->s, c, st, &cws);
  if (e == hipSuccess && !mixed)
    e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, pr, false, queue, st);
  if (e == hipSuccess && mixed)
    e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, pr_pol, false, queue, st);
  hipEvent_t fork = nullptr, join = nullptr;
  if (e == hipSuccess && side) {
    e = launch_fill_i64(reinterpret_cast<long long *>(queue + 2), 0, 4, st);
    if (e == hipSuccess) e = launch_fill_i64(plist, -1, P, st);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(fork, st);
    pr32.plist = plist;
    pr32.pctr = queue + 2;
  }
  int64_t waves32 = 0;
  if (e == hipSuccess && mixed)
    e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, pr32, true, queue, st, 0,
                     &waves32);
  if (e == hipSuccess && side) {  // the FP64 re-tracks beside the FP32 launch
    TrackDev prh = pr;
    prh.claim = 0;
    prh.helper = 1;
    prh.plist = plist;
    prh.pctr = queue + 2;
    prh.fp32_waves = (unsigned long long)waves32;
    prh.patience = (params->flags & HOM_TRACK_SIDE_NOWAIT) ? 0ull : kSidePatience;
    // Once the side launch may be queued, the call's stream must not free the workspace (or
    // reuse the coefficient tables) before it ends, whatever fails afterwards: the stream waits
    // for `join`, or, if that event could not be recorded, the host waits for the side stream.
    bool side_queued = false, joined = false;
    e = hipStreamWaitEvent(side, fork, 0);
    if (e == hipSuccess) {
      side_queued = true;
      e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, prh, false, queue + 1, side,
                       kSideBlocks);
      const hipError_t er = hipEventRecord(join, side);
      joined = er == hipSuccess;
      if (e == hipSuccess) e = er;
    }
    // the endgames meanwhile (disjoint from the re-tracks), then whatever re-track the side
    // launch left (none unless it stopped waiting)
    TrackDev pr_end = pr64, pr_left = pr64;
    pr_end.claim = 8;
    pr_left.claim = 4;
    pr_left.pctr = queue + 2;
    pr_left.drained_exit = 1;
    if (e == hipSuccess)
      e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, pr_end, false, queue, st);
    if (side_queued) {
      const hipError_t ew = joined ? hipStreamWaitEvent(st, join, 0) : hipStreamSynchronize(side);
      if (e == hipSuccess) e = ew;
      if (ew != hipSuccess && joined) {  // the stream could not be ordered: wait on the host
        const hipError_t es = hipStreamSynchronize(side);
        if (e == hipSuccess) e = es;
      }
    }
    if (e == hipSuccess)
      e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, pr_left, false, queue, st);
  } else if (e == hipSuccess && mixed) {
    e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, pr64, false, queue, st);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (join) (void)hipEventDestroy(join);
  hipError_t e2 = coeff_end(cws, st);
  hipError_t e3 = hipFreeAsync(queue, st);
  HOM_HIP(e, "hom_track");
  HOM_HIP(e2, "hom_track: free workspace");
  HOM_HIP(e3, "hom_track: free workspace");
  return HOM_OK;
}

// ---- hom_track_noalloc: the tracker with the library's static device scratch ----
// The scratch array lives in this file.  Its name is a host-side stand-in in host code: kernels
// and copies get the device address that hipGetSymbolAddress returns, resolved once per device
// (with that device current) and kept.
static __device__ __align__(256) unsigned char scratch[HOM_NOALLOC_SCRATCH_BYTES];
static constexpr size_t kScratchCounters = 256;  // work-queue counters, then the coefficients

static hipError_t scratch_ptr(unsigned char **out) {
  static std::mutex mu;
  static unsigned char *ptrs[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptrs[dev] = static_cast<unsigned char *>(p);
  }
  *out = ptrs[dev];
  return hipSuccess;
}

int hom_track_noalloc(hom_system_t h, const double *c, int64_t P, double *z, double *s, double *ds,
                      const hom_track_params *params, int32_t *status, int32_t *counters,
                      hom_stream_t stream) {
  g_err.clear();
  if (h && h->s.num_sys > 0)
    HOM_FAIL(HOM_EUNSUPPORTED, "hom_track_noalloc: batch handles are not supported (hom_track)");
  bool none = false;
  const int rc = check_track_args("hom_track_noalloc", h, c, P, z, s, ds, nullptr, params, status,
                                  counters, &none);
  if (rc != HOM_OK || none) return rc;
  const size_t need = kScratchCounters + h->s.coeff_ws_bytes();
  if (need > (size_t)HOM_NOALLOC_SCRATCH_BYTES)
    HOM_FAIL(HOM_EUNSUPPORTED,
             "hom_track_noalloc: the system's coefficient table (" +
                 std::to_string(h->s.coeff_ws_bytes()) + " bytes) exceeds the static scratch of " +
                 std::to_string((size_t)HOM_NOALLOC_SCRATCH_BYTES - kScratchCounters) +
                 " bytes; use hom_track");
  unsigned char *base = nullptr;
  HOM_HIP(scratch_ptr(&base), "hom_track_noalloc: scratch address");
  hipStream_t st = (hipStream_t)stream;
  // no profiling records here: they would create events
  const bool prof = g_prof;
  g_prof = false;
  unsigned long long *queue = reinterpret_cast<unsigned long long *>(base);
  void *cws = h->s.global_tables ? static_cast<void *>(base + kScratchCounters) : nullptr;
  const TrackDev pr = to_dev(params);
  hipError_t e = hipSuccess;
  if (cws) e = launch_coeff_tables(h->s, c, cws, st);
  if (params->precision == HOM_FP64) {
    if (e == hipSuccess)
      e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, pr, false, queue, st);
  } else {  // the three launches of the mixed form in their serial order (no second stream)
    TrackDev pr_pol = pr, pr32 = pr, pr64 = pr;
    pr_pol.claim = 1;
    pr_pol.polish_only = 1;
    pr32.claim = 2;
    pr64.claim = 4 | 8;
    if (e == hipSuccess)
      e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, pr_pol, false, queue, st);
    if (e == hipSuccess)
      e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, pr32, true, queue, st);
    if (e == hipSuccess)
      e = launch_track(h->s, cws, c, P, z, s, ds, status, counters, pr64, false, queue, st);
  }
  g_prof = prof;
  HOM_HIP(e, "hom_track_noalloc");
  return HOM_OK;
}

int hom_endpoint_grad(hom_system_t h, const double *c, int64_t P, const double *z_end,
                      const double *grad_x, double *grad_c, int precision, hom_stream_t stream) {
  g_err.clear();
  if (!h) HOM_FAIL(HOM_EINVAL, "hom_endpoint_grad: NULL handle");
  if (h->s.projective) HOM_FAIL(HOM_EUNSUPPORTED, "hom_endpoint_grad: projective handles support hom_step_proj only");
  if (h->s.num_sys > 0) HOM_FAIL(HOM_EUNSUPPORTED, "hom_endpoint_grad: batch handles are supported by hom_track only");
  if (P < 0) HOM_FAIL(HOM_EINVAL, "hom_endpoint_grad: P < 0");
  if (precision != HOM_FP64 && precision != HOM_MIXED)
    HOM_FAIL(HOM_EINVAL, "hom_endpoint_grad: bad precision");
  if (!c || !grad_c || (P > 0 && (!z_end || !grad_x)))
    HOM_FAIL(HOM_EINVAL, "hom_endpoint_grad: NULL array");
  hipStream_t st = (hipStream_t)stream;
  const size_t elems = grad_work_elems(h->s, P);
  double *work = nullptr;
  HOM_HIP(hipMallocAsync((void **)&work, elems * 8, st), "hom_endpoint_grad: workspace");
  void *cws = nullptr;
  hipError_t e = coeff_begin(h->s, c, st, &cws);
  if (e == hipSuccess)
    e = launch_grad(h->s, cws, c, P, z_end, grad_x, grad_c, precision, work, elems, st);
  hipError_t e2 = coeff_end(cws, st);
  hipError_t e3 = hipFreeAsync(work, st);
  HOM_HIP(e, "hom_endpoint_grad");
  HOM_HIP(e2, "hom_endpoint_grad: free workspace");
  HOM_HIP(e3, "hom_endpoint_grad: free workspace");
  return HOM_OK;
}

}  // extern "C"
