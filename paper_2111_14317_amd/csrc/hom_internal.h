// Internal declarations shared by the C ABI and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hom.h"
#include "hom_device.h"

namespace hom {

// Compiled group sizes; a system with n unknowns runs on the smallest N >= n.
constexpr int kSizes[] = {2, 3, 4, 5, 6, 7, 8, 10, 12, 16, 20, 24, 32};
int bucket_for(int n);   // smallest compiled N >= n, or 0
int table_ld(int N);     // TableLD<N>::value at run time

// One system of a batch handle, as the batch kernel sees it.
struct BatchSysDev {
  int n, N, mmax, M;
  int64_t T_off;     // offset (doubles) of the exponent table in the batch's table buffer
  int64_t ints_off;  // offset of m_k [n] then the equation offsets [n] in the int buffer
  int64_t c_off;     // first coefficient (complex index) in the concatenated c
  int64_t C_off;     // offset of the table-order coefficients in the per-call workspace
  int lds_bytes;     // LDS image of the tables, or 0 when they are read from global memory
  int pad;
};

// Matrix-core tables of a dense-support system (built by hom_create when the largest m_k is at
// least kDenseMinM).  Each equation's monomials are padded to a multiple of 32 with copies of its
// first monomial (coefficient 0), so 16-monomial tiles and 32-monomial chunks never straddle two
// equations.  Lane layouts are those of the gfx950 16x16 MFMA operands.
constexpr int kDenseMinM = 32;
// LDS of one wave of the common-support engine: the point tile's exponentials (16 points x the
// padded support, complex double)
constexpr size_t kUnionLdsBytes = 64 * 1024;
struct DenseDev {
  int n;                 // unknowns
  int nct;               // 16-column tiles of the Jacobian (ceil(n / 16))
  int nks;               // K steps of 4 coordinates for the FP64 engine (ceil(n / 4))
  int Md;                // padded monomials
  const int32_t *tile0;  // [n + 1] first 16-monomial tile of equation k (tile0[n] = Md / 16)
  const int32_t *src;    // [Md] monomial index into c, or -1 for padding
  const uint4 *EAb;      // [Md/16][64] bf16x8: exponents a[16t + l%16][8(l/16) + e] (A operand)
  const double *EAd;     // [Md/16][8][64]: a[16t + l%16][4ks + l/16] (FP64 A operand)
  const uint4 *CBb;      // [Md/32][2][64] bf16x8: exponent columns, bf16 engine B operand
  const double *CBd;     // [Md/16][4][2][64]: exponent columns, FP64 engine B operand
  const double *W;       // [Md] lifting
  int w_f32;             // every lifting is exactly a float (the BF16x3 engine stages them so)
};

struct System {
  int n = 0, N = 0, mmax = 0, M = 0;
  // batched form (num_sys > 0): n = largest n, M = total, mmax = largest m_k
  int num_sys = 0;
  BatchSysDev *dBatch = nullptr;     // device [num_sys]
  double *dT_all = nullptr;          // device tables of all systems
  int32_t *dInts_all = nullptr;      // device m_k and offsets of all systems
  int64_t C_total = 0;               // table-order coefficient entries over all systems
  int64_t M_total = 0;               // monomials over all systems
  size_t batch_lds = 0;              // largest LDS image among the systems staged in LDS
  int device = 0;
  double *dT = nullptr;     // device [mmax][n][LD] exponent table + lifting
  int32_t *dmk = nullptr;   // device [n]
  int32_t *doff = nullptr;  // device [n]
  int32_t *dA = nullptr;    // device [M][n] exponents as int32 (adjoint kernel)
  size_t lds_bytes = 0;     // LDS image of the tables; 0 when they stay in global memory
  bool global_tables = false;
  // projective handle (hom_create with HOM_CREATE_PROJECTIVE): n equations in n + 1 homogeneous
  // unknowns; the tables hold the homogenised exponents; N = proj_group_size(n)
  bool projective = false;
  // cws: this call's table-order coefficients (coeff_ws_bytes), for global_tables only
  SysDev dev(const void *cws = nullptr) const {
    const Cx<double> *Cg = global_tables ? static_cast<const Cx<double> *>(cws) : nullptr;
    const double *Ca = Cg ? reinterpret_cast<const double *>(Cg + (size_t)mmax * n) : nullptr;
    return SysDev{n, mmax, M, dT, dmk, doff, Cg, Ca};
  }
  size_t coeff_ws_bytes() const { return global_tables ? (size_t)mmax * n * 24 : 0; }
  // matrix-core tables (dense supports); null pointers when not built
  int Md = 0;
  void *dDense = nullptr;  // one allocation holding every DenseDev array
  DenseDev dense{};
  // union support (Sec. 5.1's unmixed case): every equation has the same monomials, in the same
  // order, with the same liftings; the dense FP64 engine then forms each point's exponentials once
  // and contracts them with every equation's coefficients (k_union_f64)
  bool union_support = false;
  int union_tiles = 0;  // 16-monomial tiles of the common support (padded to a multiple of 32)
  bool has_dense() const { return dDense != nullptr; }
};

// Tracker constants as the kernels see them.
struct TrackDev {
  double ds0, ds_max, ds_min, tol_polish, tol_track, tol_end, res_tol, div_re, sing_ratio,
      tol_predict;
  int max_polish, max_newton, max_end, max_steps, max_iters;
  int exact_shift;
  int tile;
  int claim;  // statuses a launch takes up: bit 0 fresh (1), bit 1 running (2), bit 2 parked
              // (3), bit 3 parked for the endgame (4)
  int polish_only;  // fresh paths stop RUNNING once polished (the mixed form's first launch)
  // Park list of the mixed form's FP32 launch, read by a concurrent FP64 launch (null: none).
  // plist[i] is the i-th path parked for a re-track (-1 until published); pctr[0] counts the
  // reserved entries, pctr[1] the helper's claims, pctr[2] the FP32 launch's finished waves,
  // pctr[3] the entries the helper took up (and tracked to their end).
  long long *plist;
  unsigned long long *pctr;
  unsigned long long fp32_waves;  // waves of the FP32 launch (all finished: no more entries)
  int helper;                     // this FP64 launch claims from the park list
  int drained_exit;  // launched after both: return at once when the helper took every entry
  // helper: ticks of the 100 MHz constant clock it waits without a sign of the FP32 launch's
  // progress (a new park-list entry, a finished wave) before it stops claiming; whatever it
  // leaves is re-tracked by the FP64 launch that follows both
  unsigned long long patience;
  int predictor;  // HOM_PREDICT_EULER or HOM_PREDICT_HERMITE
};
constexpr unsigned long long kSidePatience = 20000000ull;  // 0.2 s


void set_error(const std::string &msg);

// Kernel timing: when profiling is on for this thread, prof_begin/prof_end record a pair of
// events around a launch (no-ops otherwise).
// prof_units returns a zeroed device counter for the launch's work units (nullptr when off).
void prof_begin(hipStream_t stream);
unsigned long long *prof_units(hipStream_t stream);
void prof_end(hipStream_t stream, const char *label);

// launchers (return a hipError_t).  cws: the per-call coefficient workspace of a system with
// global tables (filled by launch_coeff_tables first), else null.
hipError_t launch_coeff_tables(const System &S, const double *c, void *cws, hipStream_t stream);
hipError_t launch_eval(const System &S, const void *cws, const double *c, int64_t P,
                       const double *z, const double *s, double *G, double *logscale, int flags,
                       hipStream_t stream);
hipError_t launch_step(const System &S, const void *cws, const double *c, int64_t P,
                       const double *z, const double *s, double *dE, double *dN,
                       int32_t *status, int precision, hipStream_t stream);
// blocks: the grid (0: as many blocks as fit on the device at once); waves_out (optional): the
// number of waves launched.
hipError_t launch_track(const System &S, const void *cws, const double *c, int64_t P, double *z,
                        double *s, double *ds, int32_t *status, int32_t *counters,
                        const TrackDev &pr, bool mixed, unsigned long long *queue,
                        hipStream_t stream, int blocks = 0, int64_t *waves_out = nullptr);
hipError_t launch_fill_i64(long long *p, long long v, int64_t n, hipStream_t stream);
hipError_t launch_track_batch(const System &S, const double *c, int64_t P, double *z, double *s,
                              double *ds, const int32_t *sys_idx, int32_t *status,
                              int32_t *counters, const TrackDev &pr, bool mixed, void *ws,
                              hipStream_t stream);
size_t track_batch_ws_bytes(const System &S);
hipError_t launch_grad(const System &S, const void *cws, const double *c, int64_t P,
                       const double *z_end,
                       const double *grad_x, double *grad_c, int precision, double *work,
                       size_t work_elems, hipStream_t stream);
size_t grad_work_elems(const System &S, int64_t P);

// Dense-support evaluation and step on the matrix cores.  engine: 0 = FP64 MFMA, 1 = BF16x3 MFMA
// with FP32 accumulation.  dws: dense_ws_bytes(S, P, step) bytes of workspace.
size_t dense_ws_bytes(const System &S, int64_t P, bool step, int engine);
hipError_t launch_dense_eval(const System &S, const double *c, int64_t P, const double *z,
                             const double *s, double *G, double *logscale, int flags, int engine,
                             void *dws, hipStream_t stream);
hipError_t launch_dense_step(const System &S, const void *cws, const double *c, int64_t P,
                             const double *z, const double *s, double *dE, double *dN,
                             int32_t *status, int precision, void *dws, hipStream_t stream);

// Projective step (hom_step_proj): group size for n equations (a power of two >= n + 3, or 0).
int proj_group_size(int n);
hipError_t launch_step_proj(const System &S, const void *cws, const double *c, int64_t P,
                            const double *y, const double *s, double *dE, double *dN,
                            int32_t *status, hipStream_t stream);

// number of compute units of the current device (cached)
int num_cus();

// Start points (k_start.hip).  Per cell of n unknowns (n <= 32): a plan record of
// start_record_words(n) int64 words (L, the count of invariant factors above one, z_base, their
// radices and V columns).
__host__ __device__ constexpr int64_t start_record_words(int n) {
  return 2 + 2 * (int64_t)n + n + (int64_t)n * n;
}
struct StartHdr {
  int64_t row0;   // first output row of the cell
  int64_t first;  // first root index
  int64_t count;  // roots written
};
hipError_t peak_probe(int kind, double *rate, hipStream_t stream);  // k_peak.hip
const char *start_status_text(int32_t status);  // "" for a cell planned without error
int start_status_code(int32_t status);          // HOM_EINVAL or HOM_EUNSUPPORTED
hipError_t launch_start_plan(int n, int64_t num_cells, const int32_t *D, const double *beta,
                             int64_t *rec, int32_t *status, int64_t *det, hipStream_t stream);
hipError_t launch_binomial_starts(int n, int num_cells, const StartHdr *hdr, const int64_t *rec,
                                  int64_t rows, double *z, hipStream_t stream);

}  // namespace hom
