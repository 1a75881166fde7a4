// Persistent predictor-corrector tracker (A6).
//
// Every lane group owns one path slot.  Each iteration every active slot does exactly one
// evaluation and one consolidated Euler/Newton solve (Sec. 6: the Euler and Newton directions
// come out of the same LU, so the data path is identical for predictor and corrector steps and
// only the scalar update branches).  The update then either applies the Newton step
// (corrector), accepts the point and predicts along the Euler direction, rejects and halves the
// step, or runs the endgame at s = 0.  A finished slot claims the next path from a device-wide
// counter, so slots stay full until the queue is empty.  Nothing returns to the host per step.
//
// Step control (the paper fixes none; Sec. 8 only times a fixed Euler + Newton protocol):
//   polish   : Newton at the start point until ||dN|| <= tol_polish (max_polish iterations);
//   corrector: converged when ||dN|| <= tol_track: the evaluated point is accepted, and the
//              step doubles (up to ds_max) when it took at most one correction;
//              otherwise apply dN while k < max_newton and ||dN|| contracts by 1/2, else reject;
//   reject   : ds /= 2 (fail below ds_min) and predict again from the last accepted point;
//   predict  : z = z_a + h dE_a, s = s_a + h, h = min(ds, -s_a);
//   endgame  : at s = 0 Newton until ||dN|| <= tol_end (1 + ||z||), max_end iterations, or the
//              step stops contracting; OK when the relative residual <= res_tol.
// The CPU oracle runs the same rules with the same constants.
//
// Mixed form: the evaluation (exponentials, contraction) and the LU run in FP32; the exponent
// sums, the state z, s and every decision stay FP64.  A path that reaches s = 0 stops with an
// internal pending status and the FP64 launch that follows runs its endgame.  A path the mixed
// form fails (e.g. pivots below FP32 resolution) continues in FP64 from its last accepted point,
// or is re-tracked from its start when it failed before accepting any point.
#include <stdio.h>

#include "hom_internal.h"

namespace hom {

constexpr int kTrackBlock = 256;

enum : int { PH_POLISH = 0, PH_TRACK = 1, PH_END = 2, PH_RESUME = 3 };
enum : int { ACT_NONE = 0, ACT_REJECT = 1, ACT_PREDICT = 2, ACT_END = 3 };

template <int N>
__host__ __device__ constexpr size_t track_state_bytes() {
  return (size_t)(kTrackBlock / 64) * Geo<N>::G * 4 * N * sizeof(Cx<double>);
}

// At most 256 registers per lane, so two waves share each SIMD (the FP64 form at n = 10 needs
// slightly more than 256 without the bound and would run one wave per SIMD).
template <int N, bool MIXED>
__global__ void __launch_bounds__(kTrackBlock) __attribute__((amdgpu_waves_per_eu(2)))
    k_track(SysDev sd, const double *__restrict__ c, int64_t P, double *__restrict__ z,
            double *__restrict__ s, double *__restrict__ ds_io, int32_t *__restrict__ status,
            int32_t *__restrict__ counters, TrackDev pr, unsigned long long *__restrict__ queue,
            size_t table_bytes, unsigned long long *__restrict__ units) {
  extern __shared__ __align__(16) char smem[];
  const SysLds<N> S = stage_tables<N>(smem, sd, c);
  const Geo<N> geo;
  const int n = sd.n, r = geo.r;
  // per-group state in LDS: accepted point, Euler direction there, current dE and dN
  const int slot = (threadIdx.x >> 6) * Geo<N>::G + (geo.valid ? geo.g : 0);
  Cx<double> *sZa = reinterpret_cast<Cx<double> *>(smem + table_bytes) + slot * 4 * N;
  Cx<double> *sEa = sZa + N;
  Cx<double> *sEc = sZa + 2 * N;
  Cx<double> *sNc = sZa + 3 * N;

  double zr[N], zi[N];  // the path's point, replicated in every lane of the group
  double zo_r = 0.0, zo_i = 0.0;  // this lane's own coordinate z_r (same bits as zr[r], zi[r])
  double sc = 0.0, sa = 0.0, ds = 0.0, nrm_prev = 0.0;
  int64_t path = -1;
  int phase = PH_POLISH, k = 0, steps_here = 0, iters = 0;
  bool has_acc = false;  // the slot's path has an accepted point (sZa, sEa, sa valid)
  bool need_exact = true;  // next evaluation recomputes the row maximum (fresh path, lost lag)
  double Mlag = 0.0;       // this lane's row maximum from the previous evaluation
  int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  bool exhausted = !geo.valid;
#pragma unroll
  for (int j = 0; j < N; ++j) zr[j] = zi[j] = 0.0;

  for (;;) {
    // ---- claim paths for idle slots (wave-uniform loop: it shuffles) ----
    bool need = !exhausted && path < 0;
    while (__any(need)) {
      unsigned long long cl = 0;
      if (need && r == 0) cl = atomicAdd(queue, 1ull);
      cl = __shfl(cl, geo.base, 64);
      if (need) {
        // claims [0, P) take paths with a full or partial track ahead (fresh, resumed, handed
        // over from the mixed form); claims [P, 2P) take the short pending endgames, so that the
        // few long paths start first instead of forming the tail of the launch
        const int64_t lim = MIXED ? P : 2 * P;
        if ((int64_t)cl >= lim) {
          exhausted = true;
          need = false;
        } else {
          const bool second = (int64_t)cl >= P;
          const int64_t p = second ? (int64_t)cl - P : (int64_t)cl;
          const int st = status[p];
          const bool fresh = !second && st == 1, pend = second && st == kPendingEnd;
          const bool resume = !second && (st == 2 || (st == kHandoff && !MIXED));
          if ((fresh || resume) || (pend && !MIXED)) {
            path = p;
            need = false;
#pragma unroll
            for (int j = 0; j < N; ++j) {
              zr[j] = j < n ? z[2 * (p * n + j)] : 0.0;
              zi[j] = j < n ? z[2 * (p * n + j) + 1] : 0.0;
            }
            zo_r = r < n ? z[2 * (p * n + r)] : 0.0;
            zo_i = r < n ? z[2 * (p * n + r) + 1] : 0.0;
            sc = s[p];
            sa = sc;
            ds = fresh ? pr.ds0 : ds_io[p];
            phase = fresh ? PH_POLISH : (resume ? PH_RESUME : PH_END);
            k = 0;
            steps_here = 0;
            iters = 0;
            nrm_prev = 0.0;
            has_acc = false;
            need_exact = true;  // also always true with pr.exact_shift
            c0 = counters[4 * p];
            c1 = counters[4 * p + 1];
            c2 = counters[4 * p + 2];
            c3 = counters[4 * p + 3];
          }
        }
      }
    }
    if (__all(exhausted)) break;
    const bool active = path >= 0;

    // ---- one evaluation + consolidated solve (every lane) ----
    double nE, nN, resid, ratio;
    Cx<double> e, q;
    bool sing, shift_ok;
    {
      double M;
      if constexpr (MIXED) {
        Cx<float> row[N + 2], ef, qf;
        float absum, rf;
        shift_ok = eval_row<N, float>(S, r, zr, zi, sc, row, M, absum, Mlag, need_exact);
        const float h2 = (row[N + 1].x * row[N + 1].x + row[N + 1].y * row[N + 1].y) * fast_rcp(absum * absum);
        sing = lu_solve2<N, float>(row, r, geo.base, n, ef, qf, nE, nN, rf);
        resid = group_max<N, double>((double)h2, r, geo.base);  // squared
        e = {ef.x, ef.y};
        q = {qf.x, qf.y};
        ratio = rf;
      } else {
        Cx<double> row[N + 2];
        double absum;
        shift_ok = eval_row<N, double>(S, r, zr, zi, sc, row, M, absum, Mlag, need_exact);
        const double h2 = (row[N + 1].x * row[N + 1].x + row[N + 1].y * row[N + 1].y) * fast_rcp(absum * absum);
        sing = lu_solve2<N, double>(row, r, geo.base, n, e, q, nE, nN, ratio);
        resid = group_max<N, double>(h2, r, geo.base);  // squared relative residual
      }
    }
    // every lane of the group must have kept its terms in range, else redo with exact shifts
    const bool group_shift_ok = group_max_u32<N>(shift_ok ? 0u : 1u, r, geo.base) == 0u;
    if (geo.valid) {  // lanes past the last full group own no slot
      sEc[r] = e;
      sNc[r] = q;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();

    if (!active) continue;
    need_exact = !group_shift_ok || pr.exact_shift;
    if (!group_shift_ok) continue;  // discard this evaluation; the next one uses exact shifts

    // ---- scalar update of the slot (divergent across groups, identical within a group) ----
    bool fin = false;
    int fst = 0;
    if (iters >= pr.max_iters) {
      fin = true;
      fst = -7;
    } else {
      ++iters;
      ++c3;
      const double nrm = nN;
      // the mixed form cannot resolve pivots below FP32's precision, nor polish below its
      // tracking tolerance: such points are rejected, or the path fails and is re-tracked in FP64
      const double sing_ratio = MIXED ? fmax(pr.sing_ratio, 1e-7) : pr.sing_ratio;
      const double tol_polish = MIXED ? fmax(pr.tol_polish, pr.tol_track) : pr.tol_polish;
      const bool bad_lu = sing || !(ratio >= sing_ratio);
      const bool nonfin = !(nN <= INFINITY) || !(nE <= INFINITY);
      int act = ACT_NONE;
      if (bad_lu || nonfin) {
        if (phase == PH_TRACK) {
          act = ACT_REJECT;
        } else {
          fin = true;
          fst = bad_lu ? -1 : -4;
        }
      } else if (phase == PH_POLISH) {
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j < n) {
            zr[j] += sNc[j].x;
            zi[j] += sNc[j].y;
          }
        zo_r += q.x;
        zo_i += q.y;
        ++k;
        ++c2;
        if (nrm <= tol_polish) {
          phase = PH_RESUME;
          k = 0;
        } else if (k >= pr.max_polish) {
          fin = true;
          fst = -5;
        }
      } else if (phase == PH_RESUME || (phase == PH_TRACK && nrm <= pr.tol_track)) {
        if (phase == PH_TRACK) {
          ++c0;
          ++steps_here;
          if (k <= 1) ds = fmin(2.0 * ds, pr.ds_max);
        }
        sZa[r] = Cx<double>{zo_r, zo_i};
        sEa[r] = e;
        sa = sc;
        has_acc = true;
        if (sa >= 0.0) {
          phase = PH_END;
          k = 0;
          act = ACT_END;
        } else if (steps_here >= pr.max_steps) {
          fin = true;
          fst = 2;  // RUNNING
        } else {
          act = ACT_PREDICT;
        }
      } else if (phase == PH_END) {
        act = ACT_END;
      } else {  // corrector not converged yet
        if (k < pr.max_newton && (k == 0 || nrm <= 0.5 * nrm_prev)) {
          bool div = false;
#pragma unroll
          for (int j = 0; j < N; ++j)
            if (j < n) {
              zr[j] += sNc[j].x;
              zi[j] += sNc[j].y;
              div |= fabs(zr[j]) > pr.div_re;
            }
          zo_r += q.x;
          zo_i += q.y;
          ++k;
          ++c2;
          nrm_prev = nrm;
          if (div) {
            fin = true;
            fst = -3;
          }
        } else {
          act = ACT_REJECT;
        }
      }
      if (act == ACT_REJECT) {
        ++c1;
        ds *= 0.5;
        if (ds < pr.ds_min) {
          fin = true;
          fst = -2;
          // the reported point is the last accepted one
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
#pragma unroll
          for (int j = 0; j < N; ++j)
            if (j < n) {
              zr[j] = sZa[j].x;
              zi[j] = sZa[j].y;
            }
          if (geo.valid) {
            zo_r = sZa[r].x;
            zo_i = sZa[r].y;
          }
          sc = sa;
        } else {
          act = ACT_PREDICT;
        }
      }
      if (act == ACT_PREDICT) {
        const double hstep = fmin(ds, -sa);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
#pragma unroll
        for (int j = 0; j < N; ++j)
          if (j < n) {
            const Cx<double> za = sZa[j], ea = sEa[j];
            zr[j] = fma(hstep, ea.x, za.x);
            zi[j] = fma(hstep, ea.y, za.y);
          }
        if (geo.valid) {
          const Cx<double> za = sZa[r], ea = sEa[r];
          zo_r = fma(hstep, ea.x, za.x);
          zo_i = fma(hstep, ea.y, za.y);
        }
        sc = (hstep == -sa) ? 0.0 : sa + hstep;
        k = 0;
        phase = PH_TRACK;
      }
      if (act == ACT_END) {
        if (MIXED) {
          fin = true;
          fst = kPendingEnd;  // FP64 endgame runs in the following launch
        } else {
          double zn2 = 0.0;
#pragma unroll
          for (int j = 0; j < N; ++j)
            if (j < n) {
              zr[j] += sNc[j].x;
              zi[j] += sNc[j].y;
              const double a = zr[j] * zr[j] + zi[j] * zi[j];
              zn2 = (a > zn2 || a != a) ? a : zn2;
            }
          const double zn = sqrt(zn2);
          zo_r += q.x;
          zo_i += q.y;
          ++c2;
          ++k;
          if (nrm <= pr.tol_end * (1.0 + zn) || k >= pr.max_end || (k >= 3 && nrm > 0.5 * nrm_prev)) {
            fin = true;
            fst = (resid <= pr.res_tol * pr.res_tol) ? 0 : -6;
          } else {
            nrm_prev = nrm;
          }
        }
      }
    }
    if (MIXED && fin && fst < 0 && fst != -7 && has_acc) {
      // hand the path to the FP64 pass at its last accepted point
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      zo_r = sZa[r < N ? r : 0].x;
      zo_i = sZa[r < N ? r : 0].y;
      sc = sa;
      ds = pr.ds0;
      fst = kHandoff;
    }
    if (fin) {
      const int64_t p = path;
      if (r < n) {
        z[2 * (p * n + r)] = zo_r;
        z[2 * (p * n + r) + 1] = zo_i;
      }
      if (r == 0) {
        s[p] = sc;
        ds_io[p] = ds;
        status[p] = fst;
        counters[4 * p] = c0;
        counters[4 * p + 1] = c1;
        counters[4 * p + 2] = c2;
        counters[4 * p + 3] = c3;
        if (units) atomicAdd(units, (unsigned long long)iters);  // eval+solves of this launch
      }
      path = -1;
    }
  }
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

template <int N>
static hipError_t track_n(const System &S, const double *c, int64_t P, double *z, double *s,
                          double *ds, int32_t *status, int32_t *counters, const TrackDev &pr,
                          bool mixed, unsigned long long *queue, hipStream_t stream) {
  const size_t tb = (S.lds_bytes + 15) & ~(size_t)15;
  const size_t lds = tb + track_state_bytes<N>();
  auto kern = mixed ? k_track<N, true> : k_track<N, false>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kTrackBlock, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int64_t gpb = (kTrackBlock / 64) * Geo<N>::G;
  int64_t blocks = (int64_t)per_cu * num_cus();
  const int64_t need = (P + gpb - 1) / gpb;
  if (blocks > need) blocks = need > 0 ? need : 1;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, stream, queue);
  char label[64];
  snprintf(label, sizeof label, "k_track<%d,%s>", N, mixed ? "mixed" : "fp64");
  prof_begin(stream);
  unsigned long long *units = prof_units(stream);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kTrackBlock), lds, stream, S.dev(), c,
                     P, z, s, ds, status, counters, pr, queue, tb, units);
  prof_end(stream, label);
  return hipGetLastError();
}

#define HOM_SWITCH_T(N, CALL)            \
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

hipError_t launch_track(const System &S, const double *c, int64_t P, double *z, double *s,
                        double *ds, int32_t *status, int32_t *counters, const TrackDev &pr,
                        bool mixed, unsigned long long *queue, hipStream_t stream) {
  HOM_SWITCH_T(S.N, return track_n<NN>(S, c, P, z, s, ds, status, counters, pr, mixed, queue,
                                       stream))
}

}  // namespace hom
