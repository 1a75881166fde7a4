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
//   predicted point: rejected when its first ||dN|| exceeds tol_predict (it may lie nearer another
//              path than its own, where the corrector would converge to the wrong path);
//   corrector: converged when ||dN|| <= tol_track: the evaluated point is accepted, and the
//              step doubles (up to ds_max) when it took at most one correction;
//              otherwise apply dN while k < max_newton and ||dN|| contracts by 1/2, else reject;
//   reject   : ds /= 2 (fail below ds_min) and predict again from the last accepted point;
//   predict  : z = z_a + h dE_a, s = s_a + h, h = min(ds, -s_a) (Euler); or, with the Hermite
//              predictor, the cubic through the last two accepted points and their Euler
//              directions (when h <= 4 (s_a - s_p); the first step after a claim is Euler);
//              or the classical Runge-Kutta scheme on dz/ds = dE, its three stage points
//              evaluated one per iteration (phases PH_RK1..PH_RK3; a failed stage rejects the
//              step);
//   endgame  : at s = 0 Newton until ||dN|| <= tol_end (1 + ||z||), max_end iterations, or the
//              step stops contracting; OK when the relative residual <= res_tol.
// The CPU oracle runs the same rules with the same constants.
//
// Mixed form, three launches.  An FP64 launch polishes the fresh start points (and leaves them
// RUNNING).  The FP32 launch tracks: the evaluation (exponentials, contraction) and the LU run in
// FP32; the exponent sums, the state z, s and every decision stay FP64.  A failed FP32 evaluation
// at a predicted or corrected point (pivots below FP32's reach, non-finite values), or a
// correction that leaves the region |Re z| <= div_re, rejects the step like any failed
// correction.  A path whose FP32 evaluation fails at its accepted point, whose step falls below
// kMixedMinStep or that has kMixedFp64Rejects consecutive rejected steps is parked at its last
// accepted point (kParked: re-tracked in FP64 with a fresh step); one that reaches s = 0 is
// parked for its endgame (kParkedEnd).  A last FP64 launch finishes the parked paths: first the
// rest of the tracks, then the (short) endgames, so that long work does not form the launch's
// tail.  The FP32 launch holds no FP64 evaluation code, which keeps its register budget to the
// FP32 path: switching a group to FP64 inside the FP32 launch makes its whole wave run both
// precisions, and even an FP64 residual pass for the few paths that need it (FP32 LU, FP64
// residual) slowed the whole launch by a third through its register and code layout, both
// measured.
#include <stdio.h>

#include "hom_internal.h"

namespace hom {

constexpr int kTrackBlock = 256;

// PH_RK1..PH_RK3: evaluating the Runge-Kutta predictor's stage point 1..3
enum : int { PH_POLISH = 0, PH_TRACK = 1, PH_END = 2, PH_RESUME = 3, PH_RK1 = 4, PH_RK3 = 6 };
enum : int { ACT_NONE = 0, ACT_REJECT = 1, ACT_PREDICT = 2, ACT_END = 3 };

// mixed form: a path with this many consecutive rejected steps is handed to FP64.  Near an
// ill-conditioned point the FP32 Newton noise exceeds tol_track and halving the step cannot fix
// that; left in FP32 such a path creeps on with tiny steps until its iteration budget runs out.
constexpr int kMixedFp64Rejects = 10;
// ... and so is a path whose step falls below this (steps this small resolve nothing at the FP32
// Newton tolerance; a path alternating accepted and rejected steps never reaches the reject run)
constexpr double kMixedMinStep = 1e-6;
// statuses of paths parked by the FP32 launch of a mixed call (internal: the call's FP64 launch
// claims them, so they are never returned)
constexpr int kParked = 3;     // re-tracked in FP64 from its last accepted point
constexpr int kParkedEnd = 4;  // at s = 0: only its endgame is left

// LDS of the tracker's lane groups: 7 N complex values per group.
template <int N>
__host__ __device__ constexpr size_t track_state_bytes() {
  return (size_t)(kTrackBlock / 64) * Geo<N>::G * 7 * N * sizeof(Cx<double>);
}

// The group's current point, read from LDS into registers for one evaluation (so the replicas are
// dead during the LU, which matters for the register budget at large N).  Padding lanes store
// zeros there, so the entries past n need no masking; the FP64 tracker masks them anyway, which
// measured fewer register spills for its large groups.
template <int N, bool MASK>
__device__ __forceinline__ void load_point_lds(const Cx<double> *sZc, int n, double (&zr)[N],
                                               double (&zi)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const Cx<double> v = sZc[j];
    zr[j] = (!MASK || j < n) ? v.x : 0.0;
    zi[j] = (!MASK || j < n) ? v.y : 0.0;
  }
}

// The tracker loop of one block's lane groups over the paths [p_begin, p_end) of one system.
// Groups claim paths through `queue` (global memory for a whole launch, or LDS for one work item of
// the batched form).  Path p's point is z[p * zstride + j], j < n.  slot_state: LDS for the
// block's groups (track_state_bytes).
// RK: the Runge-Kutta predictor's phases are compiled in (the FP32 launch has a variant without
// them, launched unless that predictor is asked for).
template <int N, bool MIXED, bool RK = true>
__device__ __forceinline__ void track_slots(const SysLds<N> &S, int n, Cx<double> *slot_state,
                                            int64_t p_begin, int64_t p_end, int zstride,
                                            double *__restrict__ z, double *__restrict__ s,
                                            double *__restrict__ ds_io,
                                            int32_t *__restrict__ status,
                                            int32_t *__restrict__ counters, const TrackDev &pr,
                                            unsigned long long *queue,
                                            unsigned long long *__restrict__ units,
                                            const double *kcoef,
                                            const F32Tables<N> *ft = nullptr) {
  // The side launch's re-tracks are the mixed form's critical path once the FP32 launch drains:
  // its waves take issue priority over the FP32 launch's waves on the SIMDs they share.
  if (pr.helper) __builtin_amdgcn_s_setprio(2);
  const Geo<N> geo;
  const int r = geo.r;
  // per-group state in LDS: accepted point, Euler direction there, current dE and dN, current
  // point (each lane keeps its own coordinate in registers and writes it here)
  const int slot = (threadIdx.x >> 6) * Geo<N>::G + (geo.valid ? geo.g : 0);
  Cx<double> *sZa = slot_state + slot * 7 * N;
  Cx<double> *sEa = sZa + N;
  Cx<double> *sEc = sZa + 2 * N;
  Cx<double> *sNc = sZa + 3 * N;
  Cx<double> *sZc = sZa + 4 * N;
  Cx<double> *sZp = sZa + 5 * N;  // the accepted point before (z_a, s_a), and its Euler direction
  Cx<double> *sEp = sZa + 6 * N;  // (the Hermite predictor's second point)
  // the Runge-Kutta predictor's sum k1 + 2 k2 + 2 k3 + k4, in the Hermite predictor's slot (the
  // two are never used together; an acceptance overwrites it only after the stages are done)
  Cx<double> *sKs = sZp;
  const int64_t P = p_end - p_begin;

  double zo_r = 0.0, zo_i = 0.0;  // this lane's own coordinate z_r of the current point
  double sc = 0.0, sa = 0.0, ds = 0.0, nrm_prev = 0.0, sp = 0.0;
  bool have_p = false;  // (sZp, sEp, sp) hold an accepted point before (sZa, sEa, sa)
  int64_t path = -1;
  int phase = PH_POLISH, k = 0, steps_here = 0, iters = 0;
  bool need_exact = true;  // next evaluation recomputes the row maximum (fresh path, lost lag)
  double Mlag = 0.0;       // this lane's row maximum from the previous evaluation
  int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  int rej_run = 0;  // mixed form: consecutive rejected steps since the last accepted point
  bool exhausted = !geo.valid;

  // the path's state at a claim (fresh: polish from the start point; endgame: Newton at s = 0;
  // otherwise resumed from its last accepted point)
  auto begin_path = [&](int64_t p, bool fresh, bool endgame) {
    path = p;
    zo_r = r < n ? z[2 * (p * zstride + r)] : 0.0;
    zo_i = r < n ? z[2 * (p * zstride + r) + 1] : 0.0;
    sZc[r] = Cx<double>{zo_r, zo_i};
    sc = s[p];
    sa = sc;
    ds = fresh ? pr.ds0 : ds_io[p];
    have_p = false;
    phase = fresh ? PH_POLISH : (endgame ? PH_END : PH_RESUME);
    k = 0;
    steps_here = 0;
    iters = 0;
    nrm_prev = 0.0;
    need_exact = true;  // also always true with pr.exact_shift
    rej_run = 0;
    c0 = counters[4 * p];
    c1 = counters[4 * p + 1];
    c2 = counters[4 * p + 2];
    c3 = counters[4 * p + 3];
  };
  // helper launch (pr.helper): this group's claimed park-list index whose entry has not been
  // published yet, and the last change seen in the FP32 launch's progress
  long long pend = -1;
  unsigned long long seen = ~0ull, seen_at = 0;

  for (;;) {
    if (pr.helper) {
      // ---- claims from the park list of the concurrent FP32 launch (never blocks the wave) ----
      if (!exhausted && path < 0) {
        long long v = -1;
        int done = 0;
        if (r == 0) {
          if (pend < 0) pend = (long long)atomicAdd(&pr.pctr[1], 1ull);
          if (pend < P) v = __hip_atomic_load(&pr.plist[pend], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          if (v < 0) {
            const unsigned long long fin32 =
                __hip_atomic_load(&pr.pctr[2], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long tail =
                __hip_atomic_load(&pr.pctr[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            if (fin32 >= pr.fp32_waves) {  // no more entries: this one exists iff below the tail
              if ((unsigned long long)pend >= tail) done = 1;
              else v = __hip_atomic_load(&pr.plist[pend], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (v < 0 && !done) {  // give up after pr.patience without any change seen
              const unsigned long long now = wall_clock64(), mark = (fin32 << 32) ^ tail;
              if (mark != seen) {
                seen = mark;
                seen_at = now;
              } else if (now - seen_at > pr.patience) {
                done = 1;
              }
            }
          }
        }
        v = __shfl(v, geo.base, 64);
        done = __shfl(done, geo.base, 64);
        pend = __shfl(pend, geo.base, 64);
        if (v >= 0) {
          __threadfence();  // the parked path's state is read after its publication
          if (r == 0) atomicAdd(&pr.pctr[3], 1ull);
          begin_path(v, false, false);
          pend = -1;
        } else if (done) {
          exhausted = true;
        }
      }
      if (__all(exhausted)) break;
      if (!__any(path >= 0)) {  // nothing to track yet: wait for the FP32 launch to park more
        __builtin_amdgcn_s_sleep(32);
        continue;
      }
    }
    // ---- claim paths for idle slots (wave-uniform loop: it shuffles) ----
    bool need = !pr.helper && !exhausted && path < 0;
    while (__any(need)) {
      unsigned long long cl = 0;
      if (need && r == 0) cl = atomicAdd(queue, 1ull);
      cl = __shfl(cl, geo.base, 64);
      if (need) {
        // pr.claim: bit 0 fresh paths, bit 1 running ones, bit 2 parked ones (resumed), bit 3
        // parked endgames.  Endgames are claimed in a second sweep [P, 2P), after every longer
        // piece of work has started.
        const int64_t lim = (pr.claim & 8) ? 2 * P : P;
        if ((int64_t)cl >= lim) {
          exhausted = true;
          need = false;
        } else {
          const bool second = (int64_t)cl >= P;
          const int64_t p = p_begin + (second ? (int64_t)cl - P : (int64_t)cl);
          const int st = status[p];
          const bool fresh = !second && st == 1 && (pr.claim & 1);
          const bool resume = !second && ((st == 2 && (pr.claim & 2)) ||
                                          (st == kParked && (pr.claim & 4)));
          const bool endgame = second && st == kParkedEnd && (pr.claim & 8);
          if (fresh || resume || endgame) {
            need = false;
            begin_path(p, fresh, endgame);
          }
        }
      }
    }
    if (__all(exhausted)) break;
    const bool active = path >= 0;

    // ---- one evaluation + consolidated solve (every lane) ----
    // The mixed form's launch evaluates in FP32 only (its paths arrive polished in FP64).
    constexpr bool use64 = !MIXED;
    double nE = 0.0, nN = 0.0, resid = 0.0, ratio = 0.0;
    Cx<double> e = {0.0, 0.0}, q = {0.0, 0.0};
    bool sing = false, shift_ok = true;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // the group's sZc writes
    __builtin_amdgcn_wave_barrier();
    {
      const double Min = Mlag;
      double M;
      if constexpr (MIXED) {
        {
          Cx<float> row[N + 2], ef, qf;
          float absum, rf;
          double Ml = Min;
          double zr[N], zi[N];
          load_point_lds<N, !MIXED>(sZc, n, zr, zi);
          shift_ok = eval_row<N, float>(S, r, zr, zi, sc, row, M, absum, Ml, need_exact, ft);
          const float h2 = (row[N + 1].x * row[N + 1].x + row[N + 1].y * row[N + 1].y) * fast_rcp(absum * absum);
          sing = lu_solve2<N, float>(row, r, geo.base, n, ef, qf, nE, nN, rf);
          resid = group_max_nonneg<N>(h2, r, geo.base);
          e = {ef.x, ef.y};
          q = {qf.x, qf.y};
          ratio = rf;
          Mlag = Ml;
        }
      }
      if constexpr (!MIXED) {
        Cx<double> row[N + 2], ed, qd;
        double absum, rd, nEd, nNd, Ml = Min;
        bool okd;
        if constexpr (N >= 16) {
          // large groups: the point and the FP64 coefficients are read from LDS at each use,
          // since the FP64 row leaves no registers for them (C4's FP64 run: 17.0 -> 9.7 s); small
          // ones keep them in registers (read from LDS, the 10-lane FP64 tracker ran 1.6x slower)
          okd = eval_row_at<N, double>(S, r, PointLds{sZc}, sc, row, M, absum, Ml, need_exact,
                                       CoefLds{kcoef});
        } else {
          double zr[N], zi[N];
          load_point_lds<N, true>(sZc, n, zr, zi);
          okd = eval_row<N, double>(S, r, zr, zi, sc, row, M, absum, Ml, need_exact);
        }
        const double h2 = (row[N + 1].x * row[N + 1].x + row[N + 1].y * row[N + 1].y) * fast_rcp(absum * absum);
        const bool sd = lu_solve2<N, double>(row, r, geo.base, n, ed, qd, nEd, nNd, rd);
        const double resd = group_max<N, double>(h2, r, geo.base);  // squared relative residual
        e = ed;
        q = qd;
        sing = sd;
        ratio = rd;
        nE = nEd;
        nN = nNd;
        resid = resd;
        shift_ok = okd;
        Mlag = Ml;
      }
    }
    // group-wide flags in one reduction: every lane of the group must have kept its terms in
    // range (else redo with exact shifts), and the Newton update z + dN must stay in the region
    const double cre = zo_r + q.x, cim = zo_i + q.y;
    const uint32_t flags = group_or_u32<N>((shift_ok ? 0u : 1u) |
                                           ((r < n && fabs(cre) > pr.div_re) ? 2u : 0u), r, geo.base);
    const bool group_shift_ok = (flags & 1u) == 0u;
    const bool div_any = (flags & 2u) != 0u;
    double zn2 = 0.0;  // max_j |z_j + dN_j|^2, for the endgame's stopping test (every group that
    // may run an endgame step in this iteration: in the endgame, or accepting its point at s = 0;
    // the mixed form's FP32 launch parks its endgames instead)
    if (!MIXED && __any(active && (phase == PH_END || sc >= 0.0)))
      zn2 = group_max<N, double>(r < n ? cre * cre + cim * cim : 0.0, r, geo.base);
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
    bool fin = false, park = false;
    int fst = 0;
    if (MIXED && iters >= pr.max_iters / 8 && (phase == PH_TRACK || (RK && phase >= PH_RK1))) {
      park = true;  // an eighth of the iteration budget spent in FP32: FP64 takes over
      fst = kParked;
      ds = pr.ds0;
    } else if (iters >= pr.max_iters) {
      fin = true;
      fst = -7;
    } else {
      ++iters;
      ++c3;
      const double nrm = nN;
      // the mixed form cannot resolve pivots below FP32's precision, nor polish below its
      // tracking tolerance: such points are rejected, or the path fails and is re-tracked in FP64
      const double sing_ratio = use64 ? pr.sing_ratio : fmax(pr.sing_ratio, 1e-7);
      const double tol_polish = use64 ? pr.tol_polish : fmax(pr.tol_polish, pr.tol_track);
      const bool bad_lu = sing || !(ratio >= sing_ratio);
      const bool nonfin = !(nN <= INFINITY) || !(nE <= INFINITY);
      int act = ACT_NONE;
      if (MIXED && (bad_lu || nonfin) && phase != PH_TRACK && !(RK && phase >= PH_RK1)) {
        park = true;  // the accepted point itself: re-tracked in FP64 from there
        fst = kParked;
        ds = pr.ds0;
      } else if (bad_lu || nonfin) {  // a predicted, stage or corrected point: a rejected step
        if (phase == PH_TRACK || (RK && phase >= PH_RK1)) {
          act = ACT_REJECT;
        } else {
          fin = true;
          fst = bad_lu ? -1 : -4;
        }
      } else if (RK && phase >= PH_RK1 && nrm > pr.tol_predict) {
        act = ACT_REJECT;  // a stage point outside the corrector's trust region
      } else if (RK && phase >= PH_RK1) {
        // a Runge-Kutta stage point: its Euler direction is k_{j+1}, j = the stage (each lane
        // its own coordinate); the step h and its end are those of the prediction (ds and s_a
        // do not change during the stages)
        const int j = phase - PH_RK1 + 1;
        const double hstep = fmin(ds, -sa), st = (hstep == -sa) ? 0.0 : sa + hstep;
        if (geo.valid) {
          const Cx<double> za = sZa[r], ks = sKs[r];
          const double wgt = j < 3 ? 2.0 : 1.0;
          const Cx<double> kn = {fma(wgt, e.x, ks.x), fma(wgt, e.y, ks.y)};
          if (j < 3) {  // the next stage point: z_a + h/2 k2, then z_a + h k3
            const double a = j + 1 < 3 ? 0.5 * hstep : hstep;
            zo_r = fma(a, e.x, za.x);
            zo_i = fma(a, e.y, za.y);
            sKs[r] = kn;
          } else {  // the predicted point z_a + h/6 (k1 + 2 k2 + 2 k3 + k4)
            zo_r = fma(hstep / 6.0, kn.x, za.x);
            zo_i = fma(hstep / 6.0, kn.y, za.y);
          }
        }
        if (j < 3) {
          sc = j + 1 < 3 ? sa + 0.5 * hstep : st;
          ++phase;
        } else {
          sc = st;
          k = 0;
          phase = PH_TRACK;
        }
      } else if (phase == PH_POLISH) {
        zo_r = cre;
        zo_i = cim;
        ++k;
        ++c2;
        if (nrm <= tol_polish && pr.polish_only) {
          fin = true;  // polished: the mixed form's FP32 launch resumes it
          fst = 2;
        } else if (nrm <= tol_polish) {
          phase = PH_RESUME;
          k = 0;
        } else if (k >= pr.max_polish) {
          fin = true;
          fst = -5;
        }
      } else if (phase == PH_TRACK && k == 0 && nrm > pr.tol_predict) {
        act = ACT_REJECT;  // the predicted point lies outside the corrector's trust region
      } else if (phase == PH_RESUME || (phase == PH_TRACK && nrm <= pr.tol_track)) {
        if (phase == PH_TRACK) {
          ++c0;
          ++steps_here;
          if (k <= 1) ds = fmin(2.0 * ds, pr.ds_max);
          // the accepted point so far becomes the Hermite predictor's earlier point (each lane
          // moves its own coordinate)
          sZp[r] = sZa[r];
          sEp[r] = sEa[r];
          sp = sa;
          have_p = true;
        } else {
          have_p = false;  // a path's first accepted point in this call
        }
        sZa[r] = Cx<double>{zo_r, zo_i};
        sEa[r] = e;
        sa = sc;
        rej_run = 0;
        if (sa >= 0.0) {
          if (MIXED) {
            park = true;  // the endgame runs in the FP64 launch
            fst = kParkedEnd;
          } else {
            phase = PH_END;
            k = 0;
            act = ACT_END;
          }
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
          zo_r = cre;
          zo_i = cim;
          ++k;
          ++c2;
          nrm_prev = nrm;
          if (div_any && MIXED) {
            act = ACT_REJECT;  // a jump out of the region (FP32 noise can cause it): a shorter step
          } else if (div_any) {
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
        if (MIXED && (++rej_run >= kMixedFp64Rejects || ds < kMixedMinStep || ds < pr.ds_min)) {
          park = true;  // in FP64, from the last accepted point with a fresh step
          fst = kParked;
          ds = pr.ds0;
        } else if (ds < pr.ds_min) {
          fin = true;
          fst = -2;
          // the reported point is the last accepted one
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
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
        const double st = (hstep == -sa) ? 0.0 : sa + hstep;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        if (RK && pr.predictor == HOM_PREDICT_RK4) {
          // Runge-Kutta: first the stage point z_a + h/2 k1 at s_a + h/2 (k1 = the Euler
          // direction at the accepted point)
          if (geo.valid) {
            const Cx<double> za = sZa[r], ea = sEa[r];
            sKs[r] = ea;
            zo_r = fma(0.5 * hstep, ea.x, za.x);
            zo_i = fma(0.5 * hstep, ea.y, za.y);
          }
        } else if (geo.valid) {
          const Cx<double> za = sZa[r], ea = sEa[r];
          if (pr.predictor == HOM_PREDICT_HERMITE && have_p && hstep <= 4.0 * (sa - sp)) {
            // the cubic through (sp, z_p) and (sa, z_a) with slopes e_p, e_a (Sec. 2.3's
            // Hermite predictor from the Euler directions already computed), at st
            const Cx<double> zp = sZp[r], ep = sEp[r];
            const double d = sa - sp, t = (st - sp) / d, t2 = t * t, t3 = t2 * t;
            const double h00 = 2.0 * t3 - 3.0 * t2 + 1.0, h10 = (t3 - 2.0 * t2 + t) * d;
            const double h01 = -2.0 * t3 + 3.0 * t2, h11 = (t3 - t2) * d;
            zo_r = h00 * zp.x + h10 * ep.x + h01 * za.x + h11 * ea.x;
            zo_i = h00 * zp.y + h10 * ep.y + h01 * za.y + h11 * ea.y;
          } else {
            zo_r = fma(hstep, ea.x, za.x);
            zo_i = fma(hstep, ea.y, za.y);
          }
        }
        if (RK && pr.predictor == HOM_PREDICT_RK4) {
          sc = sa + 0.5 * hstep;
          phase = PH_RK1;
        } else {
          sc = st;
          phase = PH_TRACK;
        }
        k = 0;
      }
      if (act == ACT_END) {
        {
          const double zn = sqrt(zn2);
          zo_r = cre;
          zo_i = cim;
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
    if (geo.valid)  // read by the group's next evaluation (zero for the padding unknowns)
      sZc[r] = r < n ? Cx<double>{zo_r, zo_i} : Cx<double>{0.0, 0.0};
    if (park) {  // the last accepted point (in PH_RESUME the current point is that point)
      if (phase == PH_TRACK || (RK && phase >= PH_RK1)) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        if (geo.valid) {
          zo_r = sZa[r].x;
          zo_i = sZa[r].y;
        }
        sc = sa;
      }
      fin = true;
    }
    if (fin) {
      const int64_t p = path;
      if (r < n) {
        z[2 * (p * zstride + r)] = zo_r;
        z[2 * (p * zstride + r) + 1] = zo_i;
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
      if (MIXED && pr.plist && fst == kParked) {  // publish it to the concurrent FP64 launch
        __threadfence();                          // (after every lane's writes of its state)
        if (r == 0) {
          const unsigned long long idx = atomicAdd(&pr.pctr[0], 1ull);
          __hip_atomic_store(&pr.plist[idx], (long long)p, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      path = -1;
    }
  }
  if (MIXED && pr.plist) {  // this wave parks nothing more
    __threadfence();
    if ((threadIdx.x & 63) == 0) atomicAdd(&pr.pctr[2], 1ull);
  }
}

// Single system: all P paths, one global work queue.  At most 256 registers per lane, so two
// waves share each SIMD (the FP64 form at n = 10 needs slightly more without the bound).
template <int N, bool MIXED, bool GT, bool RK = true>
__global__ void __launch_bounds__(kTrackBlock) __attribute__((amdgpu_waves_per_eu(2)))
    k_track(SysDev sd, const double *__restrict__ c, int64_t P, double *__restrict__ z,
            double *__restrict__ s, double *__restrict__ ds_io, int32_t *__restrict__ status,
            int32_t *__restrict__ counters, TrackDev pr, unsigned long long *__restrict__ queue,
            size_t table_bytes, unsigned long long *__restrict__ units) {
  // The mixed form's last launch, after the side launch: with every parked path taken up there
  // (the counters are final: both earlier launches have completed), no path is left to claim.
  // Every thread reads the same values, so whole blocks return before any barrier.
  if (pr.drained_exit && pr.pctr[3] == pr.pctr[0]) return;
  extern __shared__ __align__(16) char smem[];
  __shared__ double kcoef[kCoefCount];
  stage_coefficients(kcoef);
  if constexpr (GT) __syncthreads();  // (staged tables end with a barrier of their own)
  const SysLds<N> S = stage_tables<N, GT>(smem, sd, c);
  if constexpr (MIXED && !GT) {  // the FP32 evaluation's own tables follow the FP64 ones
    const F32Tables<N> ft = stage_f32_tables<N>(smem + table_bytes, S);
    track_slots<N, MIXED, RK>(S, sd.n,
                          reinterpret_cast<Cx<double> *>(smem + table_bytes +
                                                         lds_f32_bytes<N>(sd.n, sd.mmax)),
                          0, P, sd.n, z, s, ds_io, status, counters, pr, queue, units, kcoef, &ft);
  } else {
    track_slots<N, MIXED, RK>(S, sd.n, reinterpret_cast<Cx<double> *>(smem + table_bytes), 0, P, sd.n,
                          z, s, ds_io, status, counters, pr, queue, units, kcoef);
  }
}

__global__ void k_zero_u64(unsigned long long *p) { *p = 0ull; }

template <int N>
static hipError_t track_n(const System &S, const void *cws, const double *c, int64_t P, double *z,
                          double *s, double *ds, int32_t *status, int32_t *counters,
                          const TrackDev &pr, bool mixed, unsigned long long *queue,
                          hipStream_t stream, int blocks_req, int64_t *waves_out) {
  const size_t tb = (S.lds_bytes + 15) & ~(size_t)15;
  const size_t f32 = (mixed && !S.global_tables) ? lds_f32_bytes<N>(S.n, S.mmax) : 0;
  const size_t lds = tb + f32 + track_state_bytes<N>();
  const bool rk = pr.predictor == HOM_PREDICT_RK4;  // (FP64 launches always carry it)
  auto kern = mixed ? (S.global_tables ? (rk ? k_track<N, true, true, true> : k_track<N, true, true, false>)
                                       : (rk ? k_track<N, true, false, true> : k_track<N, true, false, false>))
                    : (S.global_tables ? k_track<N, false, true> : k_track<N, false, false>);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kTrackBlock, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int64_t gpb = (kTrackBlock / 64) * Geo<N>::G;
  int64_t blocks = (int64_t)per_cu * num_cus();
  const int64_t need = (P + gpb - 1) / gpb;
  if (blocks_req > 0) blocks = blocks_req < blocks ? blocks_req : blocks;
  else if (blocks > need) blocks = need > 0 ? need : 1;
  if (waves_out) *waves_out = blocks * (kTrackBlock / 64);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, stream, queue);
  char label[64];
  // the plain FP64 form's launch is "fp64"; the mixed form's FP64 launches are named for their part
  const char *part = mixed ? "mixed"
                     : pr.helper ? "fp64-beside"
                     : pr.polish_only ? "fp64-polish"
                     : pr.drained_exit ? "fp64-left"
                     : pr.claim == 8 ? "fp64-endgame"
                     : pr.claim == (4 | 8) ? "fp64-finish"
                     : "fp64";
  snprintf(label, sizeof label, "k_track<%d,%s>", N, part);
  prof_begin(stream);
  unsigned long long *units = prof_units(stream);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kTrackBlock), lds, stream, S.dev(cws), c,
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

hipError_t launch_track(const System &S, const void *cws, const double *c, int64_t P, double *z,
                        double *s, double *ds, int32_t *status, int32_t *counters,
                        const TrackDev &pr, bool mixed, unsigned long long *queue,
                        hipStream_t stream, int blocks, int64_t *waves_out) {
  HOM_SWITCH_T(S.N, return track_n<NN>(S, cws, c, P, z, s, ds, status, counters, pr, mixed,
                                       queue, stream, blocks, waves_out))
}

__global__ void k_fill_i64(long long *p, long long v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_i64(long long *p, long long v, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + 255) / 256;
  const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
  hipLaunchKernelGGL(k_fill_i64, dim3(grid), dim3(256), 0, stream, p, v, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Batched form: many systems of uneven n and support sizes in one persistent launch.
// ------------------------------------------------------------------------------------------
constexpr size_t kBatchStateBytes = 28 * 1024;  // >= track_state_bytes<N>() for every N
static_assert(track_state_bytes<2>() <= kBatchStateBytes && track_state_bytes<3>() <= kBatchStateBytes &&
                  track_state_bytes<5>() <= kBatchStateBytes && track_state_bytes<7>() <= kBatchStateBytes,
              "batch LDS state budget");

// One work item: paths [p_begin, p_end) of system b, tracked by the block's lane groups sized
// for b.N.  The tables go to LDS when they fit the budget, else they are read where they are.
template <int N, bool MIXED>
__device__ __forceinline__ void batch_item(char *smem, const BatchSysDev &b,
                                           const double *__restrict__ T_all,
                                           const int32_t *__restrict__ ints_all,
                                           const double *__restrict__ c,
                                           const Cx<double> *__restrict__ Cg,
                                           const double *__restrict__ Cabs_g, int64_t p_begin,
                                           int64_t p_end, int zstride, double *z, double *s,
                                           double *ds, int32_t *status, int32_t *counters,
                                           const TrackDev &pr, unsigned long long *lq,
                                           unsigned long long *units, size_t table_budget,
                                           const double *kcoef) {
  const SysDev sd{b.n, b.mmax, b.M, T_all + b.T_off, ints_all + b.ints_off,
                  ints_all + b.ints_off + b.n};
  // block-uniform branch (one item per block); one inlined tracker per table location, so the
  // staged case reads its tables with LDS instructions
  Cx<double> *slots = reinterpret_cast<Cx<double> *>(smem + table_budget);
  if (b.lds_bytes > 0) {
    const SysLds<N> S = stage_tables<N, false>(smem, sd, c + 2 * b.c_off);
    track_slots<N, MIXED>(S, b.n, slots, p_begin, p_end, zstride, z, s, ds, status, counters, pr,
                          lq, units, kcoef);
  } else {
    const SysLds<N> S{sd.T, Cg + b.C_off, Cabs_g + b.C_off, sd.mk, b.n, b.mmax};
    track_slots<N, MIXED>(S, b.n, slots, p_begin, p_end, zstride, z, s, ds, status, counters, pr,
                          lq, units, kcoef);
  }
}

template <bool MIXED>
__global__ void __launch_bounds__(kTrackBlock) __attribute__((amdgpu_waves_per_eu(2)))
    k_track_batch(const BatchSysDev *__restrict__ sys, int num_sys,
                  const double *__restrict__ T_all, const int32_t *__restrict__ ints_all,
                  const double *__restrict__ c, const Cx<double> *__restrict__ Cg,
                  const double *__restrict__ Cabs_g, const int64_t *__restrict__ sys_off,
                  const int64_t *__restrict__ item_off, int tile, int zstride,
                  double *__restrict__ z, double *__restrict__ s, double *__restrict__ ds,
                  int32_t *__restrict__ status, int32_t *__restrict__ counters, TrackDev pr,
                  unsigned long long *__restrict__ gqueue, size_t table_budget,
                  unsigned long long *__restrict__ units) {
  extern __shared__ __align__(16) char smem[];
  __shared__ unsigned long long lq;
  __shared__ long long sh_item;
  __shared__ double kcoef[kCoefCount];
  stage_coefficients(kcoef);  // visible after the item loop's first barrier
  const int64_t n_items = item_off[num_sys];
  for (;;) {
    __syncthreads();  // the previous item is finished by every wave before LDS is reused
    if (threadIdx.x == 0) {
      sh_item = (long long)atomicAdd(gqueue, 1ull);
      lq = 0ull;
    }
    __syncthreads();
    const int64_t item = sh_item;
    if (item >= n_items) break;
    int lo = 0, hi = num_sys - 1;  // last system whose first item is <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (item_off[mid] <= item) lo = mid;
      else hi = mid - 1;
    }
    const BatchSysDev b = sys[lo];
    const int64_t first = item - item_off[lo];
#define HOM_BATCH_CASE(NN)                                                                      \
  case NN: {                                                                                  \
    const int64_t chunk = (int64_t)tile * (kTrackBlock / 64) * Geo<NN>::G;                     \
    const int64_t pb = sys_off[lo] + first * chunk;                                           \
    const int64_t pe = pb + chunk < sys_off[lo + 1] ? pb + chunk : sys_off[lo + 1];           \
    batch_item<NN, MIXED>(smem, b, T_all, ints_all, c, Cg, Cabs_g, pb, pe, zstride, z, s, ds,  \
                          status, counters, pr, &lq, units, table_budget, kcoef);              \
    break;                                                                                    \
  }
    switch (b.N) {
      HOM_BATCH_CASE(2)
      HOM_BATCH_CASE(3)
      HOM_BATCH_CASE(4)
      HOM_BATCH_CASE(5)
      HOM_BATCH_CASE(6)
      HOM_BATCH_CASE(7)
      HOM_BATCH_CASE(8)
      HOM_BATCH_CASE(10)
      HOM_BATCH_CASE(12)
      HOM_BATCH_CASE(16)
      HOM_BATCH_CASE(20)
      HOM_BATCH_CASE(24)
      HOM_BATCH_CASE(32)
      default:
        break;
    }
#undef HOM_BATCH_CASE
  }
}

// Per call: table-order coefficients and |c| of every system (used by systems read from global
// memory), and each system's first path (sys_idx is non-decreasing).
__global__ void k_batch_prep(const BatchSysDev *__restrict__ sys, int num_sys,
                             const int32_t *__restrict__ ints_all, const double *__restrict__ c,
                             const int32_t *__restrict__ sys_idx, int64_t P,
                             Cx<double> *__restrict__ Cg, double *__restrict__ Cabs_g,
                             int64_t *__restrict__ sys_off) {
  const int sidx = blockIdx.x;
  if (sidx < num_sys) {
    const BatchSysDev b = sys[sidx];
    const int32_t *mk = ints_all + b.ints_off, *off = mk + b.n;
    for (int idx = threadIdx.x; idx < b.mmax * b.n; idx += blockDim.x) {
      const int i = idx / b.n, r = idx - (idx / b.n) * b.n;
      Cx<double> v = {0.0, 0.0};
      if (i < mk[r]) {
        const int64_t q = b.c_off + off[r] + i;
        v.x = c[2 * q];
        v.y = c[2 * q + 1];
      }
      Cg[b.C_off + idx] = v;
      Cabs_g[b.C_off + idx] = sqrt(v.x * v.x + v.y * v.y);
    }
  }
  if (threadIdx.x == 0 && sidx <= num_sys) {  // lower_bound(sys_idx, sidx)
    int64_t lo = 0, hi = P;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (sys_idx[mid] < sidx) lo = mid + 1;
      else hi = mid;
    }
    sys_off[sidx] = lo;
  }
}

// item_off[s] = number of work items before system s (one thread; num_sys is small).
__global__ void k_batch_items(const BatchSysDev *__restrict__ sys, int num_sys, int tile,
                              const int64_t *__restrict__ sys_off, int64_t *__restrict__ item_off) {
  int64_t acc = 0;
  for (int s = 0; s < num_sys; ++s) {
    item_off[s] = acc;
    const int N = sys[s].N;
    const int64_t chunk = (int64_t)tile * (kTrackBlock / 64) * (64 / N);
    const int64_t np = sys_off[s + 1] - sys_off[s];
    acc += (np + chunk - 1) / chunk;
  }
  item_off[num_sys] = acc;
}

size_t track_batch_ws_bytes(const System &S) {
  return 256 + (size_t)(S.num_sys + 1) * 16 + (size_t)S.C_total * 24 + 256;
}

hipError_t launch_track_batch(const System &S, const double *c, int64_t P, double *z, double *s,
                              double *ds, const int32_t *sys_idx, int32_t *status,
                              int32_t *counters, const TrackDev &pr, bool mixed, void *ws,
                              hipStream_t stream) {
  char *w = static_cast<char *>(ws);
  unsigned long long *queue = reinterpret_cast<unsigned long long *>(w);
  int64_t *sys_off = reinterpret_cast<int64_t *>(w + 256);
  int64_t *item_off = sys_off + (S.num_sys + 1);
  Cx<double> *Cg = reinterpret_cast<Cx<double> *>(item_off + (S.num_sys + 1));
  double *Cabs_g = reinterpret_cast<double *>(Cg + S.C_total);
  const int tile = pr.tile > 0 ? pr.tile : 4;
  hipLaunchKernelGGL(k_batch_prep, dim3((unsigned)(S.num_sys + 1)), dim3(256), 0, stream, S.dBatch,
                     S.num_sys, S.dInts_all, c, sys_idx, P, Cg, Cabs_g, sys_off);
  hipLaunchKernelGGL(k_batch_items, dim3(1), dim3(1), 0, stream, S.dBatch, S.num_sys, tile,
                     sys_off, item_off);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, stream, queue);
  const size_t budget = (S.batch_lds + 15) & ~(size_t)15;
  const size_t lds = budget + kBatchStateBytes;
  auto kern = mixed ? k_track_batch<true> : k_track_batch<false>;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kTrackBlock, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const unsigned blocks = (unsigned)(per_cu * num_cus());
  prof_begin(stream);
  unsigned long long *units = prof_units(stream);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(kTrackBlock), lds, stream, S.dBatch, S.num_sys,
                     S.dT_all, S.dInts_all, c, Cg, Cabs_g, sys_off, item_off, tile, S.n, z, s, ds,
                     status, counters, pr, queue, budget, units);
  prof_end(stream, mixed ? "k_track_batch<mixed>" : "k_track_batch<fp64>");
  return hipGetLastError();
}

}  // namespace hom
