/*
 * hom.h - C ABI of the MI355X polyhedral-homotopy hot path (arXiv 2111.14317).
 *
 * The library evaluates a lifted Laurent system together with all its partial derivatives and
 * solves the Euler and Newton directions in one consolidated solve, at many points or paths at
 * once, on one AMD Instinct MI355X (gfx950).
 *
 * Notation (Sec. 2, eq. (1) and (2); Sec. 5.1):
 *   h_k(x, t) = sum_{a in S_k} c_{k,a} x^a t^{w_k(a)},  k = 0..n-1, with x = e^z (any branch of
 *   log) and t = e^s.  Equation k has m_k monomials; M = sum_k m_k.
 *   A   : int8 [M][n] row-major exponent vectors, equation-major (equation 0's rows first),
 *         |a| <= 127.
 *   w   : double [M] liftings (non-negative; rational values allowed).
 *   c   : complex128 [M] coefficients (interleaved re, im), passed per call.
 *   z   : complex128 [P][n] points in log coordinates; s : double [P] (s <= 0, t = 1 <=> s = 0).
 *
 * Ownership and memory: every array argument of the compute calls (eval, step, track,
 * endpoint_grad) is a caller-owned DEVICE buffer, contiguous, in the layout stated.  hom_create
 * takes HOST arrays and copies them.  The library owns only its handle tables and workspaces.
 *
 * Errors: every call returns HOM_OK (0) or a negative code; hom_last_error() gives a
 * thread-local message.  Per-point or per-path numerical outcomes go to status arrays and never
 * fail a call.  Compute calls are asynchronous on `stream`; device faults surface at the next
 * synchronisation.  A handle is immutable after creation, so one handle may be used from
 * several streams at once.
 */
#ifndef HOM_H
#define HOM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hom_system_s *hom_system_t;
typedef void *hom_stream_t; /* a hipStream_t; NULL is the null stream */

/* return codes */
#define HOM_OK 0
#define HOM_EINVAL (-1)       /* invalid argument (null pointer, n out of range, ...) */
#define HOM_ENOMEM (-2)       /* device allocation failed */
#define HOM_EDEVICE (-3)      /* a HIP call failed */
#define HOM_EUNSUPPORTED (-4) /* valid but not supported (e.g. tables too large) */

/* precision of the compute calls */
#define HOM_FP64 0  /* everything in FP64 */
#define HOM_MIXED 1 /* FP32 exponentials, contraction and LU; FP64 exponent sums, state and
                       decisions; FP64 endgame (see hom_track) */

/* hom_eval flags */
#define HOM_UNSCALED 1 /* multiply row k back by e^{logscale_k} (may overflow) */
#define HOM_AFFINE 2   /* return J_x = J_z diag(e^{-z}) and H_t = e^{-s} H_s instead */
#define HOM_EVAL_FP32 4 /* the mixed form's evaluation: FP32 exponentials and contraction
                           (exponent sums still FP64), results widened to FP64; on a handle
                           with matrix-core tables: the BF16x3 engine (below) */
#define HOM_EVAL_VALU 8 /* on a handle with matrix-core tables, use the vector-unit kernels
                           (one lane per equation) instead */

/* hom_create flags */
#define HOM_CREATE_VALU 1 /* build no matrix-core tables (see hom_create) */
#define HOM_CREATE_PROJECTIVE 2 /* the homogenised system in n + 1 unknowns (hom_step_proj only) */
#define HOM_CREATE_PER_EQUATION 4 /* no common-support engine even when the supports coincide */

/* per-path status (hom_step: OK or SINGULAR; hom_track: all) */
#define HOM_PATH_OK 0            /* reached s = 0, endgame converged, residual <= res_tol */
#define HOM_PATH_START 1         /* input: a fresh start point (polish at s, then track) */
#define HOM_PATH_RUNNING 2       /* in/out: stopped at an accepted point; call again to resume */
#define HOM_PATH_SINGULAR (-1)   /* pivot ratio below sing_ratio off the tracking phase */
#define HOM_PATH_STEP_MIN (-2)   /* step size fell below ds_min */
#define HOM_PATH_DIVERGED (-3)   /* |Re z_j| > div_re */
#define HOM_PATH_NONFINITE (-4)  /* NaN or Inf off the tracking phase */
#define HOM_PATH_POLISH_FAIL (-5) /* start point did not converge at s0 */
#define HOM_PATH_ENDGAME_FAIL (-6) /* residual at s = 0 above res_tol */
#define HOM_PATH_MAX_ITERS (-7)  /* iteration cap reached */

/*
 * Create a system handle (the initialisation step of Sec. 7, Alg. 1): validates the input,
 * copies A and w to the device and builds the per-equation tables the kernels stage into LDS
 * (tables beyond the 48 KB LDS budget are read from global memory instead, and each compute call
 * then builds its coefficient table in a stream-ordered workspace).
 * When the largest m_k is at least 32 (a dense support) it also builds the matrix-core tables:
 * hom_eval and hom_step then run the two contractions of Sec. 5.1 on MFMA, per equation and per
 * tile of 16 points (FP64: 16x16x4 f64 MFMA; HOM_EVAL_FP32 / HOM_MIXED: BF16x3, i.e. z and the
 * exponentials split into three bf16 parts with FP32 accumulation, the phase formed exactly
 * from integer digit sums); hom_step keeps the LU on the vector units.  flags: 0 or
 * HOM_CREATE_VALU (no matrix-core tables), HOM_CREATE_PROJECTIVE (a handle for hom_step_proj),
 * HOM_CREATE_PER_EQUATION (see below).
 * Common support (the unmixed case of Sec. 5.1): when every equation lists the same monomials in
 * the same order with the same liftings (n > 1, at most 256 monomials, at least 32), the FP64
 * matrix-core evaluation forms each point's exponentials e^{<a, z> + w s} once, shared by all
 * equations, and contracts them with every equation's coefficients and the common exponent
 * columns (Sec. 5.1: one exponential row e^{Z A} for all of [B_1 ... B_n]); the row shift
 * logscale is then one value per point, the row maximum over the common support to within about
 * 0.1.  HOM_CREATE_PER_EQUATION keeps the per-equation engines instead.
 * n in [1, 32]; m[k] >= 1; M <= 65536.  Synchronous.
 * Errors: HOM_EINVAL (bad argument), HOM_ENOMEM, HOM_EDEVICE.
 */
int hom_create(int n, const int32_t *m, const int8_t *A, const double *w, int flags,
               hom_system_t *out);

/* One system of a batch: n unknowns, m [n], A [M][n] int8 (equation-major), w [M] (host). */
typedef struct {
    int32_t n;
    const int32_t *m;
    const int8_t *A;
    const double *w;
} hom_sys_desc;

/*
 * Create a handle over several systems of uneven n and support sizes (the batched form), tracked
 * together by one persistent launch of hom_track.  Each system is validated as in hom_create;
 * num_sys in [1, 65536].  Systems whose tables do not fit the LDS budget are read from global
 * memory.  Only hom_track accepts batch handles (the other compute calls return
 * HOM_EUNSUPPORTED).  Synchronous.  flags must be 0.
 */
int hom_create_batch(int num_sys, const hom_sys_desc *descs, int flags, hom_system_t *out);

/* Release a handle (waits for the device).  NULL is accepted. */
int hom_destroy(hom_system_t sys);

/* n (the largest n of a batch), M (total over a batch), the largest m_k and the number of
 * systems of a handle (any pointer may be NULL). */
int hom_system_info(hom_system_t sys, int *n, int64_t *M, int *m_max, int *num_sys);

/*
 * Evaluate the extended Jacobian [J_z | H_s | H] at P points (Sec. 5.1 and 5.2; Sec. 7, Alg. 2):
 *   G[p][k][j] = dh_k/dz_j (j < n),  G[p][k][n] = dh_k/ds,  G[p][k][n+1] = h_k,
 * each row k multiplied by e^{-logscale[p][k]}, where logscale[p][k] is the largest
 * <a, Re z_p> + w(a) s_p over the monomials of equation k (so no term over- or underflows).
 * c: complex128 [M]; z: complex128 [P][n]; s: double [P]; G: complex128 [P][n][n+2];
 * logscale: double [P][n] or NULL (zeros with HOM_UNSCALED).  flags: any of HOM_UNSCALED,
 * HOM_AFFINE, HOM_EVAL_FP32, HOM_EVAL_VALU.  On the matrix-core engines the shift logscale is
 * the row maximum to within about 0.1 (any shift gives the same directions).  P = 0 is a no-op.
 */
int hom_eval(hom_system_t sys, const double *c, int64_t P, const double *z, const double *s,
             double *G, double *logscale, int flags, hom_stream_t stream);

/*
 * One evaluation plus the consolidated Euler/Newton solve at P points (Sec. 6 in its affine
 * form; Sec. 7, Alg. 2 followed by Alg. 3): one LU with partial pivoting of J_z applied to
 * both right-hand sides gives
 *   dz_euler  = -J_z^{-1} H_s   (= dz/ds along the path through (z, s); Davidenko, Sec. 2.3)
 *   dz_newton = -J_z^{-1} H     (the Newton step in z; Sec. 2.3).
 * dz_euler, dz_newton: complex128 [P][n]; status: int32 [P] (HOM_PATH_OK, or
 * HOM_PATH_SINGULAR when a pivot is zero or min|pivot|/max|pivot| < 1e-14).
 * precision: HOM_FP64 or HOM_MIXED (FP32 exponentials, contraction and LU; the LU is redone in
 * FP64 when its FP32 pivot ratio is below 1e-4).
 */
int hom_step(hom_system_t sys, const double *c, int64_t P, const double *z, const double *s,
             double *dz_euler, double *dz_newton, int32_t *status, int precision,
             hom_stream_t stream);

/*
 * The Euler and Newton directions in homogeneous coordinates (Sec. 2.2, eq. (3)-(5)), computed as
 * in Sec. 6 and Alg. 2-3: from the null space of the unified system
 *   J = [ dH~/dy  dH~/ds  H~ ; y^*  0  0 ]      ((n+1) x (n+3))
 * by Householder reflections (the QR decomposition of J^T), then the row reduction that makes the
 * two null vectors' last two entries the identity: (dy_euler, 1, 0) and (dy_newton, 0, 1).  So
 *   dH~/dy dy_euler + dH~/ds = 0,  y^* dy_euler = 0;   dH~/dy dy_newton + H~ = 0,  y^* dy_newton = 0.
 * The handle must come from hom_create with HOM_CREATE_PROJECTIVE: its equation k is homogenised
 * as h~_k(y, s) = sum_a c_a y^(a, d_k - |a|) e^{s w(a)} with d_k the largest total degree |a| of
 * the equation's monomials (the homogenising exponents must not exceed 127; n <= 29).  y_j pairs
 * with x_j for j < n and y_n is the homogenising coordinate, so an affine point x is y = (x, 1).
 * The evaluation runs in log coordinates z = log y (A1-A3) followed by the y-coordinate epilogue
 * of Alg. 2 (column j times 1 / y_j); every y_j must be nonzero.
 * c: complex128 [M]; y: complex128 [P][n+1]; s: double [P]; dy_euler, dy_newton: complex128
 * [P][n+1]; status: int32 [P] (HOM_PATH_OK, or HOM_PATH_SINGULAR when min|L_jj| / max|L_jj| of
 * the triangular factor is below 1e-14, the 2 x 2 block is singular or a result is not finite).
 * FP64.  P = 0 is a no-op.
 */
int hom_step_proj(hom_system_t sys, const double *c, int64_t P, const double *y, const double *s,
                  double *dy_euler, double *dy_newton, int32_t *status, hom_stream_t stream);

/* Tracker constants.  The paper fixes no step control; these are this library's rules. */
typedef struct {
    double ds0;        /* initial step in s for fresh paths */
    double ds_max;     /* largest step */
    double ds_min;     /* step below which a path fails (HOM_PATH_STEP_MIN) */
    double tol_polish; /* start point accepted when ||dz_newton||_inf <= tol_polish */
    double tol_track;  /* corrector converged when ||dz_newton||_inf <= tol_track */
    double tol_end;    /* endgame stops when ||dz_newton||_inf <= tol_end (1 + ||z||_inf) */
    double res_tol;    /* endpoint OK when max_k |h_k| / sum_a |c_a x^a| <= res_tol */
    double div_re;     /* |Re z_j| > div_re => HOM_PATH_DIVERGED */
    double sing_ratio; /* min|pivot| / max|pivot| below this => singular */
    double tol_predict; /* a predicted point whose first ||dz_newton||_inf exceeds this is
                           rejected before any correction (the predictor left the corrector's
                           trust region, where the Newton iteration may converge to another
                           path); the step is halved */
    int32_t max_polish; /* Newton iterations allowed at the start point */
    int32_t max_newton; /* corrector iterations per step before the step is rejected */
    int32_t max_end;    /* endgame Newton iterations */
    int32_t max_steps;  /* accepted steps per call; then HOM_PATH_RUNNING */
    int32_t max_iters;  /* eval+solve cap per path per call; then HOM_PATH_MAX_ITERS */
    int32_t precision;  /* HOM_FP64 or HOM_MIXED */
    int32_t flags;      /* 0 or any of HOM_TRACK_EXACT_SHIFT, HOM_TRACK_SERIAL,
                           HOM_TRACK_SIDE_NOWAIT */
    int32_t tile;       /* batched form: paths per work item = tile x lane groups per block
                           (0: the default, 4) */
    int32_t predictor;  /* HOM_PREDICT_EULER (default), HOM_PREDICT_HERMITE or HOM_PREDICT_RK4 */
} hom_track_params;

/* hom_track_params.predictor.  Euler: z = z_a + h dz_euler(z_a) (Sec. 2.3).  Hermite: the cubic
 * through the last two accepted points (s_p, z_p), (s_a, z_a) with slopes dz_euler there (the
 * Euler directions the consolidated solve already returned at those points; Sec. 2.3 lists the
 * cubic Hermite method among the predictors built on them), used when the step h <= 4 (s_a - s_p);
 * the first step after a path's start or resume is an Euler step (so a resumed run is not
 * bitwise the uninterrupted one with this predictor, though it reaches the same endpoints). */
#define HOM_PREDICT_EULER 0
#define HOM_PREDICT_HERMITE 1
/* Runge-Kutta (Sec. 2.3 names Runge-Kutta predictors built on the Euler direction): the
 * classical fourth-order scheme on dz/ds = dE(z, s) from the accepted point,
 *   k2 = dE(z_a + h/2 k1, s_a + h/2), k3 = dE(z_a + h/2 k2, s_a + h/2), k4 = dE(z_a + h k3, s_a + h),
 *   z = z_a + h/6 (k1 + 2 k2 + 2 k3 + k4);
 * three more eval+solves per step (counted like the others); a stage point whose evaluation
 * fails, or whose Newton step exceeds tol_predict (outside the corrector's trust region, as for
 * the predicted point), rejects the step. */
#define HOM_PREDICT_RK4 2

/* hom_track_params.flags: recompute every row's maximum (the e^{-M_k} row shift) at every
 * evaluation instead of reusing the previous evaluation's maximum.  Slower (one more pass over
 * the monomials); makes a resumed run bitwise equal to an uninterrupted one. */
#define HOM_TRACK_EXACT_SHIFT 1
/* hom_track_params.flags, mixed form of a single-system handle: run the FP64 re-tracks of parked
 * paths after the FP32 launch instead of beside it.  By default a small FP64 launch on a
 * library-owned second stream takes each parked path from a device list as soon as the FP32
 * launch parks it; the call's stream waits for that stream before the call's last launch, so the
 * call stays ordered on its stream.  Under stream capture the serial order is always used.  The
 * results are the same either way (the same FP64 kernel re-tracks every parked path). */
#define HOM_TRACK_SERIAL 2
/* hom_track_params.flags, mixed form with the FP64 re-tracks beside the FP32 launch: the side
 * launch stops claiming as soon as it finds no parked path waiting (instead of waiting up to
 * 0.2 s for the FP32 launch to park more); the call's last launch re-tracks whatever it left.
 * The results are the same; this exercises that hand-over (tests) and is otherwise slower. */
#define HOM_TRACK_SIDE_NOWAIT 4

/* Fill `p` with this library's defaults for `precision`. */
int hom_track_params_default(hom_track_params *p, int precision);

/*
 * Track P paths of the homotopy to t = 1 (s = 0) with the consolidated Euler/Newton step as
 * predictor/corrector (Sec. 2.3 and Sec. 6), all paths in one persistent launch: lane groups
 * claim paths from a device queue and refill as paths finish.
 * z: complex128 [P][n], in: start points, out: endpoints (or the point reached).
 * s: double [P] in/out; ds: double [P] in/out (read for RUNNING paths).
 * status: int32 [P] in/out: HOM_PATH_START (fresh) or HOM_PATH_RUNNING (resume); other values
 * are left untouched and the path is skipped.
 * counters: int32 [P][4] accumulated: accepted steps, rejected steps, corrector iterations,
 * eval+solves.  sys_idx must be NULL for a single-system handle.
 * Batch handle (hom_create_batch): c is the concatenation of the systems' coefficient arrays
 * (complex128 [sum of M]); z is complex128 [P][n_max] (path p uses its first n of its system);
 * sys_idx int32 [P] gives each path's system, non-decreasing (each system's paths contiguous),
 * values in [0, num_sys).  Work items are (system, run of consecutive paths); a block stages the
 * system's tables and its lane groups (sized for that system's n) claim the item's paths.
 * With precision HOM_MIXED the call makes three launches: FP64 polish of the fresh start
 * points; FP32 tracking (evaluations and solves; exponent sums, state and decisions in FP64),
 * which parks every path that reaches s = 0, and at its last accepted point every path whose
 * FP32 evaluation fails at that point, whose step falls below 1e-6 (or ds_min), that has 10
 * consecutive rejected steps or that has spent max_iters / 8 iterations (statuses 3 and 4,
 * internal; an FP32 failure or a jump out of |Re z| <= div_re at a predicted or corrected point
 * is a rejected step); FP64 for the parked paths, first the rest of those tracks, then the
 * endgames (single-system handles: the re-tracks run on the library's second stream while the
 * FP32 launch runs and the endgames follow it, unless HOM_TRACK_SERIAL is set).
 * Resume: calling with max_steps = k until no path is RUNNING gives the same endpoints as one
 * call; bitwise the same z and s with HOM_TRACK_EXACT_SHIFT (the counters then include one extra
 * eval+solve per resume), equal to rounding otherwise (the row shifts differ after a resume).
 */
int hom_track(hom_system_t sys, const double *c, int64_t P, double *z, double *s, double *ds,
              const int32_t *sys_idx, const hom_track_params *params, int32_t *status,
              int32_t *counters, hom_stream_t stream);

/*
 * hom_track without any device allocation, for callers that cannot allocate: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments, rules
 * and results as hom_track on a single-system handle (the mixed form's three launches run in
 * their serial order, as with HOM_TRACK_SERIAL, so the results equal hom_track's bit for bit).
 * Its work-queue counters and, for a system whose tables stay in global memory, this call's
 * coefficient table live in one static device array of HOM_NOALLOC_SCRATCH_BYTES per GPU, held
 * until the process ends; the kernels clear what must start at zero.  All calls on one GPU
 * share that array: calls that overlap in time on one GPU (other streams, other threads) race
 * and must not be made.  No profiling records are made for it.
 * Errors: as hom_track; HOM_EUNSUPPORTED for batch handles and for systems whose coefficient
 * table (24 bytes per entry of the largest m_k x n table) exceeds the scratch.
 */
#define HOM_NOALLOC_SCRATCH_BYTES (4u << 20) /* 4 MiB per GPU */
int hom_track_noalloc(hom_system_t sys, const double *c, int64_t P, double *z, double *s,
                      double *ds, const hom_track_params *params, int32_t *status,
                      int32_t *counters, hom_stream_t stream);

/*
 * Gradient of a real loss L(x*) on endpoints x* = e^{z_end} (t = 1) with respect to the
 * coefficients, by the implicit function theorem (the argument behind the Davidenko equation,
 * Sec. 2.3).  Per path: J_x^H nu = -g, computed as J_z^H nu = -conj(x*) .* g; then
 *   grad_c[k,a] = sum_p nu_{p,k} conj(x_p*^a),
 * summed over paths in a fixed order (bitwise reproducible).
 * grad_x: complex128 [P][n], g = dL/dRe x + i dL/dIm x (PyTorch's convention); grad_c:
 * complex128 [M], overwritten, same convention.  Paths whose Jacobian is singular contribute 0.
 * precision: HOM_FP64 or HOM_MIXED (FP32 evaluation and solve).
 */
int hom_endpoint_grad(hom_system_t sys, const double *c, int64_t P, const double *z_end,
                      const double *grad_x, double *grad_c, int precision, hom_stream_t stream);

/*
 * Start points (Sec. 2): the paths of polyhedral homotopy start at the roots of each mixed cell's
 * binomial system x^{d_k} = beta_k, k = 0..n-1 (d_k = the difference of the cell's two exponent
 * vectors in equation k, beta_k = -c_{k,j0} / c_{k,j1}); the paper takes them as given.  This
 * writes them, for any number of cells of one size n, in log coordinates z = log x.
 *   D      host int32 [num_cells][n][n], row k of cell c = d_k (nonsingular).
 *   beta   host complex [num_cells][n] (interleaved re, im), finite and nonzero.
 *   first, count   host int64 [num_cells] or both NULL: cell c's roots with index q in
 *          [first[c], first[c] + count[c]) (NULL: all of them, 0 .. |det D_c| - 1).  Root q of a
 *          cell is the one whose mixed-radix digits over the Smith invariant factors of D that
 *          exceed one (the first factor's digit varying fastest) are j: z = z_base + 2 pi i
 *          V S^{-1} j with z_base = D^{-1} log(beta) (principal logarithm), U D V = S.
 *   num_roots  host int64 [num_cells], out: |det D_c|, the number of roots of cell c.
 *   z      device complex [z_rows][n] or NULL: the roots, cell after cell; Im z in [-pi, pi).
 *          NULL: only num_roots is computed.
 * The cells are planned on the GPU, one wavefront per cell (the Smith form on int64 with overflow
 * checks, twice; z_base by an FP64 LU solve), then one launch writes the roots.  n in [1, 32];
 * the Smith form's entries within int64, |det D_c| < 2^62 and its largest invariant factor
 * < 2^31 (HOM_EUNSUPPORTED otherwise).  Blocks until the plans are read back (each cell's status
 * and root count); the roots are written asynchronously on `stream`.
 * Errors: HOM_EINVAL (bad argument, singular D, zero or non-finite beta, a range outside
 * [0, |det D_c|], more rows than z_rows), HOM_EUNSUPPORTED, HOM_ENOMEM, HOM_EDEVICE.
 */
int hom_binomial_starts(int n, int num_cells, const int32_t *D, const double *beta,
                        const int64_t *first, const int64_t *count, int64_t *num_roots, double *z,
                        int64_t z_rows, hom_stream_t stream);

/*
 * Peak probes: the rate of one unit of the device the calling thread has current, measured by a
 * bounded kernel (the denominators the kernels' rooflines can be set against, beside the
 * published peaks).  kind and the unit of *rate:
 *   HOM_PEAK_HBM_READ, HOM_PEAK_HBM_WRITE   GB/s  (a 4 GiB buffer read / written once per launch)
 *   HOM_PEAK_FP64_FMA, HOM_PEAK_FP32_FMA    TFLOP/s (vector FMA, 2 flops each)
 *   HOM_PEAK_FP32_EXP2                      G evaluations/s of the hardware exp2
 *   HOM_PEAK_MFMA_F64, HOM_PEAK_MFMA_BF16   TFLOP/s (16x16x4 f64, 16x16x32 bf16 with FP32 sums)
 *   HOM_PEAK_EXP_F64, HOM_PEAK_SINCOS_F64   G evaluations/s of this library's FP64 exponential
 *                                           and sine/cosine pair of the evaluation's terms
 * Allocates its own buffers (4 GiB for the HBM probes) and blocks until done; not for use under
 * stream capture.  Errors: HOM_EINVAL (unknown kind, NULL rate), HOM_ENOMEM, HOM_EDEVICE.
 */
#define HOM_PEAK_HBM_READ 0
#define HOM_PEAK_HBM_WRITE 1
#define HOM_PEAK_FP64_FMA 2
#define HOM_PEAK_FP32_FMA 3
#define HOM_PEAK_FP32_EXP2 4
#define HOM_PEAK_MFMA_F64 5
#define HOM_PEAK_MFMA_BF16 6
#define HOM_PEAK_EXP_F64 7
#define HOM_PEAK_SINCOS_F64 8
int hom_peak_probe(int kind, double *rate, hom_stream_t stream);

/*
 * Kernel timing (tracing).  While profiling is on for the calling thread, every kernel the
 * compute calls launch is bracketed by two hipEvents recorded on the launch stream, and the
 * tracker kernels also count the eval+solves they perform.  hom_profile_read waits for those
 * events and writes up to `cap` records in launch order: the kernel label as a NUL-terminated
 * string of at most 63 characters at names[64*i], the duration in milliseconds in ms[i], and
 * the number of eval+solves done by that launch in units[i] (-1 where not counted).  It clears
 * the list and returns the number of records written (records beyond `cap` are dropped), or a
 * negative error code.  At most 4096 records are kept.  Switching profiling on the first time
 * on a thread allocates its eval+solve counters (32 KiB) on the current device; the compute
 * calls themselves allocate nothing for it.
 */
int hom_set_profiling(int on);
int hom_profile_read(char *names, double *ms, int64_t *units, int cap);

/* Message for the last error on this thread ("" if none). */
const char *hom_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HOM_H */
