/*
 * Plain FP64 CPU oracle for the polyhedral-homotopy hot path (arXiv 2111.14317).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is checked against.  It
 * is used by the test suite, by the smoke check and by the benchmark's CPU-baseline leg, and by
 * nothing else; it shares no code with the GPU path.
 *
 * It follows the definitions directly, with no blocking or reordering:
 *   - eval : h_k(x,t) = sum_a c_{k,a} x^a t^{w_k(a)} (Sec. 2, eq. (1)) with x = e^z, t = e^s
 *            (eq. (2)).  Monomials x^a are built by repeated multiplication (x_j^{-1} for
 *            negative exponents).  The partials in log coordinates are
 *              dh_k/dz_j = sum_a a_j c_{k,a} x^a t^{w(a)}   and   dh_k/ds = sum_a w(a) c_{k,a} x^a t^{w(a)}
 *            (Sec. 5.1, the Hadamard-product form of the derivative and the extended row
 *            [D_z h_k, D_tau h_k, h_k]).  Output row k is [J_z | H_s | H] in that column order.
 *   - solve: the Euler direction dE solves J_z dE = -H_s (Davidenko equation, Sec. 2.3) and the
 *            Newton direction dN solves J_z dN = -H (Sec. 2.3).  Both come from one LU with partial
 *            pivoting of the augmented matrix [J_z | H_s | H] (the unified system of Sec. 6, in
 *            its affine form).
 *   - track: a predictor-corrector loop over s in [s0, 0] that uses dE as Euler predictor (or,
 *            optionally, the cubic Hermite predictor through the last two accepted points and
 *            their Euler directions, Sec. 2.3) and dN as Newton corrector (Sec. 2.3); the paper
 *            gives no step control, so the constants and rules come from the parameter struct.
 *   - proj : the Euler and Newton directions in homogeneous coordinates (Sec. 2.2, eq. (3)-(5)):
 *            the homogenised system's Jacobian with the row y^*, one (n+1) x (n+1) solve for
 *            both (the unified system of Sec. 6, solved plainly instead of by QR).
 *   - grad : gradient of a real loss on the endpoints with respect to the coefficients, through
 *            the implicit function theorem (the same argument as the Davidenko equation,
 *            Sec. 2.3): J_x^H nu = -g, grad c_{k,a} = sum_paths nu_k conj(x^a).
 *
 * Row scaling.  With `scaled` set, every row k is multiplied by e^{-M_k}, where M_k is the
 * largest log-magnitude max_a (<a, Re z> + w(a) s) of a monomial of equation k (without c), so
 * that t^w factors far below the FP64 range do not vanish and x^a far above it does not
 * overflow.  The term is then formed in polar form, c * (x/|x|)^a * exp(<a, Re z> + s w - M_k),
 * with the unit-modulus phase factor still built by repeated multiplication.  Directions dE and
 * dN are invariant under this row scaling.  Without `scaled` (M_k = 0) the term is literally
 * c * x^a * t^w with x^a and integer powers of t by repeated multiplication.
 *
 * Complex numbers are C99 `double complex`, stored interleaved (re, im) like complex128.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <limits.h>

typedef double complex cplx;

/* Largest n: per-point work arrays live on the stack.  Every entry point returns -1 (and
 * touches no output) for n outside [1, OR_NMAX]. */
#define OR_NMAX 32

/* ---------------------------------------------------------------------------------------- */
/* monomials                                                                                */
/* ---------------------------------------------------------------------------------------- */

/* x^a by repeated multiplication */
static cplx monomial(int n, const cplx *x, const cplx *xinv, const int8_t *a) {
    cplx r = 1.0;
    for (int j = 0; j < n; j++) {
        int e = a[j];
        for (int q = 0; q < e; q++) r *= x[j];
        for (int q = 0; q < -e; q++) r *= xinv[j];
    }
    return r;
}

/* t^w: repeated multiplication for integer w, exp(s w) otherwise */
static double lift_power(double s, double w) {
    if (w == floor(w) && w >= 0 && w <= 4096) {
        double t = exp(s), r = 1.0;
        for (int q = 0; q < (int)w; q++) r *= t;
        return r;
    }
    return exp(s * w);
}

/* ---------------------------------------------------------------------------------------- */
/* eval                                                                                      */
/* ---------------------------------------------------------------------------------------- */

/* One point.  G: n x (n+2) row-major; logscale: n (0 when unscaled); den (optional):
 * n x (n+2), den[k][col] = sum_a |term_a| * |C_a,col| with C_a = (a_1..a_n, w(a), 1). */
static void eval_point(int n, const int32_t *m, const int8_t *A, const double *w, const cplx *c,
                       const cplx *z, double s, int scaled, cplx *G, double *logscale,
                       double *den) {
    cplx x[OR_NMAX], xinv[OR_NMAX], u[OR_NMAX], uinv[OR_NMAX];
    for (int j = 0; j < n; j++) {
        x[j] = cexp(z[j]);
        xinv[j] = 1.0 / x[j];
        u[j] = cexp(I * cimag(z[j])); /* x_j / |x_j| */
        uinv[j] = conj(u[j]);
    }
    int off = 0;
    for (int k = 0; k < n; k++) {
        const int mk = m[k];
        double Mk = 0.0;
        if (scaled) {
            Mk = -INFINITY;
            for (int i = off; i < off + mk; i++) {
                double e = w[i] * s;
                for (int j = 0; j < n; j++) e += (double)A[(size_t)i * n + j] * creal(z[j]);
                if (e > Mk) Mk = e;
            }
        }
        cplx *row = G + (size_t)k * (n + 2);
        double *drow = den ? den + (size_t)k * (n + 2) : NULL;
        for (int col = 0; col < n + 2; col++) {
            row[col] = 0.0;
            if (drow) drow[col] = 0.0;
        }
        for (int i = off; i < off + mk; i++) {
            const int8_t *a = A + (size_t)i * n;
            cplx term;
            if (scaled) {
                /* polar form: phase by repeated multiplication of unit-modulus x_j/|x_j|,
                 * magnitude |x^a t^w| e^{-M_k} = exp(<a, Re z> + s w - M_k) */
                double lm = s * w[i] - Mk;
                for (int j = 0; j < n; j++) lm += (double)a[j] * creal(z[j]);
                term = c[i] * monomial(n, u, uinv, a) * exp(lm);
            } else {
                term = c[i] * monomial(n, x, xinv, a) * lift_power(s, w[i]);
            }
            for (int j = 0; j < n; j++) row[j] += (double)a[j] * term;
            row[n] += w[i] * term;
            row[n + 1] += term;
            if (drow) {
                double at = cabs(term);
                for (int j = 0; j < n; j++) drow[j] += fabs((double)a[j]) * at;
                drow[n] += fabs(w[i]) * at;
                drow[n + 1] += at;
            }
        }
        if (logscale) logscale[k] = Mk;
        off += mk;
    }
}

int oracle_eval(int n, const int32_t *m, const int8_t *A, const double *w, const double *c,
                int64_t P, const double *z, const double *s, int scaled, double *G,
                double *logscale, double *den, int threads) {
    if (n < 1 || n > OR_NMAX) return -1;
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
    for (int64_t p = 0; p < P; p++) {
        eval_point(n, m, A, w, (const cplx *)c, (const cplx *)z + p * n, s[p], scaled,
                   (cplx *)G + p * n * (n + 2), logscale ? logscale + p * n : NULL,
                   den ? den + p * n * (n + 2) : NULL);
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* solve                                                                                     */
/* ---------------------------------------------------------------------------------------- */

/* LU with partial pivoting (largest modulus, ties to the lowest row) of the n x n block of the
 * augmented n x (n+nrhs) matrix Gw (row stride ld), applied to the nrhs right-hand columns,
 * then back substitution.  X[r][j] (r-th rhs, j-th unknown) = -(J^{-1} rhs_r)_j.
 * Returns 0, or 1 if a pivot is exactly zero.  *ratio = min |pivot| / max |pivot|. */
static int lu_solve(int n, int nrhs, cplx *Gw, int ld, cplx *X, double *ratio) {
    double pmin = INFINITY, pmax = 0.0;
    for (int j = 0; j < n; j++) {
        int piv = j;
        double best = -1.0;
        for (int r = j; r < n; r++) {
            cplx v = Gw[r * ld + j];
            double mag = creal(v) * creal(v) + cimag(v) * cimag(v);
            if (mag > best) {
                best = mag;
                piv = r;
            }
        }
        if (!(best > 0.0)) {
            if (ratio) *ratio = 0.0;
            return 1;
        }
        if (piv != j)
            for (int col = 0; col < n + nrhs; col++) {
                cplx t = Gw[j * ld + col];
                Gw[j * ld + col] = Gw[piv * ld + col];
                Gw[piv * ld + col] = t;
            }
        double pm = sqrt(best);
        if (pm < pmin) pmin = pm;
        if (pm > pmax) pmax = pm;
        cplx inv = 1.0 / Gw[j * ld + j];
        for (int r = j + 1; r < n; r++) {
            cplx l = Gw[r * ld + j] * inv;
            for (int col = j + 1; col < n + nrhs; col++) Gw[r * ld + col] -= l * Gw[j * ld + col];
            Gw[r * ld + j] = 0.0;
        }
    }
    for (int q = 0; q < nrhs; q++) {
        for (int j = n - 1; j >= 0; j--) {
            cplx acc = Gw[j * ld + n + q];
            for (int col = j + 1; col < n; col++) acc -= Gw[j * ld + col] * X[q * n + col];
            X[q * n + j] = acc / Gw[j * ld + j];
        }
        for (int j = 0; j < n; j++) X[q * n + j] = -X[q * n + j];
    }
    if (ratio) *ratio = pmin / pmax;
    return 0;
}

/* one eval + consolidated 2-rhs solve at (z, s). */
static int step_point(int n, const int32_t *m, const int8_t *A, const double *w, const cplx *c,
                      const cplx *z, double s, cplx *dE, cplx *dN, double *ratio, double *resid) {
    cplx G[OR_NMAX * (OR_NMAX + 2)];
    double den[OR_NMAX * (OR_NMAX + 2)];
    eval_point(n, m, A, w, c, z, s, 1, G, NULL, den);
    if (resid) { /* relative backward error max_k |h_k| / sum_a |term_a| */
        double r = 0.0;
        for (int k = 0; k < n; k++) {
            double v = cabs(G[k * (n + 2) + n + 1]) / den[k * (n + 2) + n + 1];
            if (!(v <= r)) r = v;
        }
        *resid = r;
    }
    cplx X[2 * OR_NMAX];
    int st = lu_solve(n, 2, G, n + 2, X, ratio);
    for (int j = 0; j < n; j++) {
        dE[j] = st ? NAN : X[j];
        dN[j] = st ? NAN : X[n + j];
    }
    return st;
}

int oracle_step(int n, const int32_t *m, const int8_t *A, const double *w, const double *c,
                int64_t P, const double *z, const double *s, double *dE, double *dN,
                int32_t *status, double *ratio, int threads) {
    if (n < 1 || n > OR_NMAX) return -1;
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
    for (int64_t p = 0; p < P; p++) {
        double r;
        int st = step_point(n, m, A, w, (const cplx *)c, (const cplx *)z + p * n, s[p],
                            (cplx *)dE + p * n, (cplx *)dN + p * n, &r, NULL);
        status[p] = st ? -1 : 0;
        if (ratio) ratio[p] = r;
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* projective step                                                                            */
/* ---------------------------------------------------------------------------------------- */

/* Homogenising exponent of monomial a of equation k (Sec. 2.2): the homogenised exponent vector
 * is (a, d_k - sum_j a_j) with d_k = max over the monomials of equation k of sum_j a_j, so that
 * every monomial of h~_k has total degree d_k and the extra exponent is non-negative.  d [n]. */
static void homog_degrees(int n, const int32_t *m, const int8_t *A, int32_t *d) {
    int off = 0;
    for (int k = 0; k < n; k++) {
        int dk = INT32_MIN;
        for (int i = off; i < off + m[k]; i++) {
            int t = 0;
            for (int j = 0; j < n; j++) t += A[(size_t)i * n + j];
            if (t > dk) dk = t;
        }
        d[k] = dk;
        off += m[k];
    }
}

/* One point y in C^{n+1} (homogeneous coordinates; y_j pairs with a_j for j < n and y_n with the
 * homogenising exponent).  The homogenised homotopy (Sec. 2.2, eq. (3)) is
 *   h~_k(y, s) = sum_a c_{k,a} y^{(a, d_k - |a|)} e^{s w_k(a)},
 * its partials dh~_k/dy_j = sum_a e_j c y^{(a, d_k - |a|) - e_j} e^{s w} (e_j the j-th exponent),
 * dh~_k/ds = sum_a w c y^(...) e^{s w}.  The Euler and Newton directions in homogeneous
 * coordinates solve (eq. (4), (5); the unified system of Sec. 6)
 *   [ dH~/dy ; y^* ] dE = [ -dH~/ds ; 0 ],     [ dH~/dy ; y^* ] dN = [ -H~ ; 0 ],
 * an (n+1) x (n+1) system with two right-hand sides, solved here by LU with partial pivoting.
 * Row k of the equations is scaled by e^{-M_k} (M_k = max over its monomials of
 * <e, log|y|> + s w) so that no term over- or underflows; the solution does not depend on it.
 * The terms are formed in polar form: phase by repeated multiplication of y_j/|y_j|, magnitude
 * exp(<e, log|y|> + s w - M_k).  Returns 0, or 1 when a pivot is exactly zero. */
static int step_proj_point(int n, const int32_t *m, const int8_t *A, const double *w,
                           const cplx *c, const int32_t *d, const cplx *y, double s, cplx *dE,
                           cplx *dN, double *ratio) {
    const int nu = n + 1; /* unknowns */
    cplx u[OR_NMAX + 1], uinv[OR_NMAX + 1], yinv[OR_NMAX + 1];
    double ly[OR_NMAX + 1];
    for (int j = 0; j < nu; j++) {
        ly[j] = log(cabs(y[j]));
        u[j] = y[j] / cabs(y[j]);
        uinv[j] = conj(u[j]);
        yinv[j] = 1.0 / y[j];
    }
    /* augmented (n+1) x (n+3): [dH~/dy | -dH~/ds ... ] built as [dH~/dy | dH~/ds | H~] rows
     * for the equations and [y^* | 0 | 0] for the last row; lu_solve negates the right-hand
     * sides. */
    cplx G[(OR_NMAX + 1) * (OR_NMAX + 3)];
    const int ld = nu + 2;
    int off = 0;
    for (int k = 0; k < n; k++) {
        cplx *row = G + (size_t)k * ld;
        for (int col = 0; col < ld; col++) row[col] = 0.0;
        int8_t e[OR_NMAX + 1];
        double Mk = -INFINITY;
        for (int i = off; i < off + m[k]; i++) {
            int tot = 0;
            double lm = s * w[i];
            for (int j = 0; j < n; j++) {
                tot += A[(size_t)i * n + j];
                lm += A[(size_t)i * n + j] * ly[j];
            }
            lm += (double)(d[k] - tot) * ly[n];
            if (lm > Mk) Mk = lm;
        }
        for (int i = off; i < off + m[k]; i++) {
            int tot = 0;
            for (int j = 0; j < n; j++) {
                e[j] = A[(size_t)i * n + j];
                tot += e[j];
            }
            e[n] = (int8_t)(d[k] - tot);
            double lm = s * w[i] - Mk;
            for (int j = 0; j < nu; j++) lm += e[j] * ly[j];
            const cplx term = c[i] * monomial(nu, u, uinv, e) * exp(lm);
            for (int j = 0; j < nu; j++) row[j] += (double)e[j] * term * yinv[j];
            row[nu] += w[i] * term;
            row[nu + 1] += term;
        }
        off += m[k];
    }
    cplx *last = G + (size_t)n * ld;
    for (int j = 0; j < nu; j++) last[j] = conj(y[j]);
    last[nu] = 0.0;
    last[nu + 1] = 0.0;
    cplx X[2 * (OR_NMAX + 1)];
    int st = lu_solve(nu, 2, G, ld, X, ratio);
    for (int j = 0; j < nu; j++) {
        dE[j] = st ? NAN : X[j];
        dN[j] = st ? NAN : X[nu + j];
    }
    return st;
}

/* Projective Euler and Newton directions at P points y [P][n+1] (complex), s [P]; dE, dN
 * [P][n+1]; status 0 or -1 (a zero pivot); ratio min|pivot| / max|pivot| (optional).  The
 * homogenising degrees d [n] are written when d_out is not NULL.  The homogenising exponents must
 * fit int8 (|d_k - |a|| <= 127); returns -1 for n out of range, -2 otherwise. */
int oracle_step_proj(int n, const int32_t *m, const int8_t *A, const double *w, const double *c,
                     int64_t P, const double *y, const double *s, double *dE, double *dN,
                     int32_t *status, double *ratio, int32_t *d_out, int threads) {
    if (n < 1 || n > OR_NMAX) return -1;
    int32_t d[OR_NMAX];
    homog_degrees(n, m, A, d);
    int off = 0;
    for (int k = 0; k < n; k++) {
        for (int i = off; i < off + m[k]; i++) {
            int tot = 0;
            for (int j = 0; j < n; j++) tot += A[(size_t)i * n + j];
            if (d[k] - tot > 127) return -2;
        }
        off += m[k];
    }
    if (d_out)
        for (int k = 0; k < n; k++) d_out[k] = d[k];
    const int nu = n + 1;
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
    for (int64_t p = 0; p < P; p++) {
        double r;
        int st = step_proj_point(n, m, A, w, (const cplx *)c, d, (const cplx *)y + p * nu, s[p],
                                 (cplx *)dE + p * nu, (cplx *)dN + p * nu, &r);
        status[p] = st ? -1 : 0;
        if (ratio) ratio[p] = r;
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* track                                                                                     */
/* ---------------------------------------------------------------------------------------- */

/* Tracker constants.  Field for field the same meaning as the GPU library's parameters. */
typedef struct {
    double ds0, ds_max, ds_min;
    double tol_polish;  /* start-point Newton: stop when ||dN||_inf <= tol_polish */
    double tol_track;   /* corrector converged when ||dN||_inf <= tol_track */
    double tol_end;     /* endgame: stop when ||dN||_inf <= tol_end (1 + ||z||_inf) */
    double res_tol;     /* endpoint accepted when the relative residual <= res_tol */
    double div_re;      /* |Re z_j| > div_re => diverged */
    double sing_ratio;  /* min/max |pivot| below this => singular */
    double tol_predict; /* a predicted point whose first correction exceeds this is rejected */
    int max_polish, max_newton, max_end, max_steps, max_iters;
    int predictor;      /* 0: Euler; 1: cubic Hermite through the last two accepted points;
                           2: classical Runge-Kutta (three more evaluations per step) */
} or_params;

/* Cubic Hermite predictor (the predictor family of Sec. 2.3 built on the Euler direction): the
 * cubic through (s0, z0) and (s1, z1) with slopes e0 and e1 (dz/ds at those points, s0 < s1),
 * evaluated at s (past s1: an extrapolation).  With t = (s - s0) / (s1 - s0) and
 * d = s1 - s0 the Hermite basis gives
 *   z(s) = (2t^3 - 3t^2 + 1) z0 + (t^3 - 2t^2 + t) d e0 + (-2t^3 + 3t^2) z1 + (t^3 - t^2) d e1. */
static void hermite(int n, double s0, const cplx *z0, const cplx *e0, double s1, const cplx *z1,
                    const cplx *e1, double s, cplx *out) {
    const double d = s1 - s0, t = (s - s0) / d;
    const double t2 = t * t, t3 = t2 * t;
    const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + t;
    const double h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
    for (int j = 0; j < n; j++)
        out[j] = h00 * z0[j] + h10 * d * e0[j] + h01 * z1[j] + h11 * d * e1[j];
}

/* Classical fourth-order Runge-Kutta predictor (Sec. 2.3's Runge-Kutta family, built on the Euler
 * direction: dz/ds = dE(z, s)).  From the accepted point (z_a, s_a) with k1 = dE(z_a, s_a):
 *   k2 = dE(z_a + h/2 k1, s_a + h/2),  k3 = dE(z_a + h/2 k2, s_a + h/2),
 *   k4 = dE(z_a + h k3, s_a + h),       z = z_a + h/6 (k1 + 2 k2 + 2 k3 + k4).
 * Stage j = 1, 2, 3 evaluates at rk_stage_point(j); rk_accumulate adds its direction with the
 * weight of k_{j+1}. */
static double rk_stage_offset(int j, double h) { return j < 3 ? 0.5 * h : h; }
static void rk_stage_point(int n, int j, double h, const cplx *za, const cplx *k, cplx *z) {
    const double a = rk_stage_offset(j, h);
    for (int i = 0; i < n; i++) z[i] = za[i] + a * k[i];
}
static void rk_accumulate(int n, int j, const cplx *k, cplx *ksum) {
    const double wgt = j < 3 ? 2.0 : 1.0;
    for (int i = 0; i < n; i++) ksum[i] += wgt * k[i];
}
static void rk_finish(int n, double h, const cplx *za, const cplx *ksum, cplx *z) {
    for (int i = 0; i < n; i++) z[i] = za[i] + (h / 6.0) * ksum[i];
}

/* The Runge-Kutta predictor alone, for its tests: from (za[p], sa[p]) with step h[p], through the
 * same stage functions as the tracker.  Returns -1 for bad n; out[p] = NaN where a stage
 * evaluation is singular. */
int oracle_rk4_predict(int n, const int32_t *m, const int8_t *A, const double *w, const double *c,
                       int64_t P, const double *za, const double *sa, const double *h,
                       double *out) {
    if (n < 1 || n > OR_NMAX) return -1;
    for (int64_t p = 0; p < P; p++) {
        const cplx *z0 = (const cplx *)za + p * n;
        cplx *zo = (cplx *)out + p * n;
        cplx dE[OR_NMAX], dN[OR_NMAX], ksum[OR_NMAX], zs[OR_NMAX];
        double ratio;
        int bad = step_point(n, m, A, w, (const cplx *)c, z0, sa[p], dE, dN, &ratio, NULL);
        for (int i = 0; i < n; i++) ksum[i] = dE[i];
        for (int j = 1; j <= 3 && !bad; j++) {
            rk_stage_point(n, j, h[p], z0, dE, zs);
            bad = step_point(n, m, A, w, (const cplx *)c, zs, sa[p] + rk_stage_offset(j, h[p]), dE,
                             dN, &ratio, NULL);
            rk_accumulate(n, j, dE, ksum);
        }
        if (bad)
            for (int i = 0; i < n; i++) zo[i] = NAN;
        else
            rk_finish(n, h[p], z0, ksum, zo);
    }
    return 0;
}

/* The predictor alone, for its tests: P independent evaluations (complex arrays [P][n]). */
int oracle_hermite(int n, int64_t P, const double *s0, const double *z0, const double *e0,
                   const double *s1, const double *z1, const double *e1, const double *s,
                   double *out) {
    if (n < 1 || n > OR_NMAX) return -1;
    for (int64_t p = 0; p < P; p++)
        hermite(n, s0[p], (const cplx *)z0 + p * n, (const cplx *)e0 + p * n, s1[p],
                (const cplx *)z1 + p * n, (const cplx *)e1 + p * n, s[p], (cplx *)out + p * n);
    return 0;
}

enum { OR_OK = 0, OR_START = 1, OR_RUNNING = 2, OR_SINGULAR = -1, OR_STEP_MIN = -2,
       OR_DIVERGED = -3, OR_NONFINITE = -4, OR_POLISH_FAIL = -5, OR_ENDGAME_FAIL = -6,
       OR_MAX_ITERS = -7 };
enum { PH_POLISH = 0, PH_TRACK = 1, PH_END = 2, PH_RESUME = 3, PH_RK = 4 };

static double norm_inf(int n, const cplx *v) {
    double r = 0.0;
    for (int j = 0; j < n; j++) {
        double a = cabs(v[j]);
        if (!(a <= r)) r = a; /* propagates NaN */
    }
    return r;
}

/* Track one path.  z, s, ds in/out; status in/out (OR_START: polish first, OR_RUNNING: resume
 * at an accepted point with step ds); counters: steps, rejects, corrector iterations, evals. */
static void track_path(int n, const int32_t *m, const int8_t *A, const double *w, const cplx *c,
                       const or_params *pr, cplx *z, double *s_io, double *ds_io, int32_t *status,
                       int32_t *cnt) {
    if (*status != OR_START && *status != OR_RUNNING) return;
    cplx za[OR_NMAX], dEa[OR_NMAX], dE[OR_NMAX], dN[OR_NMAX];
    cplx zp[OR_NMAX], dEp[OR_NMAX]; /* the accepted point before (z_a, s_a), for the Hermite predictor */
    cplx ksum[OR_NMAX];              /* the Runge-Kutta predictor's weighted sum of directions */
    double s = *s_io, sa = s, ds = *ds_io, nrm_prev = 0.0, sp = 0.0, h_rk = 0.0, st_rk = 0.0;
    int rk = 0;                      /* the Runge-Kutta stage being evaluated (PH_RK) */
    int have_a = 0, have_p = 0;     /* accepted points held in (za, sa) and (zp, sp) */
    int phase = (*status == OR_START) ? PH_POLISH : PH_RESUME;
    if (*status == OR_START) ds = pr->ds0;
    int k = 0, steps_here = 0;
    for (int j = 0; j < n; j++) za[j] = z[j];
    for (int it = 0;; it++) {
        if (it >= pr->max_iters) { *status = OR_MAX_ITERS; break; }
        double ratio, resid;
        int sing = step_point(n, m, A, w, c, z, s, dE, dN, &ratio, &resid);
        cnt[3]++;
        double nrm = norm_inf(n, dN);
        if (sing || ratio < pr->sing_ratio) {
            if (phase == PH_TRACK || phase == PH_RK) goto reject; /* step back and shrink */
            *status = OR_SINGULAR;
            break;
        }
        if (!isfinite(nrm) || !isfinite(norm_inf(n, dE))) {
            if (phase == PH_TRACK || phase == PH_RK) goto reject;
            *status = OR_NONFINITE;
            break;
        }
        if (phase == PH_RK) {
            /* a Runge-Kutta stage point: its Euler direction is k_{rk+1}.  Like the predicted
             * point, every stage point must lie in the corrector's trust region (its Newton step
             * at most tol_predict); otherwise the stages have left the path's neighbourhood and
             * the step is rejected */
            if (nrm > pr->tol_predict) goto reject;
            rk_accumulate(n, rk, dE, ksum);
            if (rk < 3) {
                rk_stage_point(n, rk + 1, h_rk, za, dE, z);
                s = (rk + 1 < 3) ? sa + 0.5 * h_rk : st_rk;
                rk++;
            } else {
                rk_finish(n, h_rk, za, ksum, z);
                s = st_rk;
                k = 0;
                phase = PH_TRACK;
            }
            continue;
        }
        if (phase == PH_POLISH) {
            for (int j = 0; j < n; j++) z[j] += dN[j];
            k++;
            cnt[2]++;
            if (nrm <= pr->tol_polish) {
                /* on the path: accept (z, s) with the Euler direction just computed */
                phase = PH_RESUME;
                k = 0;
                continue; /* re-evaluate at the polished point before predicting */
            }
            if (k >= pr->max_polish) { *status = OR_POLISH_FAIL; break; }
            continue;
        }
        if (phase == PH_RESUME) {
            /* (z, s) is an accepted point: keep it and predict with its Euler direction */
            for (int j = 0; j < n; j++) { za[j] = z[j]; dEa[j] = dE[j]; }
            sa = s;
            have_a = 1;
            have_p = 0;
            if (sa >= 0.0) { phase = PH_END; k = 0; goto endgame; }
            if (steps_here >= pr->max_steps) { *status = OR_RUNNING; break; }
            goto predict;
        }
        if (phase == PH_END) goto endgame;

        /* PH_TRACK: corrector.  At the predicted point itself (no correction yet) the Newton
         * step measures how far the predictor left the path: beyond tol_predict the point may
         * lie nearer another path than its own, so the step is rejected before any correction */
        if (k == 0 && nrm > pr->tol_predict) goto reject;
        if (nrm <= pr->tol_track) {
            /* accept the evaluated point (the previous one is kept for the Hermite predictor) */
            if (have_a) {
                for (int j = 0; j < n; j++) { zp[j] = za[j]; dEp[j] = dEa[j]; }
                sp = sa;
                have_p = 1;
            }
            for (int j = 0; j < n; j++) { za[j] = z[j]; dEa[j] = dE[j]; }
            sa = s;
            have_a = 1;
            cnt[0]++;
            steps_here++;
            if (k <= 1) ds = fmin(2.0 * ds, pr->ds_max);
            if (sa >= 0.0) { phase = PH_END; k = 0; goto endgame; }
            if (steps_here >= pr->max_steps) { *status = OR_RUNNING; break; }
            goto predict;
        }
        if (k < pr->max_newton && (k == 0 || nrm <= 0.5 * nrm_prev)) {
            for (int j = 0; j < n; j++) z[j] += dN[j];
            k++;
            cnt[2]++;
            nrm_prev = nrm;
            int div = 0;
            for (int j = 0; j < n; j++) div |= fabs(creal(z[j])) > pr->div_re;
            if (div) { *status = OR_DIVERGED; break; }
            continue;
        }
    reject:
        cnt[1]++;
        ds *= 0.5;
        if (ds < pr->ds_min) { *status = OR_STEP_MIN; break; }
        for (int j = 0; j < n; j++) z[j] = za[j];
        s = sa;
    predict: {
        double h = fmin(ds, -sa);
        const double st = (h == -sa) ? 0.0 : sa + h;
        if (pr->predictor == 2) { /* Runge-Kutta: three stage evaluations first */
            for (int j = 0; j < n; j++) ksum[j] = dEa[j];
            h_rk = h;
            st_rk = st;
            rk = 1;
            rk_stage_point(n, 1, h, za, dEa, z);
            s = sa + 0.5 * h;
            phase = PH_RK;
            continue;
        }
        if (pr->predictor == 1 && have_p && h <= 4.0 * (sa - sp))
            hermite(n, sp, zp, dEp, sa, za, dEa, st, z);  /* cubic through the last two points */
        else
            for (int j = 0; j < n; j++) z[j] = za[j] + h * dEa[j];
        s = st;
        k = 0;
        phase = PH_TRACK;
        continue;
    }
    endgame:
        /* s = 0: Newton until the step is tiny or stops contracting */
        for (int j = 0; j < n; j++) z[j] += dN[j];
        cnt[2]++;
        k++;
        if (nrm <= pr->tol_end * (1.0 + norm_inf(n, z)) || k >= pr->max_end ||
            (k >= 3 && nrm > 0.5 * nrm_prev)) {
            *status = (resid <= pr->res_tol) ? OR_OK : OR_ENDGAME_FAIL;
            break;
        }
        nrm_prev = nrm;
        continue;
    }
    *s_io = s;
    *ds_io = ds;
}

/* Track P paths.  dparams: ds0, ds_max, ds_min, tol_polish, tol_track, tol_end, res_tol, div_re,
 * sing_ratio, tol_predict; iparams: max_polish, max_newton, max_end, max_steps, max_iters,
 * predictor (0 Euler, 1 cubic Hermite, 2 Runge-Kutta). */
int oracle_track(int n, const int32_t *m, const int8_t *A, const double *w, const double *c,
                 int64_t P, double *z, double *s, double *ds, const double *dparams,
                 const int32_t *iparams, int32_t *status, int32_t *counters, int threads) {
    if (n < 1 || n > OR_NMAX) return -1;
    or_params pr;
    pr.ds0 = dparams[0];
    pr.ds_max = dparams[1];
    pr.ds_min = dparams[2];
    pr.tol_polish = dparams[3];
    pr.tol_track = dparams[4];
    pr.tol_end = dparams[5];
    pr.res_tol = dparams[6];
    pr.div_re = dparams[7];
    pr.sing_ratio = dparams[8];
    pr.tol_predict = dparams[9];
    pr.max_polish = iparams[0];
    pr.max_newton = iparams[1];
    pr.max_end = iparams[2];
    pr.max_steps = iparams[3];
    pr.max_iters = iparams[4];
    pr.predictor = iparams[5];
#pragma omp parallel for schedule(dynamic, 16) num_threads(threads > 0 ? threads : 1)
    for (int64_t p = 0; p < P; p++)
        track_path(n, m, A, w, (const cplx *)c, &pr, (cplx *)z + p * n, s + p, ds + p,
                   status + p, counters + 4 * p);
    return 0;
}

/* ---------------------------------------------------------------------------------------- */
/* residual at t = 1 and endpoint gradient                                                   */
/* ---------------------------------------------------------------------------------------- */

/* relative backward error r(x) = max_k |f_k(x)| / sum_a |c_{k,a} x^a| at t = 1 */
int oracle_residual(int n, const int32_t *m, const int8_t *A, const double *c, int64_t P,
                    const double *z, double *out, int threads) {
    if (n < 1 || n > OR_NMAX) return -1;
#pragma omp parallel for schedule(static) num_threads(threads > 0 ? threads : 1)
    for (int64_t p = 0; p < P; p++) {
        const cplx *zp = (const cplx *)z + p * n;
        cplx x[OR_NMAX], xinv[OR_NMAX];
        for (int j = 0; j < n; j++) {
            x[j] = cexp(zp[j]);
            xinv[j] = 1.0 / x[j];
        }
        double r = 0.0;
        int off = 0;
        for (int k = 0; k < n; k++) {
            cplx f = 0.0;
            double a = 0.0;
            for (int i = off; i < off + m[k]; i++) {
                cplx t = ((const cplx *)c)[i] * monomial(n, x, xinv, A + (size_t)i * n);
                f += t;
                a += cabs(t);
            }
            double v = cabs(f) / a;
            if (!(v <= r)) r = v;
            off += m[k];
        }
        out[p] = r;
    }
    return 0;
}

/* grad_c (M complex) of L(x*) with upstream g = dL/dRe x + i dL/dIm x at the endpoints.
 * Per path: J_x^H nu = -g with J_x = J_z diag(e^{-z}), i.e. J_z^H nu = -conj(x) . g; then
 * grad c_{k,a} += nu_k conj(x^a).  Paths are summed in index order.  Returns the number of
 * paths whose Jacobian was singular (they are skipped), or -1 when n is out of range. */
int oracle_endpoint_grad(int n, const int32_t *m, const int8_t *A, const double *w,
                         const double *c, int64_t P, const double *z_end, const double *grad_x,
                         double *grad_c) {
    if (n < 1 || n > OR_NMAX) return -1;
    int M = 0;
    for (int k = 0; k < n; k++) M += m[k];
    cplx *gc = (cplx *)grad_c;
    for (int i = 0; i < M; i++) gc[i] = 0.0;
    int nsing = 0;
    for (int64_t p = 0; p < P; p++) {
        const cplx *zp = (const cplx *)z_end + p * n;
        const cplx *gp = (const cplx *)grad_x + p * n;
        cplx G[OR_NMAX * (OR_NMAX + 2)];
        double Ms[OR_NMAX];
        eval_point(n, m, A, w, (const cplx *)c, zp, 0.0, 1, G, Ms, NULL);
        /* scaled rows: Js = diag(e^{-M}) J_z, so Js^H mu = -conj(x).g with nu = e^{-M} mu */
        cplx H[OR_NMAX * (OR_NMAX + 1)];
        for (int r = 0; r < n; r++) {
            for (int col = 0; col < n; col++) H[r * (n + 1) + col] = conj(G[col * (n + 2) + r]);
            H[r * (n + 1) + n] = conj(cexp(zp[r])) * gp[r];
        }
        cplx mu[OR_NMAX];
        if (lu_solve(n, 1, H, n + 1, mu, NULL)) { /* mu = -Js^{-H} (conj(x).g) */
            nsing++;
            continue;
        }
        cplx x[OR_NMAX], xinv[OR_NMAX];
        for (int j = 0; j < n; j++) {
            x[j] = cexp(zp[j]);
            xinv[j] = 1.0 / x[j];
        }
        int off = 0;
        for (int k = 0; k < n; k++) {
            cplx nu = mu[k] * exp(-Ms[k]);
            for (int i = off; i < off + m[k]; i++)
                gc[i] += nu * conj(monomial(n, x, xinv, A + (size_t)i * n));
            off += m[k];
        }
    }
    return nsing;
}
