/* Driver for the sanitizer build of the oracle (tests/test_oracle_sanitize.py): runs every entry
 * point of oracle/hom_oracle.c on small seeded systems, including n = 32 (the largest the oracle
 * accepts) and n = 33 (rejected), under AddressSanitizer and UndefinedBehaviorSanitizer.  The
 * values are not checked here (the pins do that); the sanitizers check the memory accesses and
 * the arithmetic's defined behaviour. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_eval(int n, const int32_t *m, const int8_t *A, const double *w, const double *c,
                int64_t P, const double *z, const double *s, int scaled, double *G,
                double *logscale, double *den, int threads);
int oracle_step(int n, const int32_t *m, const int8_t *A, const double *w, const double *c,
                int64_t P, const double *z, const double *s, double *dE, double *dN,
                int32_t *status, double *ratio, int threads);
int oracle_track(int n, const int32_t *m, const int8_t *A, const double *w, const double *c,
                 int64_t P, double *z, double *s, double *ds, const double *dparams,
                 const int32_t *iparams, int32_t *status, int32_t *counters, int threads);
int oracle_residual(int n, const int32_t *m, const int8_t *A, const double *c, int64_t P,
                    const double *z, double *out, int threads);
int oracle_endpoint_grad(int n, const int32_t *m, const int8_t *A, const double *w,
                         const double *c, int64_t P, const double *z_end, const double *grad_x,
                         double *grad_c);
int oracle_rk4_predict(int n, const int32_t *m, const int8_t *A, const double *w, const double *c,
                       int64_t P, const double *za, const double *sa, const double *h,
                       double *out);

static uint64_t rng_state = 88172645463325252ull;
static double urand(void) { /* xorshift64, uniform in [0, 1) */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

/* one random system with n unknowns, mk monomials per equation, and P random points */
static int run(int n, int mk, int P, int threads, int track) {
    const int M = n * mk;
    int32_t *m = malloc(sizeof *m * n);
    int8_t *A = malloc((size_t)M * n);
    double *w = malloc(sizeof *w * M), *c = malloc(sizeof *c * 2 * M);
    double *z = malloc(sizeof *z * 2 * P * n), *s = malloc(sizeof *s * P);
    double *G = malloc(sizeof *G * 2 * P * n * (n + 2)), *L = malloc(sizeof *L * P * n);
    double *den = malloc(sizeof *den * P * n * (n + 2));
    double *dE = malloc(sizeof *dE * 2 * P * n), *dN = malloc(sizeof *dN * 2 * P * n);
    double *ratio = malloc(sizeof *ratio * P), *res = malloc(sizeof *res * P);
    double *ds = malloc(sizeof *ds * P), *gx = malloc(sizeof *gx * 2 * P * n);
    double *gc = malloc(sizeof *gc * 2 * M);
    int32_t *st = malloc(sizeof *st * P), *cnt = malloc(sizeof *cnt * 4 * P);
    for (int k = 0; k < n; k++) m[k] = mk;
    for (int i = 0; i < M * n; i++) A[i] = (int8_t)((int)(urand() * 5.0) - 2);
    for (int i = 0; i < M; i++) {
        w[i] = floor(urand() * 8.0);
        c[2 * i] = cos(6.283 * urand());
        c[2 * i + 1] = sin(6.283 * urand());
    }
    for (int p = 0; p < P; p++) {
        for (int j = 0; j < n; j++) {
            z[2 * (p * n + j)] = 0.5 * (urand() - 0.5);
            z[2 * (p * n + j) + 1] = 6.283 * urand();
            gx[2 * (p * n + j)] = urand();
            gx[2 * (p * n + j) + 1] = urand();
        }
        s[p] = -8.0 * urand();
        ds[p] = 0.0;
        st[p] = 1;
    }
    int bad = 0;
    bad |= oracle_eval(n, m, A, w, c, P, z, s, 1, G, L, den, threads) != 0;
    bad |= oracle_eval(n, m, A, w, c, P, z, s, 0, G, NULL, NULL, threads) != 0;
    bad |= oracle_step(n, m, A, w, c, P, z, s, dE, dN, st, ratio, threads) != 0;
    bad |= oracle_residual(n, m, A, c, P, z, res, threads) != 0;
    bad |= oracle_endpoint_grad(n, m, A, w, c, P, z, gx, gc) < 0;
    if (track) { /* short budgets: exercise every phase without waiting for convergence */
        const double dp[10] = {0.05, 0.5, 1e-10, 1e-12, 1e-8, 1e-14, 1e-10, 40.0, 1e-14, 1e-2};
        const int32_t ip[6] = {10, 3, 8, 50, 200, 1};
        for (int p = 0; p < P; p++) st[p] = 1;
        bad |= oracle_track(n, m, A, w, c, P, z, s, ds, dp, ip, st, cnt, threads) != 0;
        const int32_t ip_rk[6] = {10, 3, 8, 50, 200, 2}; /* the Runge-Kutta predictor */
        for (int p = 0; p < P; p++) { st[p] = 1; s[p] = -8.0 * urand(); }
        bad |= oracle_track(n, m, A, w, c, P, z, s, ds, dp, ip_rk, st, cnt, threads) != 0;
    }
    for (int p = 0; p < P; p++) ds[p] = 0.1; /* the steps of the predictor alone */
    bad |= oracle_rk4_predict(n, m, A, w, c, P, z, s, ds, dE) != 0;
    /* out-of-range n is rejected before any array is touched */
    bad |= oracle_eval(n + 40, m, A, w, c, P, z, s, 1, G, L, den, threads) != -1;
    bad |= oracle_residual(0, m, A, c, P, z, res, threads) != -1;
    free(m); free(A); free(w); free(c); free(z); free(s); free(G); free(L); free(den);
    free(dE); free(dN); free(ratio); free(res); free(ds); free(gx); free(gc); free(st); free(cnt);
    return bad;
}

int main(void) {
    int bad = 0;
    bad |= run(3, 4, 64, 2, 1);
    bad |= run(8, 16, 16, 2, 1);
    bad |= run(32, 3, 4, 2, 0);
    bad |= oracle_eval(33, NULL, NULL, NULL, NULL, 1, NULL, NULL, 1, NULL, NULL, NULL, 1) != -1;
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
