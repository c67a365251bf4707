/*
 * bfm_oracle.c -- plain FP64 CPU oracle for BFAST Monitor.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or helper
 * with the GPU library: it rebuilds everything from the paper's definitions.
 *
 * What it computes, per pixel (one series y_1..y_N), in the paper's order and
 * notation (Section 2.1, Algorithm 1):
 *   1. design rows x_t = (1, t, sin(2 pi 1 t/f), cos(2 pi 1 t/f), ...,
 *      sin(2 pi k t/f), cos(2 pi k t/f)), t = 1..N           (Eq. 1, Eq. 2)
 *   2. least-squares fit of y_1..y_n on x_1..x_n              (Eq. 5, Eq. 6)
 *      solved by Householder QR (same minimiser as the pseudo-inverse of Eq. 6)
 *      with one step of iterative refinement
 *   3. residuals r_t = y_t - x_t' beta                         (Eq. 11)
 *   4. sigma = sqrt(sum_{t<=n} r_t^2 / (n - (2+2k)))           (Alg. 1, step 5)
 *   5. MO_t = (1/(sigma sqrt(n))) sum_{s=t-h+1..t} r_s,  t = n+1..N, each
 *      window summed from scratch (no recurrence)             (Eq. 3)
 *   6. b_t = lambda sqrt(log+(t/n)), log+ x = 1 if x <= e else ln x  (Eq. 4)
 *   7. first t with |MO_t| > b_t (strict)                      (Alg. 1, step 13)
 *      and the MOSUM value of largest magnitude                (Section 4, Chile
 *      heat map of the maximum absolute MOSUM values)
 *
 * Readings where the paper is silent or inconsistent (each one is also listed
 * in the design notes of the repository):
 *   - the window holds h observations s = t-h+1..t (Eq. 3 and the kernel
 *     listing agree; Algorithm 1 step 7 writes t-h..t, taken as a typo);
 *   - residual sign is y - yhat (Eq. 11 and the listing; Algorithm 1 step 4
 *     writes yhat - y).  The sign only flips MO and the magnitude;
 *   - h may be given as a count (h_window > 0) or as a fraction of the
 *     history (H = floor(h_frac * n));
 *   - missing observations (future work in Section 5; the footnote in
 *     Section 3 fills them) are DROPPED: the pixel's series is its valid
 *     observations in time order, design rows keep their original t, the
 *     history is the valid observations with t <= n (n_v of them), and the
 *     window, the normaliser and the boundary use compacted counts:
 *     H = floor(h_frac * n_v), sqrt(n_v), u / n_v with u the compacted
 *     position.  The break index reports the original monitor position;
 *   - magnitude: with hi = max MO and lo = min MO over the valid monitor
 *     observations, mag = hi if hi >= -lo, else lo;
 *   - a pixel whose residual scale is at most 1e-6 * max|y_hist| is
 *     DEGENERATE_SIGMA (an exact season-trend series has no MOSUM);
 *   - a history design is RANK_DEFICIENT when, with the trend column divided
 *     by n and the columns in the order of Eq. 2, its QR factor has some
 *     |R_jj| <= 1e-6 * sqrt(n_v);
 *   - irregular time (Section 4, the Chile scene): when a vector of
 *     observation times is given, the design rows of Eq. 2 take the time of
 *     each observation (there: its day number, f = 365) in place of the index
 *     t, while the history, the window h, the boundary's t/n and the break
 *     index stay counts of observations.  The trend column is then divided by
 *     (t_n - t_1) n / (n - 1), which is n for t = 1..N;
 *   - filling (the footnote of Section 3): each non-finite observation takes
 *     the value of the last finite one before it (forward fill); those before
 *     the first finite one take that one (backward fill).  The filled series
 *     then goes through the plain path; a series with no finite value is
 *     INSUFFICIENT.
 *
 * Parity: every function here is pinned by the CPU test suite against closed
 * forms, invariants, LAPACK least squares and brute force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define BFO_MASK_NONE 0
#define BFO_MASK_NAN 1
#define BFO_MASK_EXPLICIT 2
#define BFO_MASK_FILL 3

#define BFO_OK 0
#define BFO_NONFINITE 1
#define BFO_INSUFFICIENT 2
#define BFO_RANK_DEFICIENT 3
#define BFO_DEGENERATE_SIGMA 4
#define BFO_NO_MONITOR 5

#define BFO_SIGMA_REL_TOL 1e-6
#define BFO_RANK_TOL 1e-6

typedef struct {
    int32_t n_obs;    /* N: series length                        */
    int32_t n_hist;   /* n: history length, 1 <= n < N            */
    int32_t order;    /* k: number of harmonic terms, p = 2 + 2k  */
    double freq;      /* f: observations per year                 */
    double h_frac;    /* window as a fraction of the history      */
    int32_t h_window; /* window as a count; overrides h_frac if > 0 */
    double lambda;    /* critical value of the boundary           */
    int32_t mask_mode;
    const double *times; /* NULL: t = 1..N; else the time of each observation */
} bfo_params;

/* Eq. 2: one design row at time t (the 1-based index, or the observation's
 * time when times are given).  sin and cos of 2 pi j t / f are periodic in
 * j t with period f, so j t is first reduced modulo f (fmod is exact) and the
 * angle is formed from the remainder: the same values, without the rounding
 * of an angle that grows with t (about 1e-13 at t = 400, which shows in the
 * MOSUM when the noise is small). */
static void design_row(double t, int k, double f, double *x)
{
    x[0] = 1.0;
    x[1] = (double)t;
    for (int j = 1; j <= k; ++j) {
        double ang = 2.0 * M_PI * fmod((double)j * (double)t, f) / f;
        x[2 * j] = sin(ang);
        x[2 * j + 1] = cos(ang);
    }
}

/* Eq. 4: log+ and the boundary. */
static double log_plus(double x) { return x <= M_E ? 1.0 : log(x); }
static double boundary(double lambda, double ratio) { return lambda * sqrt(log_plus(ratio)); }

/*
 * Least squares min ||A beta - b|| (Eq. 5) by Householder QR, columns in the
 * order of Eq. 2.  A is m x p, row-major, overwritten.  The trend column is
 * divided by tscale (the history length) before the factorisation so that
 * every column has entries of order one; this leaves the fitted values
 * unchanged and makes the rank test |R_jj| <= tol * sqrt(m) independent of the
 * units of t.  Returns 0, or -1 if the history design is rank deficient.
 */
static int householder_lstsq(double *A, double *b, int m, int p, double tscale, double *beta)
{
    const double tol = BFO_RANK_TOL * sqrt((double)m);
    for (int i = 0; i < m; ++i) A[i * p + 1] /= tscale;
    for (int j = 0; j < p; ++j) {
        double norm = 0.0;
        for (int i = j; i < m; ++i) norm += A[i * p + j] * A[i * p + j];
        norm = sqrt(norm);
        if (norm <= tol) return -1;
        double alpha = A[j * p + j] > 0 ? -norm : norm; /* R_jj */
        /* v = x - alpha e1, stored in column j below the diagonal */
        A[j * p + j] -= alpha;
        double vtv = 0.0;
        for (int i = j; i < m; ++i) vtv += A[i * p + j] * A[i * p + j];
        /* apply (I - 2 v v'/v'v) to the remaining columns and to b */
        for (int c = j + 1; c < p; ++c) {
            double d = 0.0;
            for (int i = j; i < m; ++i) d += A[i * p + j] * A[i * p + c];
            d = 2.0 * d / vtv;
            for (int i = j; i < m; ++i) A[i * p + c] -= d * A[i * p + j];
        }
        double d = 0.0;
        for (int i = j; i < m; ++i) d += A[i * p + j] * b[i];
        d = 2.0 * d / vtv;
        for (int i = j; i < m; ++i) b[i] -= d * A[i * p + j];
        A[j * p + j] = alpha;
    }
    /* back substitution R beta~ = (Q'b)[0:p] */
    for (int j = p - 1; j >= 0; --j) {
        double s = b[j];
        for (int c = j + 1; c < p; ++c) s -= A[j * p + c] * beta[c];
        beta[j] = s / A[j * p + j];
    }
    beta[1] /= tscale;
    return 0;
}

/* Time of the observation with 1-based index t. */
static double time_of(const bfo_params *prm, int t)
{
    return prm->times ? prm->times[t - 1] : (double)t;
}

/* Divisor of the trend column in the factorisation: n for t = 1..N. */
static double trend_scale(const bfo_params *prm)
{
    const int n = prm->n_hist;
    if (!prm->times || n < 2) return (double)n;
    return (prm->times[n - 1] - prm->times[0]) * (double)n / (double)(n - 1);
}

typedef struct {
    int32_t *brk;
    double *mag;
    double *sigma;
    uint8_t *status;
    double *beta;  /* p x P, coefficient-major (beta_all of Eq. 8)  */
    double *resid; /* N x P, time-major                             */
    double *mosum; /* (N-n) x P, time-major                         */
} bfo_outputs;

static void pixel(const bfo_params *prm, const float *Y, const double *Yd, int64_t P,
                  int64_t ld, const uint8_t *valid, int64_t ldv, int64_t i,
                  const bfo_outputs *o)
{
    const int N = prm->n_obs, n = prm->n_hist, k = prm->order, p = 2 + 2 * k;
    const int M = N - n;
    double *y = malloc(sizeof(double) * N);
    int *tv = malloc(sizeof(int) * N);      /* valid times, 1-based, in order */
    double *e = malloc(sizeof(double) * N); /* residuals of valid times, compacted */
    double *A = malloc(sizeof(double) * (size_t)N * p);
    double *rhs = malloc(sizeof(double) * N);
    double beta[64], x[64];
    uint8_t st = BFO_OK;
    double sig = NAN;

    for (int t = 0; t < N; ++t)
        y[t] = Yd ? Yd[(int64_t)t * ld + i] : (double)Y[(int64_t)t * ld + i];
    if (prm->mask_mode == BFO_MASK_FILL) {
        /* footnote of Section 3: forward fill, then backward fill of the
         * leading gap from the first finite value */
        double last = NAN;
        for (int t = 0; t < N; ++t) {
            if (isfinite(y[t])) last = y[t];
            else y[t] = last;
        }
        double next = NAN;
        for (int t = N - 1; t >= 0; --t) {
            if (isfinite(y[t])) next = y[t];
            else y[t] = next;
        }
        if (N > 0 && !isfinite(y[0])) st = BFO_INSUFFICIENT; /* no finite value at all */
    }
    if (o->resid)
        for (int t = 0; t < N; ++t) o->resid[(int64_t)t * P + i] = NAN;
    if (o->mosum)
        for (int t = 0; t < M; ++t) o->mosum[(int64_t)t * P + i] = NAN;
    if (o->beta)
        for (int j = 0; j < p; ++j) o->beta[(int64_t)j * P + i] = NAN;

    /* valid set V (drop semantics for missing observations) */
    int nv_all = 0, nv = 0;
    for (int t = 1; t <= N; ++t) {
        double v = y[t - 1];
        int use;
        if (prm->mask_mode == BFO_MASK_NONE || prm->mask_mode == BFO_MASK_FILL) {
            use = 1;
            if (!isfinite(v) && st == BFO_OK) st = BFO_NONFINITE;
        } else if (prm->mask_mode == BFO_MASK_NAN) {
            use = isfinite(v);
        } else {
            use = valid[(int64_t)(t - 1) * ldv + i] != 0;
            if (use && !isfinite(v)) st = BFO_NONFINITE;
        }
        if (use) {
            tv[nv_all++] = t;
            if (t <= n) ++nv;
        }
    }
    int H = prm->h_window > 0 ? prm->h_window : (int)floor(prm->h_frac * (double)nv);
    if (st == BFO_OK && (nv <= p || H < 1 || H > nv)) st = BFO_INSUFFICIENT;

    if (st == BFO_OK) {
        /* Eq. 5/6: fit on the valid history */
        for (int u = 0; u < nv; ++u) {
            design_row(time_of(prm, tv[u]), k, prm->freq, A + (size_t)u * p);
            rhs[u] = y[tv[u] - 1];
        }
        if (householder_lstsq(A, rhs, nv, p, trend_scale(prm), beta) != 0) st = BFO_RANK_DEFICIENT;
    }
    if (st == BFO_OK) {
        /* One step of iterative refinement: the least-squares fit of the first
         * solution's residuals corrects the coefficients towards the minimiser
         * of Eq. 5 (the first solve is off by the rounding unit times the
         * conditioning of the design, which shows at high signal-to-noise). */
        double dbeta[64];
        for (int u = 0; u < nv; ++u) {
            design_row(time_of(prm, tv[u]), k, prm->freq, x);
            double yh = 0.0;
            for (int j = 0; j < p; ++j) yh += x[j] * beta[j];
            rhs[u] = y[tv[u] - 1] - yh;
            memcpy(A + (size_t)u * p, x, sizeof(double) * p);
        }
        householder_lstsq(A, rhs, nv, p, trend_scale(prm), dbeta);
        for (int j = 0; j < p; ++j) beta[j] += dbeta[j];
    }
    if (st == BFO_OK) {
        if (o->beta)
            for (int j = 0; j < p; ++j) o->beta[(int64_t)j * P + i] = beta[j];
        /* Eq. 11: residuals of every valid observation */
        for (int u = 0; u < nv_all; ++u) {
            design_row(time_of(prm, tv[u]), k, prm->freq, x);
            double yh = 0.0;
            for (int j = 0; j < p; ++j) yh += x[j] * beta[j];
            e[u] = y[tv[u] - 1] - yh;
            if (o->resid) o->resid[(int64_t)(tv[u] - 1) * P + i] = e[u];
        }
        /* Algorithm 1 step 5 */
        double rss = 0.0, ymax = 0.0;
        for (int u = 0; u < nv; ++u) {
            rss += e[u] * e[u];
            double a = fabs(y[tv[u] - 1]);
            if (a > ymax) ymax = a;
        }
        sig = sqrt(rss / (double)(nv - p));
        if (sig <= BFO_SIGMA_REL_TOL * ymax) st = BFO_DEGENERATE_SIGMA;
        else if (nv_all == nv) st = BFO_NO_MONITOR;
    }
    int brk = -1;
    double mag = NAN;
    if (st == BFO_OK) {
        /* Eq. 3 with brute-force windows; Eq. 4 boundary; first crossing */
        double norm = sig * sqrt((double)nv);
        double hi = -INFINITY, lo = INFINITY;
        for (int u = nv; u < nv_all; ++u) { /* u is 0-based compacted index */
            double s = 0.0;
            for (int w = u - H + 1; w <= u; ++w) s += e[w];
            double mo = s / norm;
            if (o->mosum) o->mosum[(int64_t)(tv[u] - n - 1) * P + i] = mo;
            double b = boundary(prm->lambda, (double)(u + 1) / (double)nv);
            if (brk < 0 && fabs(mo) > b) brk = tv[u] - n - 1;
            if (mo > hi) hi = mo;
            if (mo < lo) lo = mo;
        }
        mag = hi >= -lo ? hi : lo;
    }
    if (o->brk) o->brk[i] = brk;
    if (o->mag) o->mag[i] = mag;
    if (o->sigma) o->sigma[i] = sig;
    if (o->status) o->status[i] = st;
    free(y);
    free(tv);
    free(e);
    free(A);
    free(rhs);
}

static int run(const bfo_params *prm, const float *Y, const double *Yd, int64_t P,
               int64_t ld, const uint8_t *valid, int64_t ldv, int32_t *brk, double *mag,
               double *sigma, uint8_t *status, double *beta, double *resid, double *mosum,
               int nthreads)
{
    if (!prm || (!Y && !Yd) || P < 0 || ld < P) return -1;
    if (prm->n_hist < 1 || prm->n_obs <= prm->n_hist) return -1;
    if (prm->order < 0 || 2 + 2 * prm->order > 64 || !(prm->freq > 0)) return -1;
    if (!(prm->lambda > 0)) return -1;
    if (prm->h_window <= 0 && !(prm->h_frac > 0 && prm->h_frac <= 1)) return -1;
    if (prm->h_window > prm->n_hist) return -1;
    if (prm->mask_mode < 0 || prm->mask_mode > 3) return -1;
    if (prm->times)
        for (int t = 0; t < prm->n_obs; ++t)
            if (!isfinite(prm->times[t]) || (t > 0 && !(prm->times[t] > prm->times[t - 1])))
                return -1; /* times must be finite and strictly increasing */
    if (prm->mask_mode == BFO_MASK_EXPLICIT && (!valid || ldv < P)) return -1;
    bfo_outputs o = {brk, mag, sigma, status, beta, resid, mosum};
#ifdef _OPENMP
    if (nthreads < 1) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < P; ++i) pixel(prm, Y, Yd, P, ld, valid, ldv, i, &o);
    return 0;
}

/*
 * Run the oracle over P pixels.  Y is time-major: pixel i at time t (0-based)
 * is Y[t*ld + i].  valid (EXPLICIT mode only) uses the same indexing with ldv.
 * Every output pointer may be NULL.  Returns 0, or -1 on invalid parameters.
 */
int bfo_fit_monitor(const bfo_params *prm, const float *Y, int64_t P, int64_t ld,
                    const uint8_t *valid, int64_t ldv, int32_t *brk, double *mag,
                    double *sigma, uint8_t *status, double *beta, double *resid,
                    double *mosum, int nthreads)
{
    return run(prm, Y, NULL, P, ld, valid, ldv, brk, mag, sigma, status, beta, resid, mosum,
               nthreads);
}

/* The same on FP64 observations (used by the pins to avoid FP32 input rounding). */
int bfo_fit_monitor_f64(const bfo_params *prm, const double *Y, int64_t P, int64_t ld,
                        const uint8_t *valid, int64_t ldv, int32_t *brk, double *mag,
                        double *sigma, uint8_t *status, double *beta, double *resid,
                        double *mosum, int nthreads)
{
    return run(prm, NULL, Y, P, ld, valid, ldv, brk, mag, sigma, status, beta, resid, mosum,
               nthreads);
}

/* Threads the oracle would use for a request of nthreads (<1: all). */
int bfo_threads(int nthreads)
{
#ifdef _OPENMP
    return nthreads < 1 ? omp_get_max_threads() : nthreads;
#else
    (void)nthreads;
    return 1;
#endif
}

/* Eq. 2 and Eq. 4 exposed for the pins. */
void bfo_design_row(double t, int k, double f, double *x) { design_row(t, k, f, x); }
double bfo_boundary(double lambda, double ratio) { return boundary(lambda, ratio); }
