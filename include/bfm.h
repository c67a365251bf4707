/*
 * bfm.h -- C ABI of libbfm, BFAST Monitor on AMD MI355X (gfx950).
 *
 * For every pixel of a stacked image time series the library fits the
 * season-trend model of the paper (Eq. 1, written as the linear model of
 * Eq. 2) on the stable history period by least squares (Eq. 5-6), forms the
 * residuals and their scale (Algorithm 1, steps 3-5), the MOSUM of residuals
 * over the monitoring period (Eq. 3), and tests it against the boundary of
 * Eq. 4.  Each pixel yields its first break index, the MOSUM value of largest
 * magnitude (the quantity mapped in the paper's Chile heat map, Section 4) and
 * a status code.  The batched form of Section 3 (Eq. 7-11: one shared
 * operator for all pixels) is what makes the GPU path a streaming pass.
 *
 * Conventions shared by every entry point:
 *   - All array pointers are DEVICE pointers owned by the caller, except where
 *     a comment says "host".  The library never frees them.
 *   - Series are time-major (the N x m layout of Section 3): the observation
 *     of pixel i at time t (t = 0..N-1, i.e. the paper's time t+1) is
 *     Y[t*ld + i], with ld >= P.  Per-time optional outputs use ld = P.
 *   - Functions return BFM_SUCCESS (0) or a negative BFM_E_* code; the text of
 *     the last error of the calling thread is returned by bfm_last_error().
 *   - Conditions of single pixels are not errors: they go to the per-pixel
 *     status array (BFM_ST_*), and such pixels get brk = -1 and mag = NaN.
 */
#ifndef BFM_H
#define BFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BFM_VERSION 3

/* return codes */
#define BFM_SUCCESS 0
#define BFM_E_INVAL (-1)       /* an argument violates the contract below   */
#define BFM_E_LAYOUT (-2)      /* ld or ldv smaller than P                  */
#define BFM_E_NOMEM (-3)       /* device or host allocation failed          */
#define BFM_E_NODEVICE (-4)    /* no such HIP device                        */
#define BFM_E_HIP (-5)         /* a HIP runtime call failed                 */
#define BFM_E_UNSUPPORTED (-6) /* device is not gfx950, or option not built  */

/* how missing observations are found and treated (MASK_NAN and
 * MASK_EXPLICIT drop them; MASK_FILL fills them) */
#define BFM_MASK_NONE 0     /* every observation is used; a non-finite one
                               makes the pixel BFM_ST_NONFINITE            */
#define BFM_MASK_NAN 1      /* an observation is used iff it is finite      */
#define BFM_MASK_EXPLICIT 2 /* used iff valid[t*ldv+i] != 0; a non-finite
                               used observation makes the pixel NONFINITE  */
#define BFM_MASK_FILL 3     /* the footnote of Section 3: a non-finite
                               observation takes the value of the last
                               finite one before it, those before the first
                               finite one take that one, and the filled
                               series goes through the plain path; a series
                               with no finite value is BFM_ST_INSUFFICIENT.
                               float32 series, order <= 8                  */

/* arithmetic of the computation */
#define BFM_PREC_FP64 0
#define BFM_PREC_FP32 1

/* storage type of the series Y (bfm_fit_monitor_typed) */
#define BFM_Y_F32 0  /* IEEE float32                                        */
#define BFM_Y_BF16 1 /* bfloat16: the high 16 bits of a float32, as uint16  */
#define BFM_Y_F16 2  /* IEEE binary16 (11 significant bits), as uint16      */

/* element type of the floating-point outputs */
#define BFM_OUT_F32 0
#define BFM_OUT_F64 1

/* per-pixel status */
#define BFM_ST_OK 0
#define BFM_ST_NONFINITE 1        /* NaN/Inf among the used observations     */
#define BFM_ST_INSUFFICIENT 2     /* n_v <= p, or window H < 1 or H > n_v,
                                     or nothing finite to fill (MASK_FILL)   */
#define BFM_ST_RANK_DEFICIENT 3   /* history design rank deficient           */
#define BFM_ST_DEGENERATE_SIGMA 4 /* sigma <= 1e-6 * max |y| over history    */
#define BFM_ST_NO_MONITOR 5       /* no used observation after the history   */

/*
 * Method parameters (Algorithm 1 "Require" list; Section 2.1).
 *   n_obs     N, series length, N > n_hist.
 *   n_hist    n, length of the stable history period, 1 <= n < N.
 *   order     k, number of harmonic terms (Eq. 1); p = 2 + 2k regressors,
 *             0 <= k <= 8.
 *   h_window  MOSUM bandwidth h as a count of observations (Eq. 3),
 *             1 <= h_window <= n; 0 means "use h_frac".
 *   freq      f, observations per year (Eq. 1), > 0.
 *   h_frac    bandwidth as a fraction of the history: H = floor(h_frac * n)
 *             (with missing values: floor(h_frac * n_v)); 0 < h_frac <= 1.
 *   lambda    critical value of the boundary (Eq. 4), > 0.
 *   mask_mode one of BFM_MASK_*.
 *   precision BFM_PREC_FP64, or BFM_PREC_FP32: the MOSUM of the
 *             period-blocked missing-value path (f in {12, 23, 24}, float32 or
 *             FP16 series) in FP32, as in the paper's own float MOSUM kernel:
 *             each residual is formed in FP64 and rounded to float, and the
 *             window sums, their extremes and the boundary test run in FP32;
 *             the fit (Gram matrix, Cholesky factor, coefficients) and sigma
 *             stay FP64.  Results agree with FP64 to about 1e-6 (relative);
 *             a break index may differ where the MOSUM is within about 1e-4
 *             (relative) of the boundary.  Every other path (complete series,
 *             BF16 storage, other f, observation times) computes in FP64
 *             under either setting: those paths are bound by reading the
 *             series, and on gfx950 FP32 instructions issue at the FP64 rate.
 *   times     host, NULL or N doubles, finite and strictly increasing: the
 *             time of each observation, used in place of the index t in the
 *             design rows of Eq. 2 (Section 4 does this with day numbers and
 *             f = 365 for an unevenly sampled scene).  The history, the window
 *             and the boundary's t/n stay counts of observations, and brk
 *             stays an observation index.  Read during the call (for a server
 *             request: until the request completes); the library keeps a copy
 *             of the operators built from it.  Parameter sets with times take
 *             the table-driven kernels (float32 series only).
 */
typedef struct {
    int32_t n_obs;
    int32_t n_hist;
    int32_t order;
    int32_t h_window;
    double freq;
    double h_frac;
    double lambda;
    int32_t mask_mode;
    int32_t precision;
    const double *times;
} bfm_params;

/*
 * Outputs, all caller-owned device pointers.  Only brk is required; any other
 * pointer may be NULL.  Floating-point outputs have element type out_dtype.
 *   brk     int32[P]: first monitoring index i (0 <= i < N-n, time n+1+i in
 *           the paper's 1-based time) whose |MO| exceeds the boundary
 *           (Algorithm 1, step 13), or -1.
 *   mag     [P]: the MOSUM value of largest magnitude over the monitoring
 *           period (hi = max MO, lo = min MO; mag = hi if hi >= -lo else lo).
 *   sigma   [P]: residual scale of the history fit (Algorithm 1, step 5).
 *   status  uint8[P]: BFM_ST_*.
 *   beta    [p * P]: coefficients in the basis of Eq. 2, coefficient-major
 *           (beta[j*P + i]) like beta_all of Eq. 8.
 *   resid   [N * P]: residuals y - yhat (Eq. 11), time-major, NaN where an
 *           observation is not used.
 *   mosum   [(N-n) * P]: MO of Eq. 3, time-major, NaN where not defined.
 */
typedef struct {
    int32_t *brk;
    void *mag;
    void *sigma;
    uint8_t *status;
    void *beta;
    void *resid;
    void *mosum;
    int32_t out_dtype;
} bfm_outputs;

typedef struct bfm_ctx bfm_ctx;

/* Library version (BFM_VERSION of the build). */
int bfm_version(void);

/* Text of the calling thread's last error ("" if none).  Owned by the library;
 * valid until the thread's next call into the library. */
const char *bfm_last_error(void);

/*
 * Validate parameters and layout without touching a device.
 * Returns BFM_SUCCESS, BFM_E_INVAL or BFM_E_LAYOUT (ld < P).
 */
int bfm_check_params(const bfm_params *prm, int64_t P, int64_t ld);

/*
 * Create a context on HIP device `device`.  The context owns device copies of
 * the shared operators (built once per parameter set; Section 3 builds the
 * shared matrix M once for all pixels) and releases them in bfm_destroy.  One
 * context may be used by one host thread at a time.
 * Errors: BFM_E_INVAL (out NULL), BFM_E_NODEVICE, BFM_E_UNSUPPORTED (not
 * gfx950), BFM_E_HIP.
 */
int bfm_create(bfm_ctx **out, int device);

/* Release a context and its device memory.  NULL is accepted. */
int bfm_destroy(bfm_ctx *ctx);

/*
 * BFAST Monitor over P pixels (Algorithm 1 for every pixel; Section 3 batched
 * form).
 *   Y      device, float32, time-major, Y[t*ld + i], t < N, i < P, ld >= P.
 *   valid  device, uint8, valid[t*ldv + i]; read only when mask_mode is
 *          BFM_MASK_EXPLICIT, else may be NULL; ldv >= P.
 *   out    host struct of device output pointers (see bfm_outputs).
 *   stream hipStream_t on which all work is enqueued; the call returns
 *          without waiting for it, except that the first call with a new
 *          parameter set builds the shared operators on the host and copies
 *          them to the device synchronously (tens of KB, once per set).
 * P == 0 is accepted and does nothing (Y and the output pointers may then be
 * NULL).
 * Errors: BFM_E_INVAL (NULL ctx/prm/Y/out/out->brk, bad parameters, bad
 * out_dtype), BFM_E_LAYOUT, BFM_E_NOMEM, BFM_E_HIP.
 */
int bfm_fit_monitor(bfm_ctx *ctx, const bfm_params *prm, const float *Y, int64_t P,
                    int64_t ld, const uint8_t *valid, int64_t ldv, const bfm_outputs *out,
                    void *stream);

/*
 * bfm_fit_monitor with the series stored as y_dtype (BFM_Y_F32, BFM_Y_BF16 or
 * BFM_Y_F16).  A 16-bit series halves the bytes streamed from HBM, the bound of
 * the path (Section 5 proposes lowering the precision of the data to cut the
 * volume that has to be moved).  Each observation is decoded exactly to
 * float32 and the arithmetic stays FP64, so the results are those of
 * bfm_fit_monitor on the decoded series; what the narrower storage costs is
 * the rounding of the data itself (BF16 keeps 8 significant bits, FP16 11).
 * ld and ldv count elements.  16-bit series are served by the period-blocked
 * kernels: f in {12, 23, 24} and order <= 4, and additionally on the plain path
 * a window f <= H <= 160 (its workgroup's window rings take H KB of the 160 KB
 * of LDS), a full-rank history design and ld * 2 * f < 2^31, on the
 * missing-value paths n_hist <= 8192 and ld * 4 * f < 2^31, and neither
 * observation times nor BFM_MASK_FILL; other parameter sets return
 * BFM_E_UNSUPPORTED.
 * Errors: those of bfm_fit_monitor, BFM_E_INVAL for an unknown y_dtype, and
 * BFM_E_UNSUPPORTED as above.
 */
int bfm_fit_monitor_typed(bfm_ctx *ctx, const bfm_params *prm, const void *Y, int32_t y_dtype,
                          int64_t P, int64_t ld, const uint8_t *valid, int64_t ldv,
                          const bfm_outputs *out, void *stream);

/*
 * Tile-shape tuning.  Plain path: for f in {12, 23, 24}, a float32 series and
 * no per-row exports (resid, mosum), each group of 64 pixels may get 1, 2, 4 or
 * 8 waves that stream consecutive shares of its rows (the history sums add up
 * over the shares; each share of the monitoring period rebuilds its MOSUM
 * window from the H rows before it): a long series over few pixels then
 * finishes sooner.  By default each group of 64 pixels has one wave (the
 * fastest for the usual tile shapes on MI355X, measured).
 * Missing-value path (BFM_MASK_NAN, BFM_MASK_EXPLICIT) with f in {12, 23, 24}
 * (the period-blocked kernel): the split covers the history; wave w of a group
 * streams the w-th share of the history's blocks of f rows, the waves hand
 * their partial sums on in wave order, and the last wave fits and monitors
 * (its window's observations taken from the earlier shares where its own share
 * holds fewer than H).  A split needs a block of f history rows per wave and
 * LDS for every wave's window ring plus the staging of the sums.  Untuned, the
 * missing-value path takes 4 waves per 64 pixels for a tile of at most one
 * wave per compute unit, 2 up to four waves per compute unit, else 1 (halved
 * while it does not fit).
 * bfm_autotune times every split that fits (on Y, with scratch outputs,
 * synchronising `stream`; on the missing-value path the BFM_MASK_NAN mode only,
 * as no validity mask is passed) and keeps the fastest for this tile shape (the
 * parameters, the mask mode, y_dtype and the power-of-two bucket of P/64) in
 * the context; bfm_tune_set pins a split for a shape (both mask modes).
 * Results differ between splits only by the rounding of the history sums.
 * times_us (nullable, 4 entries) receives the median time of splits 1, 2, 4, 8
 * (0 where not run).  Both return BFM_E_UNSUPPORTED where the parameters take
 * neither period-blocked kernel (and bfm_autotune for BFM_MASK_EXPLICIT), and
 * bfm_tune_set also where the split does not fit (LDS, or more waves than
 * history blocks); BFM_E_INVAL for a split other than 1, 2, 4 or 8.
 */
int bfm_autotune(bfm_ctx *ctx, const bfm_params *prm, const void *Y, int32_t y_dtype, int64_t P,
                 int64_t ld, void *stream, int32_t *split, double *times_us);
int bfm_tune_set(bfm_ctx *ctx, const bfm_params *prm, int32_t y_dtype, int64_t P, int32_t split);

/*
 * Critical value lambda of Eq. 4 by simulation.  Section 2.1 chooses lambda so
 * that, when nothing changes, the MOSUM crosses lambda sqrt(log+(t/n)) with
 * probability alpha, and finds it by simulation for given alpha, window h and
 * horizon N/n.  These entry points simulate the MOSUM of Eq. 3 under no change
 * at the resolution of the series (n_hist, n_obs and the window H of prm; its
 * other fields are validated but unused): with i.i.d. standard normal errors
 * z_1..z_N and the intercept-only model,
 *   M_k = (sum_{i=k-H+1..k} z_i - (H/n) sum_{i=1..n} z_i) / sqrt(n),
 *   S   = max_{k=n+1..N} |M_k| / sqrt(log+(k/n)),
 * and a path crosses lambda sqrt(log+) iff S > lambda.  This is the convention
 * of the method the paper cites for lambda: critical values of the process
 * W(t) - W(t-h) - h W(1) (the limit of M, and of the residual MOSUM of models
 * whose regressors have a stable second-moment matrix).  It is not an exact
 * level-alpha value for the season-trend model of Eq. 2, whose trend slope
 * error adds a term of order one to the limit.  The discrete sup over n steps
 * per unit of time is about 0.5826 sqrt(2/n) below the continuous one.  The normals of path q
 * come from Philox4x64-10 (Salmon et al., SC 2011) with key (seed, 0) and
 * counter (j, q, 0, 0) for steps 4j+1..4j+4, through the Box-Muller transform
 * of the uniforms ((w >> 11) + 1/2) 2^-53: results depend only on (seed, q),
 * not on how paths are split over calls.
 *
 * bfm_mosum_null_sup writes S of paths path0 .. path0+paths-1 to sup (device,
 * double[paths]); it allocates nothing.
 * bfm_critical_value returns in *lambda (host) the ceil((1 - alpha) paths)-th
 * smallest S over paths 0 .. paths-1 (so at most a share alpha of the paths
 * cross it), selected on the device.  It allocates paths * 8 + 1024 bytes of
 * device memory for the call and synchronises `stream` before returning.
 * Errors: BFM_E_INVAL (NULL ctx/prm/output, bad parameters, window outside
 * [1, n_hist], alpha outside (0, 1), paths < 1 or > 2^31), BFM_E_NOMEM,
 * BFM_E_HIP.
 */
int bfm_mosum_null_sup(bfm_ctx *ctx, const bfm_params *prm, uint64_t seed, int64_t path0,
                       int64_t paths, double *sup, void *stream);
int bfm_critical_value(bfm_ctx *ctx, const bfm_params *prm, double alpha, int64_t paths,
                       uint64_t seed, double *lambda, void *stream);

/*
 * bfm_critical_value for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, result and errors as bfm_critical_value (the same kernels; the
 * value equals its for the same seed and paths), but the simulated statistics
 * and the selection's counters live in a fixed device array of the library
 * (BFM_NOALLOC_MAX_PATHS * 8 + 1024 bytes, one per GPU, held from the first
 * bfm_create on that GPU until the process ends) instead of memory allocated
 * for the call: no hipMalloc, hipFree or other allocating call is made.
 * paths must be in [1, BFM_NOALLOC_MAX_PATHS] (BFM_E_INVAL otherwise).  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (from
 * several host threads or streams) race and must be serialised by the caller.
 * The counters are cleared by a kernel at the start of each selection pass;
 * the statistics of paths 0 .. paths-1 are written before they are read.
 * Synchronises `stream` before returning.
 */
#define BFM_NOALLOC_MAX_PATHS 4194304
int bfm_critical_value_noalloc(bfm_ctx *ctx, const bfm_params *prm, double alpha, int64_t paths,
                               uint64_t seed, double *lambda, void *stream);

/*
 * Serving.  A server runs requests of different sizes and parameters as they
 * arrive, several at a time: each admitted request runs on one of `slots` HIP
 * streams of the server's device (non-blocking, default priority), so the work
 * of requests that arrive while others are on the GPU overlaps with theirs.  A
 * request is admitted, in arrival order, when a stream is free, its outputs
 * fit in the server's device pool (pool_bytes, allocated once at creation: no
 * allocation happens per request) and, for a parameter set not yet cached, its
 * operator block fits in the operator budget next to the blocks that running
 * requests read (the admission is by HBM footprint: outputs plus operators).
 * The shared operators of each parameter set are built once and stay on the
 * device while the budget allows (Section 3 builds the shared matrix once for
 * all pixels); see bfm_operator_budget for their eviction.  Results are exactly those of bfm_fit_monitor_typed on
 * the same request.  Thread-safe: any host thread may submit, wait and release.
 */
typedef struct bfm_server bfm_server;

/* output selection of a request (brk is always produced) */
#define BFM_WANT_MAG 1u
#define BFM_WANT_SIGMA 2u
#define BFM_WANT_STATUS 4u
#define BFM_WANT_BETA 8u
#define BFM_WANT_RESID 16u
#define BFM_WANT_MOSUM 32u

/*
 * A request: the arguments of bfm_fit_monitor_typed without the outputs.  Y
 * (and valid) are caller-owned device memory, and prm.times (if not NULL)
 * caller-owned host memory, that must stay unchanged until the request
 * completes.  `outputs` selects the arrays the server allocates in its
 * pool, in element type out_dtype (BFM_OUT_F32 or BFM_OUT_F64).
 */
typedef struct {
    bfm_params prm;
    const void *Y;
    int32_t y_dtype;
    int64_t P;
    int64_t ld;
    const uint8_t *valid;
    int64_t ldv;
    uint32_t outputs;
    int32_t out_dtype;
} bfm_request;

/* Completion record of a request. */
typedef struct {
    int32_t rc;         /* BFM_SUCCESS, or the error code of the request's launch */
    bfm_outputs out;    /* server-owned device arrays (NULL where not selected),
                           valid until bfm_server_release */
    double queued_us;   /* host time from submit to admission */
    double latency_us;  /* host time from submit to observed completion */
    double device_us;   /* time between events around the launch on its stream */
} bfm_result;

/* Pool bytes a request's outputs occupy (each array 256-byte aligned).
 * Errors: BFM_E_INVAL (NULL arguments, unknown output bits or out_dtype). */
int bfm_request_bytes(const bfm_request *req, size_t *bytes);

/*
 * Create a server on HIP device `device` with `slots` streams (1..64) and a
 * device pool of pool_bytes.  Errors: BFM_E_INVAL, BFM_E_NODEVICE,
 * BFM_E_UNSUPPORTED (not gfx950), BFM_E_NOMEM, BFM_E_HIP.
 */
int bfm_server_create(bfm_server **out, int device, int slots, size_t pool_bytes);

/*
 * The server's operator budget (bfm_operator_budget on its context; default
 * 64 MiB), set before the first request.  Errors: BFM_E_INVAL (NULL server,
 * or requests were submitted already).
 */
int bfm_server_operator_budget(bfm_server *s, size_t bytes);

/*
 * Queue a request; returns at once with a ticket (> 0).  Parameters are
 * validated here: BFM_E_INVAL / BFM_E_LAYOUT as for bfm_fit_monitor_typed, and
 * BFM_E_NOMEM if the request's outputs exceed the whole pool or its operator
 * block the whole operator budget.  Errors found at
 * launch (e.g. BFM_E_UNSUPPORTED) are reported in the result.
 */
int bfm_server_submit(bfm_server *s, const bfm_request *req, uint64_t *ticket);

/*
 * Wait up to timeout_ms (< 0: without limit) for a request to complete and fill
 * *res.  Returns BFM_SUCCESS when it completed (its own outcome is res->rc),
 * BFM_E_INVAL for an unknown or released ticket, or BFM_E_HIP on timeout
 * (bfm_last_error says so).
 */
int bfm_server_wait(bfm_server *s, uint64_t ticket, int timeout_ms, bfm_result *res);

/* Return a completed request's outputs to the pool.  Errors: BFM_E_INVAL
 * (unknown ticket, or the request has not completed). */
int bfm_server_release(bfm_server *s, uint64_t ticket);

/*
 * Copy a completed request's outputs into caller device arrays (the non-NULL
 * pointers of dst among those the request selected; dst->out_dtype must match
 * the request's), on `stream`, wait for the copies and release the request.
 * Errors: BFM_E_INVAL (unknown or not completed ticket, failed request, dtype
 * mismatch), BFM_E_HIP.
 */
int bfm_server_take(bfm_server *s, uint64_t ticket, const bfm_outputs *dst, void *stream);

/* Counters of a server: requests queued, running and completed-unreleased,
 * pool bytes in use, the largest number of requests that ran at once, its
 * operator cache (blocks, bytes, evictions), and how many requests waited at
 * the head of the queue for room in the operator budget. */
typedef struct {
    int64_t queued;
    int64_t running;
    int64_t completed;
    int64_t pool_in_use;
    int64_t max_running;
    int64_t operator_entries;
    int64_t operator_bytes;
    int64_t operator_evictions;
    int64_t operator_waits;
} bfm_server_stats;
int bfm_server_get_stats(bfm_server *s, bfm_server_stats *st);

/* Wait for every admitted request to finish, then release the server (queued
 * requests are dropped, outputs freed).  NULL is accepted. */
int bfm_server_destroy(bfm_server *s);

/*
 * Host-only view of the shared operators the plain path streams against, for
 * inspection and tests (no device needed).  With p = 2 + 2k, M = N - n:
 *   q     host double[N * p]: row t is q_t = R^-T x~_t, where x~_t is the
 *         design row of Eq. 2 with the trend written as (t - (n+1)/2)/n and
 *         X~_n = Q R is the QR factorisation of the history rows; rows
 *         0..n-1 are orthonormal columns spanning the history design.
 *   w     host double[M * p]: w_t = sum of q_s over the MOSUM window of
 *         monitoring time t (Eq. 3 window, H rows ending at t).
 *   bnd   host double[M]: boundary of Eq. 4 at each monitoring time.
 *   bmap  host double[p * p], row-major: beta (basis of Eq. 2) =
 *         bmap * (Q' y_n), for the uncentred series.
 * Any pointer may be NULL.  Returns BFM_E_INVAL on bad parameters, or
 * BFM_E_UNSUPPORTED if the history design is rank deficient (then every pixel
 * of a plain call gets BFM_ST_RANK_DEFICIENT).
 */
int bfm_host_operators(const bfm_params *prm, double *q, double *w, double *bnd, double *bmap);

/*
 * Device memory the library holds for a call of bfm_fit_monitor(_typed) with
 * these parameters over P pixels, for admission by HBM footprint (no device
 * needed).  The library keeps no per-pixel workspace: a call streams Y once
 * and writes the caller's outputs, so the footprint is the operator block it
 * builds once per parameter set (Section 3 forms the shared matrix once for
 * all pixels) and caches in the context until bfm_destroy: the table rows of
 * the plain path (and those of the period-blocked kernel when f is 12, 23 or
 * 24), or the design and product tables of the missing-value path.  *out gets
 * that size in bytes, whatever P.  The caller's Y and outputs are not counted
 * (bfm_request_bytes gives a serving request's outputs).
 * Errors: BFM_E_INVAL (bad parameters, out NULL), BFM_E_LAYOUT.
 */
int bfm_workspace_bytes(const bfm_params *prm, int64_t P, size_t *out);

/*
 * Operator cache of a context.  The operator blocks of the parameter sets a
 * context has run (Section 3 forms the shared matrix once for all pixels) live
 * in one device arena of `budget` bytes (default 64 MiB), allocated at the
 * first call and carved first-fit.  When a new block does not fit, least
 * recently used blocks are evicted, idle ones first; a block is returned only
 * once the last launch that reads it has finished (a wait on that launch's
 * event alone: work on other streams goes on).  A block larger than the whole
 * budget gets a device allocation of its own.
 * bfm_operator_budget sets the budget; it must come before the first call on
 * the context (BFM_E_INVAL after).  bfm_cache_get_stats reports the cached
 * blocks, their bytes, the budget and the evictions so far.
 * Errors: BFM_E_INVAL (NULL arguments, budget set too late).
 */
typedef struct {
    int64_t entries;
    int64_t bytes;
    int64_t budget;
    int64_t evictions;
} bfm_cache_stats;
int bfm_operator_budget(bfm_ctx *ctx, size_t bytes);
int bfm_cache_get_stats(bfm_ctx *ctx, bfm_cache_stats *st);

#ifdef __cplusplus
}
#endif
#endif /* BFM_H */
