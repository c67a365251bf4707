// Internal declarations shared by the host runtime and the kernel launchers of
// libbfm.  Nothing here is part of the public ABI (include/bfm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bfm.h"

namespace bfm {

constexpr int kMaxOrder = 8;                 // k <= 8, p <= 18
constexpr int kMaxP = 2 + 2 * kMaxOrder;
constexpr double kSigmaRelTol = 1e-6;        // DEGENERATE_SIGMA threshold
constexpr double kRankTol = 1e-6;            // |R_jj| <= tol * sqrt(rows)
// The history fit's RSS = yy - ||b'||^2 (Gram identity) carries an absolute
// rounding error of about 1e2 ulp(yy).  A pixel whose RSS falls below
// kRefineRatio yy (its fit explains all but 1e-4 of yy: a series whose noise is
// small against its seasonal amplitude and offset) gets its history residuals
// explicitly instead: its wave streams the history again, forms r_t = d_t -
// x~_t' beta~, RSS = sum r_t^2, and one step of iterative refinement of beta~.
// Above the ratio the identity's error stays below 1e-10 of sigma.
constexpr double kRefineRatio = 1e-4;
constexpr int kPlainBlock = 64;              // threads per block (one wave), plain path
// Threads per workgroup of the period-blocked plain kernel: four waves over 256
// adjacent pixels, so that the row segments they read together are contiguous
// (1 KB per row instead of 256 B; measured 2% faster at 1024x1024, N = 400).
constexpr int kPeriodicBlock = 256;

// Shared operators of the plain path, built on the host in FP64 (Section 3:
// the pseudo-inverse M is formed once for all pixels; here its orthonormal
// equivalent).  See bfm_host_operators() in bfm.h for the meaning of each.
struct PlainOps {
    int N = 0, n = 0, p = 0, H = 0;
    int m_flat = 0;  // leading monitoring rows with t/n <= e (boundary = lambda)
    bool rank_ok = false;
    std::vector<double> q;     // N x p
    std::vector<double> w;     // (N-n) x p
    std::vector<double> bnd;   // N-n
    std::vector<double> bmap;  // p x p
    std::vector<double> R;     // p x p, row-major, upper: X~_n = Q R
};

// Operators of the period-blocked plain kernel, used when the number of
// observations per year f is one of the integers below: the harmonic regressors
// then repeat every f rows, so the history fit accumulates one sum per phase
// and the window sums of fitted values are periodic in t (plus a linear trend).
constexpr int kPeriods[] = {12, 23, 24};
constexpr int kPeriodicMaxOrder = 4;
struct PeriodicOps {
    int F = 0;                // period in rows
    std::vector<double> rt;   // p x p, row-major: R^-T (lower)
    std::vector<double> ri;   // p x p, row-major: R^-1 (upper)
    std::vector<double> hh;   // F x 2k: sin, cos of 2 pi j (t+1)/f at phase t mod F
    std::vector<double> wh;   // F x 2k: their sums over the window ending at phase t mod F
};
// Returns the period to use for these parameters (0: not applicable).
int periodic_period(const bfm_params& prm, const PlainOps& ops);
void build_periodic_ops(const bfm_params& prm, const PlainOps& ops, int F, PeriodicOps* out);

// Operators of the masked path (host FP64).  With x~_t the design row of
// Eq. 2 in the centred-trend basis (1, tau_t, sin, cos, ...), tau_t = (t -
// (n+1)/2)/n, the per-pixel Gram matrix sum_t w_t x~_t x~_t' is assembled from
// 2 + 6k masked sums of the functions in `g` (product-to-sum identities).
constexpr int kMaskedMaxOrder = 4;  // per-pixel Gram and Cholesky held in VGPRs
struct MaskedOps {
    int N = 0, n = 0, p = 0, ng = 0, Hmax = 0, cap = 0;
    double tc = 0, ts = 1;  // trend column tau = (t - tc) / ts
    std::vector<double> x;  // N x p: x~_t
    std::vector<double> g;  // n x ng: tau, tau^2, sin(m w t), cos(m w t) for m = 1..2k,
                            // tau sin(j w t), tau cos(j w t) for j = 1..k
    // Period-blocked masked kernel (F > 0): f is one of kPeriods, so the
    // regressors repeat every F rows and the Gram matrix follows from per-phase
    // observation counts.  ph is F x 4k: sin, cos of 2 pi m (t+1)/f for m = 1..2k
    // at phase t mod F (0-based t).
    int F = 0;
    std::vector<double> ph;
};
// Largest history length the period-blocked masked kernel takes (its per-phase
// integer counters are exact up to there, and a history row index fits the
// 16-bit field of its window ring).
constexpr int kMaskedPeriodicMaxHist = 8192;
// Waves per 64 pixels that may share the history rows of the period-blocked
// missing-value kernel (its history split: 1, 2, 4 or 8).
constexpr int kMaskedMaxSplit = 8;
bool build_masked_ops(const bfm_params& prm, MaskedOps* ops);

// Centre and scale of the trend column of the design (tau = (t - tc) / ts):
// (n+1)/2 and n for t = 1..N, else from the first and last history times.
void trend_frame(const bfm_params& prm, double* tc, double* ts);

// Window length H for a history of `count` used observations.
int window_length(const bfm_params& prm, int count);

// Build the plain-path operators.  Returns false if the parameters are invalid.
bool build_plain_ops(const bfm_params& prm, PlainOps* ops);

// Arguments of the plain kernel (by value; every pointer is device memory).
struct PlainArgs {
    const float* Y;
    int64_t ld;
    int64_t P;
    const double* q;     // N x p
    const double* w;     // M x p
    const double* bnd;   // M
    const double* bmap;  // p x p
    int N, n, H;
    int m_flat;          // leading monitoring rows where the boundary equals lambda
    double lambda;
    double sqrt_n;       // sqrt(n): MOSUM normaliser of Eq. 3
    double inv_dof;      // 1 / (n - p): Algorithm 1, step 5
    int fill;            // BFM_MASK_FILL: fill missing observations as they are read
    int32_t* brk;
    void* mag;
    void* sigma;
    uint8_t* status;
    void* beta;
    void* resid;
    void* mosum;
    int out_f64;
};

hipError_t launch_plain(const PlainArgs& a, int p, hipStream_t stream);
hipError_t launch_plain_fill(const PlainArgs& a, int p, hipStream_t stream);
hipError_t launch_plain_export(const PlainArgs& a, int p, hipStream_t stream);
hipError_t launch_plain_fill_export(const PlainArgs& a, int p, hipStream_t stream);

// Arguments of the period-blocked plain kernel.
struct PeriodicArgs {
    const void* Y;       // element type y_dtype (BFM_Y_*)
    int y_dtype;
    int split;           // waves per 64 pixels that share the rows: 1, 2, 4 or 8
    int fill;            // BFM_MASK_FILL (float32 series, split 1)
    int64_t ld;
    int64_t P;
    const double* tab;   // rt | ri | hh | wh | bnd
    int N, n, H, m_flat;
    double lambda, sqrt_n, inv_dof;
    int32_t* brk;
    void* mag;
    void* sigma;
    uint8_t* status;
    void* beta;
    void* resid;
    void* mosum;
    int out_f64;
};
hipError_t launch_periodic(const PeriodicArgs& a, int order, int F, hipStream_t stream);
// LDS bytes the time-split form needs (0 if the split is not supported).
size_t periodic_split_lds(int order, int F, int split, int H);
// The time-split form (float32 series, no per-row exports; a.split in {2, 4, 8}).
hipError_t launch_periodic_split(const PeriodicArgs& a, int order, int F, hipStream_t stream);
hipError_t launch_periodic_split2(const PeriodicArgs& a, int order, int F, hipStream_t stream);
hipError_t launch_periodic_split4(const PeriodicArgs& a, int order, int F, hipStream_t stream);
hipError_t launch_periodic_split8(const PeriodicArgs& a, int order, int F, hipStream_t stream);
hipError_t launch_periodic_bf16(const PeriodicArgs& a, int order, int F, hipStream_t stream);
hipError_t launch_periodic_f16(const PeriodicArgs& a, int order, int F, hipStream_t stream);
hipError_t launch_periodic_fill(const PeriodicArgs& a, int order, int F, hipStream_t stream);

// Arguments of the masked kernel (by value; every pointer is device memory).
struct MaskedArgs {
    const void* Y;         // element type y_dtype (BFM_Y_*; 16-bit types: period-blocked kernel only)
    int y_dtype;
    int64_t ld;
    const uint8_t* valid;  // EXPLICIT mode only
    int64_t ldv;
    int64_t P;
    const double* x;       // N x p
    const double* g;       // n x ng
    const double* ph;      // F x 4k (period-blocked kernel)
    int F;                 // 0: general kernel
    int m32;               // BFM_PREC_FP32: the period-blocked kernel's MOSUM in FP32
    int split;             // period-blocked kernel: waves per 64 pixels sharing the history (1, 2, 4, 8)
    int N, n, h_window, cap;
    double h_frac, lambda;
    double tc, ts;         // time centre and scale of the trend column: tau = (t - tc) / ts
    int32_t* brk;
    void* mag;
    void* sigma;
    uint8_t* status;
    void* beta;
    void* resid;
    void* mosum;
    int out_f64;
};

hipError_t launch_masked(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream);
hipError_t launch_masked_periodic(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream);
hipError_t launch_masked_periodic_bf16(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream);
hipError_t launch_masked_periodic_f16(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream);
hipError_t launch_masked_periodic_m32(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream);
hipError_t launch_masked_periodic_m32_f16(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream);
size_t masked_periodic_lds_bytes(int cap, int F, int split);
size_t masked_lds_bytes(int cap);

// Null-path MOSUM sup statistics for the simulated critical value (one lane per
// path; sup[i] for path path0 + i) and the device rank selection over them
// (rank 1-based among cnt positive doubles; counts: 256 uint32 of scratch).
hipError_t launch_mosum_null_sup(int n, int N, int H, uint64_t seed, int64_t path0, int64_t paths,
                                 double* sup, hipStream_t stream);
hipError_t select_rank(const double* v, int64_t cnt, int64_t rank, uint32_t* counts, double* out,
                       hipStream_t stream);
// The fixed scratch array of bfm_critical_value_noalloc (BFM_NOALLOC_MAX_PATHS
// doubles, then 256 uint32 counters): noalloc_scratch_init looks up its device
// address on `device` (which must be current) once and keeps it;
// noalloc_scratch returns the kept address (nullptr before the lookup).
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch(int device);

// Operator cache of a context, as the serving runtime sees it: an upper bound
// on the device bytes of a parameter set's operator block (256-byte aligned),
// whether that block is cached or would fit next to the blocks still read by
// unfinished launches, and the context's budget.
size_t operator_block_bound(const bfm_params& p);
bool operator_room(bfm_ctx* ctx, const bfm_params& p);
size_t operator_budget_of(bfm_ctx* ctx);

// Every pixel gets `st` (or NONFINITE if one of its used observations is not
// finite), brk = -1 and NaN floating outputs: used when the parameters make
// every pixel degenerate (history too short, rank-deficient shared design).
hipError_t launch_fill_status(const void* Y, int y_dtype, int64_t ld, int64_t P, int N, int n, int p,
                              uint8_t st, const bfm_outputs& out, int mask_mode,
                              const uint8_t* valid, int64_t ldv, hipStream_t stream);

}  // namespace bfm
