// Masked-path kernel of BFAST Monitor for gfx950 (FP64 arithmetic): pixels
// whose series have missing observations.
//
// Missing observations are dropped (the paper fills them in Section 3 and leaves
// variants with many missing values to future work, Section 5).  A pixel's
// series is its observed values in time order; design rows keep their original
// time; the history is the observed values with t <= n (n_v of them); the
// window, the normaliser and the boundary use compacted counts: H = floor(h n_v)
// observations, sqrt(n_v), and u/n_v for the compacted position u.
//
// One lane owns one pixel and streams its series once, time-major:
//   history rows   b += x~_t (y_t - c), yy += (y_t - c)^2 for observed rows, and
//                  the 2 + 6k masked sums from which the per-pixel Gram matrix
//                  sum_t x~_t x~_t' follows by product-to-sum identities
//                  (sin a sin b = (cos(a-b) - cos(a+b))/2, ...): 20 sums instead
//                  of 36 products at k = 3.  The observed history values and
//                  their times go to a per-lane LDS ring.
//   fit            Cholesky of the Gram matrix (FP64, pivot test for rank),
//                  z = L^-1 b, beta = L^-T z, RSS = yy - ||z||^2 (Eq. 5-6).
//   window start   the last H observed history values become residuals.
//   monitoring     for observed rows: r_t = (y_t - c) - x~_t' beta, the ring
//                  gives the residual H observations back, S += r_t - r_old,
//                  boundary test of Eq. 4 at the compacted position (Eq. 3).
#include <climits>
#include <cmath>

#include "bfm_internal.hpp"
#include "device_common.hpp"
#include "masked_common.hpp"

namespace bfm {
namespace {

using namespace dev;

constexpr int kMaskedBlock = 64;  // one wave per workgroup
#ifndef BFM_MASKED_ROWS
#define BFM_MASKED_ROWS 8
#endif
// Rows per prefetch chunk: each row's design and Gram-table entries are held
// in scalar registers while it is processed, so longer chunks spill them.
constexpr int kMU = BFM_MASKED_ROWS;

template <int K, bool EXPORT, bool EXPLICIT>
__global__ __launch_bounds__(kMaskedBlock) void masked_kernel(MaskedArgs a)
{
    using Gk = Gram<K>;
    constexpr int NP = Gk::NP, NG = Gk::NG, NL = Gk::NL;
    extern __shared__ double ring[];  // cap slots x kMaskedBlock lanes
    const int tid = threadIdx.x;
    const int64_t pix = (int64_t)blockIdx.x * kMaskedBlock + tid;
    const bool active = pix < a.P;
    const uint32_t lane = (uint32_t)(active ? pix : a.P - 1);
    const int n = a.n, N = a.N, cap = a.cap;
    const int64_t ld = a.ld;
    const ctab x = as_const(a.x);
    const ctab g = as_const(a.g);
    double* const myring = ring + tid;
    const float* const Y = static_cast<const float*>(a.Y);

    double c = 0.0, cnt = 0.0, yy = 0.0;
    bool have_c = false, bad = false;
    double gs[NG], bq[NP];
#pragma unroll
    for (int i = 0; i < NG; ++i) gs[i] = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) bq[j] = 0.0;
    float ymax = 0.0f;
    int wp = 0;  // next ring slot; the ring always has one slot more than the window

    auto hist_row = [&](int t, float v, bool used) {
        if (EXPLICIT) bad = bad || (used && !isfinite(v));
        c = (used && !have_c) ? (double)v : c;
        have_c = have_c || used;
        const double d = used ? (double)v - c : 0.0;
        const double w = used ? 1.0 : 0.0;
        cnt += w;
        yy = fma(d, d, yy);
        const ctab xr = x + t * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) bq[j] = fma(xr[j], d, bq[j]);
        const ctab gr = g + t * NG;
#pragma unroll
        for (int i = 0; i < NG; ++i) gs[i] = fma(w, gr[i], gs[i]);
        ymax = used ? fmaxf(ymax, fabsf(v)) : ymax;
        // (time, value) of the observation; the slot is claimed only if observed.
        myring[wp * kMaskedBlock] = __hiloint2double(t, __float_as_int(v));
        wp = used ? (wp + 1 == cap ? 0 : wp + 1) : wp;
    };
    if (EXPLICIT) {
        stream_rows<kMU>(FlaggedCursor{Y, a.valid, ld, a.ldv, lane}, 0, n,
                         [&](int t, FlaggedObs o) { hist_row(t, o.y, o.ok != 0); });
    } else {
        stream_rows<kMU>(ObsCursor{Y, ld, lane * 4u}, 0, n,
                         [&](int t, float v) { hist_row(t, v, isfinite(v)); });
    }

    // ---- fit on the observed history (Eq. 5-6) ----
    const int nv = (int)cnt;
    const int H = a.h_window > 0 ? a.h_window : (int)floor(a.h_frac * (double)nv);
    uint8_t st = BFM_ST_OK;
    if (bad)
        st = BFM_ST_NONFINITE;
    else if (nv <= NP || H < 1 || H > nv)
        st = BFM_ST_INSUFFICIENT;
    double L[NL];
    Gk::assemble(gs, cnt, L);
    const double tol = kRankTol * sqrt((double)nv);
    const bool full_rank = Gk::cholesky(L, tol * tol);
    if (st == BFM_ST_OK && !full_rank) st = BFM_ST_RANK_DEFICIENT;
    const bool fitted = st == BFM_ST_OK;  // beta and sigma are defined
    double z[NP], beta[NP];
    double zz = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        double s = bq[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s = fma(-L[tri(i, k)], z[k], s);
        z[i] = s / L[tri(i, i)];
        zz = fma(z[i], z[i], zz);
    }
#pragma unroll
    for (int i = NP - 1; i >= 0; --i) {
        double s = z[i];
#pragma unroll
        for (int k = i + 1; k < NP; ++k) s = fma(-L[tri(k, i)], beta[k], s);
        beta[i] = s / L[tri(i, i)];
    }
    // High signal-to-noise: RSS = yy - ||z||^2 cancels (see kRefineRatio).  The
    // lanes concerned get explicit residuals of their observed history rows from
    // a second pass (wave-uniform), RSS = sum r_t^2 - ||L^-1 X~' r||^2 and one
    // refinement step beta~ += L^-T L^-1 X~' r.
    double rss = yy - zz;
    const bool refine = fitted && rss < kRefineRatio * yy;
    if (__ballot(refine) != 0) {
        double dq[NP], rr = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) dq[j] = 0.0;
        auto row2 = [&](int t, float v, bool used) {
            if (used) {
                const ctab xr = x + t * NP;
                double r = (double)v - c;
#pragma unroll
                for (int j = 0; j < NP; ++j) r = fma(-xr[j], beta[j], r);
                rr = fma(r, r, rr);
#pragma unroll
                for (int j = 0; j < NP; ++j) dq[j] = fma(xr[j], r, dq[j]);
            }
        };
        if (EXPLICIT)
            stream_rows_lean<kMU>(FlaggedCursor{Y, a.valid, ld, a.ldv, lane}, 0, n,
                                  [&](int t, FlaggedObs o) { row2(t, o.y, o.ok != 0); });
        else
            stream_rows_lean<kMU>(ObsCursor{Y, ld, lane * 4u}, 0, n,
                                  [&](int t, float v) { row2(t, v, isfinite(v)); });
        rss = refine ? rr - Gk::refine(L, dq, beta, refine) : rss;
    }
    const double sig = sqrt(fmax(rss, 0.0) / (double)(nv - NP));
    const double scale = sig * sqrt((double)nv);
    if (st == BFM_ST_OK && sig <= kSigmaRelTol * (double)ymax) st = BFM_ST_DEGENERATE_SIGMA;

    // ---- the last H observed history values become residuals ----
    double S = 0.0;
    const bool monitor = st == BFM_ST_OK;
    const double* xg = a.x;  // per-lane gathers of design rows
    for (int i = 0; i < cap - 1; ++i) {
        int slot = wp - H + i;
        slot += slot < 0 ? cap : 0;
        if (monitor && i < H) {
            const double e = myring[slot * kMaskedBlock];
            const int t = __double2hiint(e);
            double r = (double)__int_as_float(__double2loint(e)) - c;
            const double* xr = xg + (int64_t)t * NP;
#pragma unroll
            for (int j = 0; j < NP; ++j) r = fma(-xr[j], beta[j], r);
            myring[slot * kMaskedBlock] = r;
            S += r;
        }
    }

    // ---- monitoring period (Eq. 3 and Eq. 4 at compacted positions) ----
    int rp = wp - H;  // slot of the residual that leaves the window next
    rp += rp < 0 ? cap : 0;
    const double thr_flat = a.lambda * scale;
    // Largest compacted count m with m / n_v <= e: up to there log+ is 1.
    int ue = (int)floor(M_E * (double)nv);
    while (ue > 0 && (double)ue / (double)nv > M_E) --ue;
    while ((double)(ue + 1) / (double)nv <= M_E) ++ue;
    int u1 = nv;  // compacted (1-based) position of the latest observation
    bool any_mon = false;
    double hi = -INFINITY, lo = INFINITY;
    int brk = INT_MAX;
    auto mon_row = [&](int t, float v, bool used) {
        if (EXPLICIT) bad = bad || (used && !isfinite(v));
        const ctab xr = x + t * NP;
        double r = (double)v - c;
#pragma unroll
        for (int j = 0; j < NP; ++j) r = fma(-xr[j], beta[j], r);
        const double old = myring[rp * kMaskedBlock];
        myring[wp * kMaskedBlock] = r;
        S = used ? S + (r - old) : S;
        wp = used ? (wp + 1 == cap ? 0 : wp + 1) : wp;
        rp = used ? (rp + 1 == cap ? 0 : rp + 1) : rp;
        u1 += used ? 1 : 0;
        any_mon = any_mon || used;
        double thr = thr_flat;
        if (u1 > ue) thr = a.lambda * sqrt(log((double)u1 / (double)nv)) * scale;
        brk = (used && fabs(S) > thr) ? min(brk, t - n) : brk;
        hi = used ? fmax(hi, S) : hi;
        lo = used ? fmin(lo, S) : lo;
        if (EXPORT && a.mosum && active)
            put_out(a.mosum, (int64_t)(t - n) * a.P + lane,
                    used && monitor ? S / scale : __builtin_nan(""), a.out_f64);
    };
    if (EXPLICIT) {
        stream_rows<kMU>(FlaggedCursor{Y + (int64_t)n * ld, a.valid + (int64_t)n * a.ldv, ld,
                                       a.ldv, lane},
                         n, N, [&](int t, FlaggedObs o) { mon_row(t, o.y, o.ok != 0); });
    } else {
        stream_rows<kMU>(ObsCursor{Y + (int64_t)n * ld, ld, lane * 4u}, n, N,
                         [&](int t, float v) { mon_row(t, v, isfinite(v)); });
    }
    if (bad) st = BFM_ST_NONFINITE;
    if (st == BFM_ST_OK && !any_mon) st = BFM_ST_NO_MONITOR;
    if (!active) return;

    const double qnan = __builtin_nan("");
    const bool have_fit = fitted && st != BFM_ST_NONFINITE;
    double mag = qnan;
    if (st == BFM_ST_OK) mag = (hi >= -lo ? hi : lo) / scale;
    if (st != BFM_ST_OK || brk == INT_MAX) brk = -1;
    a.brk[pix] = brk;
    if (a.mag) put_out(a.mag, pix, mag, a.out_f64);
    if (a.status) a.status[pix] = st;
    if (a.sigma) put_out(a.sigma, pix, have_fit ? sig : qnan, a.out_f64);
    if (a.beta) {
        // beta~ is in the centred-trend basis of the centred series; map it to
        // the basis of Eq. 2: tau = (t - tc)/ts (tc = (n+1)/2, ts = n for
        // t = 1..N; from the history's first and last times otherwise).
        for (int j = 0; j < NP; ++j) {
            double v = beta[j];
            if (j == 0) v = beta[0] - (a.tc / a.ts) * beta[1] + c;
            if (j == 1) v = beta[1] / a.ts;
            put_out(a.beta, (int64_t)j * a.P + pix, have_fit ? v : qnan, a.out_f64);
        }
    }
    if (EXPORT) {
        if (a.resid) {
            for (int t = 0; t < N; ++t) {
                const float v = Y[(int64_t)t * ld + pix];
                const bool used = EXPLICIT ? a.valid[(int64_t)t * a.ldv + pix] != 0 : isfinite(v);
                double r = qnan;
                if (have_fit && used) {
                    r = (double)v - c;
                    for (int j = 0; j < NP; ++j) r = fma(-xg[(int64_t)t * NP + j], beta[j], r);
                }
                put_out(a.resid, (int64_t)t * a.P + pix, r, a.out_f64);
            }
        }
        if (a.mosum && st != BFM_ST_OK)
            for (int m = 0; m < N - n; ++m) put_out(a.mosum, (int64_t)m * a.P + pix, qnan, a.out_f64);
    }
}

template <int K, bool EXPLICIT>
hipError_t launch_k(const MaskedArgs& a, hipStream_t stream)
{
    const dim3 grid((unsigned)((a.P + kMaskedBlock - 1) / kMaskedBlock));
    const size_t lds = (size_t)a.cap * kMaskedBlock * sizeof(double);
    if (a.resid || a.mosum)
        hipLaunchKernelGGL((masked_kernel<K, true, EXPLICIT>), grid, dim3(kMaskedBlock), lds, stream, a);
    else
        hipLaunchKernelGGL((masked_kernel<K, false, EXPLICIT>), grid, dim3(kMaskedBlock), lds, stream, a);
    return hipGetLastError();
}

template <bool EXPLICIT>
hipError_t launch_mode(const MaskedArgs& a, int order, hipStream_t stream)
{
    switch (order) {
    case 0: return launch_k<0, EXPLICIT>(a, stream);
    case 1: return launch_k<1, EXPLICIT>(a, stream);
    case 2: return launch_k<2, EXPLICIT>(a, stream);
    case 3: return launch_k<3, EXPLICIT>(a, stream);
    case 4: return launch_k<4, EXPLICIT>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t masked_lds_bytes(int cap) { return (size_t)cap * kMaskedBlock * sizeof(double); }

hipError_t launch_masked(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream)
{
    return mask_mode == BFM_MASK_EXPLICIT ? launch_mode<true>(a, order, stream)
                                          : launch_mode<false>(a, order, stream);
}

}  // namespace bfm
