// Fused plain-path kernel of BFAST Monitor for gfx950 (FP64 arithmetic).
//
// One lane owns one pixel and streams its series once, time-major, so every
// wave-wide load reads 64 consecutive pixels of one time row (coalesced; the
// paper's kernel listing in Section 3 uses the same transposed access).  The
// steps of Algorithm 1 for that pixel run in registers, with the batched form
// of Section 3 (one shared operator for all pixels, Eq. 7-8):
//
//   history rows t < n   (Eq. 5-6, Algorithm 1 steps 2-5)
//       b' += q_t (y_t - c)      coordinates in the orthonormal history basis
//       yy += (y_t - c)^2        so that RSS = yy - ||b'||^2
//     c = y_0 centres the series; the intercept absorbs it exactly.
//     Where RSS < kRefineRatio yy (the identity cancels) the wave streams its
//     history again for explicit residuals and one refinement step.
//   monitoring rows t >= n (Eq. 3, Algorithm 1 steps 6-13)
//       S_t = S_{t-1} + y_t - y_{t-H}   window sum of the observations; the
//             value H rows back comes from a per-lane ring in LDS
//       num = S_t - w_t' b'             window sum of the residuals
//       |num| > b_t sigma sqrt(n)       boundary test of Eq. 4 (first hit)
//       hi/lo = max/min num             MOSUM value of largest magnitude
//
// Neither the predictions nor the MOSUM process are materialised: Y is read
// once and each pixel writes a break index and a magnitude.  With FILL, missing
// (non-finite) observations are filled forward (backward for a leading gap) as
// the rows are consumed (footnote of Section 3), and the filled series is
// monitored.
//
// This header holds the kernel template; plain_kernel.hip (as read),
// plain_kernel_fill.hip (with filling) and their _export variants (with
// per-row exports) instantiate it.
#pragma once

#include <climits>
#include <cmath>

#include "bfm_internal.hpp"
#include "device_common.hpp"

namespace bfm {
namespace {

using namespace dev;

#ifndef BFM_PLAIN_ROWS
#define BFM_PLAIN_ROWS 16
#endif
constexpr int kU = BFM_PLAIN_ROWS;  // rows per prefetch chunk

template <int NP, bool EXPORT, bool FILL>
__global__ __launch_bounds__(kPlainBlock) void plain_kernel(PlainArgs a)
{
    extern __shared__ float ring[];  // H rows x kPlainBlock lanes
    const int tid = threadIdx.x;
    const int64_t pix = (int64_t)blockIdx.x * kPlainBlock + tid;
    const bool active = pix < a.P;
    // Lanes past the end read the last pixel's column and store nothing.
    const uint32_t lane = (uint32_t)(active ? pix : a.P - 1);
    const uint32_t lane_bytes = lane * (uint32_t)sizeof(float);
    const int n = a.n, N = a.N, H = a.H;
    const int64_t ld = a.ld;
    const float* __restrict__ Y = a.Y;
    const ctab q = as_const(a.q);
    const ctab w = as_const(a.w);
    const ctab bnd = as_const(a.bnd);
    float* myring = ring + tid;

    // c centres the series (its first observation, or with FILL its first
    // finite one, which also fills a leading gap).
    const float c0 = FILL ? first_finite(Y, ld, lane, N) : load_obs(Y, lane_bytes);
    const double c = (double)c0;
    Filler fill{c0};
    auto obs = [&](float v) { return FILL ? fill(v) : v; };
    double bq[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) bq[j] = 0.0;
    double yy = 0.0, S = 0.0;
    float ymax = 0.0f;

    // History rows before the last window: fit accumulation only.
    const int tail0 = n - H;
    stream_rows<kU>(ObsCursor{Y + (int64_t)(0) * ld, ld, lane_bytes}, 0, tail0, [&](int t, float v) {
        v = obs(v);
        const double d = (double)v - c;
        yy = fma(d, d, yy);
        const ctab qt = q + t * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) bq[j] = fma(qt[j], d, bq[j]);
        ymax = fmaxf(ymax, fabsf(v));
    });
    // Last H history rows: also start the first window and fill the ring.
    int slot = tail0 % H;
    stream_rows<kU>(ObsCursor{Y + (int64_t)(tail0) * ld, ld, lane_bytes}, tail0, n, [&](int t, float v) {
        v = obs(v);
        const double d = (double)v - c;
        yy = fma(d, d, yy);
        S += d;
        const ctab qt = q + t * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) bq[j] = fma(qt[j], d, bq[j]);
        ymax = fmaxf(ymax, fabsf(v));
        myring[slot * kPlainBlock] = v;
        slot = (slot + 1 == H) ? 0 : slot + 1;
    });

    // Algorithm 1, step 5, via the Gram identity in the orthonormal basis.
    double rss = yy;
#pragma unroll
    for (int j = 0; j < NP; ++j) rss = fma(-bq[j], bq[j], rss);
    // High signal-to-noise: the identity cancels (see kRefineRatio).  The lanes
    // concerned get explicit history residuals r_t = d_t - q_t' b' from a second
    // pass over the history (wave-uniform), RSS = sum r_t^2 - ||Q' r||^2 and one
    // refinement step b' += Q' r (Q has orthonormal columns).
    const bool refine = rss < kRefineRatio * yy;
    if (__ballot(refine) != 0) {
        double db[NP], rr = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) db[j] = 0.0;
        Filler fill2{c0};
        stream_rows_lean<kU>(ObsCursor{Y, ld, lane_bytes}, 0, n, [&](int t, float v) {
            if (FILL) v = fill2(v);
            const ctab qt = q + t * NP;
            double r = (double)v - c;
#pragma unroll
            for (int j = 0; j < NP; ++j) r = fma(-qt[j], bq[j], r);
            rr = fma(r, r, rr);
#pragma unroll
            for (int j = 0; j < NP; ++j) db[j] = fma(qt[j], r, db[j]);
        });
        double dd = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            dd = fma(db[j], db[j], dd);
            bq[j] = refine ? bq[j] + db[j] : bq[j];
        }
        rss = refine ? rr - dd : rss;
    }
    const double sig = sqrt(fmax(rss, 0.0) * a.inv_dof);
    const double scale = sig * a.sqrt_n;
    const double qnan = __builtin_nan("");
    const bool hist_bad = !isfinite(yy);
    const bool degenerate = sig <= kSigmaRelTol * (double)ymax;
    // The fit's outputs are written now, so that the coefficients need not stay
    // live through the monitoring loop; a non-finite monitoring value found later
    // turns them into NaN.
    auto write_fit = [&](bool bad) {
        if (a.sigma) put_out(a.sigma, pix, bad ? qnan : sig, a.out_f64);
        if (a.beta) {
            for (int j = 0; j < NP; ++j) {
                double v = (j == 0) ? c : 0.0;
                for (int l = 0; l < NP; ++l) v = fma(a.bmap[j * NP + l], bq[l], v);
                put_out(a.beta, (int64_t)j * a.P + pix, bad ? qnan : v, a.out_f64);
            }
        }
    };
    if (active) write_fit(hist_bad);

    double hi = -INFINITY, lo = INFINITY;
    int brk = INT_MAX;  // rows ascend, so the first crossing is the smallest m
    // One monitoring row; vo = y_{t-H}, `thr` the boundary b_t scaled by sigma sqrt(n).
    auto monitor_row = [&](int t, float v, float vo, double thr) {
        S += (double)v - (double)vo;
        const int m = t - n;
        const ctab wt = w + m * NP;
        double num = S;
#pragma unroll
        for (int j = 0; j < NP; ++j) num = fma(-wt[j], bq[j], num);
        // Branch-free, so a whole chunk of rows stays one basic block and the
        // independent dot products of different rows can be interleaved.
        brk = fabs(num) > thr ? min(brk, m) : brk;
        hi = max_num(hi, num);
        lo = min_num(lo, num);
        if (EXPORT && a.mosum && active)
            put_out(a.mosum, (int64_t)m * a.P + lane, num / scale, a.out_f64);
    };
    // Eq. 4 is flat (b_t = lambda) while t/n <= e: one threshold for those rows.
    const int t_flat = n + a.m_flat;
    const double thr_flat = a.lambda * scale;
    auto thr_at = [&](int t, bool flat) { return flat ? thr_flat : bnd[t - n] * scale; };
    if (H >= kU) {
        // Every ring value a chunk needs was written before the chunk began, so
        // the chunk's reads are issued together ahead of its arithmetic.
        float vo[kU];
        int s0 = slot;
        auto pre = [&](int, int count) {
            s0 = slot;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                int s = s0 + u;
                s -= s >= H ? H : 0;
                if (u < count) vo[u] = myring[s * kPlainBlock];
            }
        };
        auto row = [&](int u, int t, float v, bool flat) {
            v = obs(v);
            int s = s0 + u;
            s -= s >= H ? H : 0;
            myring[s * kPlainBlock] = v;
            slot = s + 1 == H ? 0 : s + 1;
            monitor_row(t, v, vo[u], thr_at(t, flat));
        };
        stream_rows<kU>(ObsCursor{Y + (int64_t)n * ld, ld, lane_bytes}, n, t_flat,
                        [&](int u, int t, float v) { row(u, t, v, true); }, pre);
        stream_rows<kU>(ObsCursor{Y + (int64_t)t_flat * ld, ld, lane_bytes}, t_flat, N,
                        [&](int u, int t, float v) { row(u, t, v, false); }, pre);
    } else {
        auto row = [&](int t, float v, bool flat) {
            v = obs(v);
            const float vo1 = myring[slot * kPlainBlock];
            myring[slot * kPlainBlock] = v;
            slot = (slot + 1 == H) ? 0 : slot + 1;
            monitor_row(t, v, vo1, thr_at(t, flat));
        };
        stream_rows<kU>(ObsCursor{Y + (int64_t)n * ld, ld, lane_bytes}, n, t_flat,
                        [&](int t, float v) { row(t, v, true); });
        stream_rows<kU>(ObsCursor{Y + (int64_t)t_flat * ld, ld, lane_bytes}, t_flat, N,
                        [&](int t, float v) { row(t, v, false); });
    }

    const bool bad = hist_bad || !isfinite(S);
    // With FILL only a series without any finite value stays non-finite.
    const uint8_t st = bad ? (FILL ? BFM_ST_INSUFFICIENT : BFM_ST_NONFINITE)
                           : degenerate ? BFM_ST_DEGENERATE_SIGMA : BFM_ST_OK;
    if (!active) return;

    double mag = qnan;
    if (st == BFM_ST_OK) mag = (hi >= -lo ? hi : lo) / scale;
    if (st != BFM_ST_OK || brk == INT_MAX) brk = -1;
    a.brk[pix] = brk;
    if (a.mag) put_out(a.mag, pix, mag, a.out_f64);
    if (a.status) a.status[pix] = st;
    if (bad && !hist_bad) write_fit(true);
    if (EXPORT) {
        if (a.resid) {
            Filler rfill{c0};
            for (int t = 0; t < N; ++t) {
                double r = qnan;
                float v = Y[(int64_t)t * ld + pix];
                if (FILL) v = rfill(v);
                if (!bad) {
                    r = (double)v - c;
                    const ctab qt = q + t * NP;
                    for (int j = 0; j < NP; ++j) r = fma(-qt[j], bq[j], r);
                }
                put_out(a.resid, (int64_t)t * a.P + pix, r, a.out_f64);
            }
        }
        if (a.mosum && st != BFM_ST_OK)
            for (int m = 0; m < N - n; ++m) put_out(a.mosum, (int64_t)m * a.P + pix, qnan, a.out_f64);
    }
}

template <int NP, bool EXPORT, bool FILL>
hipError_t launch_np(const PlainArgs& a, hipStream_t stream)
{
    const dim3 grid((unsigned)((a.P + kPlainBlock - 1) / kPlainBlock));
    const size_t lds = (size_t)a.H * kPlainBlock * sizeof(float);
    hipLaunchKernelGGL((plain_kernel<NP, EXPORT, FILL>), grid, dim3(kPlainBlock), lds, stream, a);
    return hipGetLastError();
}

// The instantiations for p regressors; each (EXPORT, FILL) pair lives in a
// translation unit of its own (plain_kernel*.hip), so that they compile in
// parallel.
template <bool EXPORT, bool FILL>
hipError_t launch_plain_t(const PlainArgs& a, int p, hipStream_t stream)
{
    switch (p) {
    case 2: return launch_np<2, EXPORT, FILL>(a, stream);
    case 4: return launch_np<4, EXPORT, FILL>(a, stream);
    case 6: return launch_np<6, EXPORT, FILL>(a, stream);
    case 8: return launch_np<8, EXPORT, FILL>(a, stream);
    case 10: return launch_np<10, EXPORT, FILL>(a, stream);
    case 12: return launch_np<12, EXPORT, FILL>(a, stream);
    case 14: return launch_np<14, EXPORT, FILL>(a, stream);
    case 16: return launch_np<16, EXPORT, FILL>(a, stream);
    case 18: return launch_np<18, EXPORT, FILL>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace bfm
