// Period-blocked plain-path kernel of BFAST Monitor for gfx950 (FP64
// arithmetic), used when the number of observations per year f is an integer
// F (12, 23, 24).  The harmonic regressors of Eq. 2 then repeat every F rows,
// which removes every per-row table read from the streaming loops:
//
//   history  d_t = y_t - c;  A[t mod F] += d_t;  Tr += (t+1) d_t;  yy += d_t^2.
//            Afterwards g = X~_n' d follows from the F phase sums (harmonics
//            at each phase from a small table) and Tr (trend), b' = R^-T g
//            (coordinates in the orthonormal basis of Section 3's shared
//            operator), RSS = yy - ||b'||^2, beta~ = R^-1 b'.  Where that
//            identity cancels (RSS < kRefineRatio yy) the wave streams its
//            history again for explicit residuals and one refinement step.
//   monitor  the window sum of fitted values (Eq. 3) is
//            Lc + gamma (t+1) + Pw[t mod F]: a linear trend part and a per-phase
//            part, both computed once per pixel.  S'_t = S'_{t-1} + y_t -
//            y_{t-H} - gamma (window sum of observations minus the trend part;
//            y_{t-H} from the per-lane LDS ring) and num_t = S'_t - Pw[t mod F]
//            is the window sum of residuals, tested against b_t sigma sqrt(n).
//
// Rows are processed in blocks aligned to multiples of F so that a row's phase
// is a compile-time register index.  The series may be stored as float32, BF16
// or FP16 (template parameter T); arithmetic is FP64 either way.  With FILL,
// missing (non-finite) observations are filled forward (backward for a leading
// gap) as the rows are consumed, and the filled series is monitored.
//
// This header holds the kernel template; periodic_kernel.hip (float32) and
// periodic_kernel_bf16.hip, periodic_kernel_f16.hip and periodic_split_*.hip
// instantiate it.
#pragma once

#include <climits>
#include <cmath>

#include "bfm_internal.hpp"
#include "device_common.hpp"

namespace bfm {
namespace {

using namespace dev;

// Residual sums over history rows [t0, t1) at the fitted coefficients beta~
// (centred-trend basis of the centred series, tau_t = (t + 1 - (n+1)/2) / n):
// r_t = (y_t - c) - x~_t' beta~, rr += r_t^2, dg += x~_t r_t.  Rows are
// streamed in blocks aligned to multiples of F like the first pass.
template <int K, int F, typename Cursor, typename Obs>
__device__ __forceinline__ void history_residual_sums(Cursor cur, int t0, int t1, int n, double c,
                                                      Obs&& obs, ctab hh, const double* beta,
                                                      double* dg, double& rr)
{
    constexpr int NH = 2 * K;
    const double tc = 0.5 * (double)(n + 1);
    const double inv_n = 1.0 / (double)n;
    stream_aligned<F>(
        cur, t0, t1,
        [&](int u, int t, float v) {
            v = obs(v);
            const double tau = ((double)(t + 1) - tc) * inv_n;
            double f = fma(beta[1], tau, beta[0]);
#pragma unroll
            for (int j = 0; j < NH; ++j) f = fma(hh[u * NH + j], beta[2 + j], f);
            const double r = ((double)v - c) - f;
            rr = fma(r, r, rr);
            dg[0] += r;
            dg[1] = fma(tau, r, dg[1]);
#pragma unroll
            for (int j = 0; j < NH; ++j) dg[2 + j] = fma(hh[u * NH + j], r, dg[2 + j]);
        },
        [](int, int, int) {});
}

// One step of iterative refinement from the residual sums of the history:
// beta~ += R^-1 R^-T dg, and RSS = rr - ||R^-T dg||^2, the residual sum of
// squares at the refined coefficients (the correction is orthogonal to the new
// residuals).  Only lanes with `take` change.
template <int NP>
__device__ __forceinline__ void refine_apply(ctab rt, ctab ri, const double* dg, double rr, bool take,
                                             double* beta, double& rss)
{
    double db[NP];
    double dd = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k <= i; ++k) s = fma(rt[i * NP + k], dg[k], s);
        db[i] = s;
        dd = fma(s, s, dd);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = i; k < NP; ++k) s = fma(ri[i * NP + k], db[k], s);
        beta[i] = take ? beta[i] + s : beta[i];
    }
    rss = take ? rr - dd : rss;
}

template <int K, int F, bool EXPORT, typename T, bool FILL>
#ifndef BFM_PERIODIC_OCC
// Three waves per SIMD: the LDS ring of a 50-row window allows twelve per CU.
#define BFM_PERIODIC_OCC __attribute__((amdgpu_waves_per_eu(3)))
#endif
__global__ __launch_bounds__(kPeriodicBlock) BFM_PERIODIC_OCC
void periodic_kernel(PeriodicArgs a)
{
    constexpr int NP = 2 + 2 * K;
    constexpr int NH = 2 * K;
    extern __shared__ float ring[];  // H rows x kPeriodicBlock lanes
    const int tid = threadIdx.x;
    const int64_t pix = (int64_t)blockIdx.x * kPeriodicBlock + tid;
    const bool active = pix < a.P;
    const uint32_t lane = (uint32_t)(active ? pix : a.P - 1);
    const uint32_t lane_bytes = lane * (uint32_t)sizeof(T);
    const int n = a.n, N = a.N, H = a.H;
    const int64_t ld = a.ld;
    const T* __restrict__ Y = static_cast<const T*>(a.Y);
    const ctab rt = as_const(a.tab);
    const ctab ri = rt + NP * NP;
    const ctab hh = ri + NP * NP;
    const ctab wh = hh + F * NH;
    const ctab bnd = wh + F * NH;
    float* const myring = ring + tid;

    // ---- history (Eq. 5-6) ----
    // c centres the series (its first observation, or with FILL its first
    // finite one, which also fills a leading gap).
    const float c0 = FILL ? first_finite(Y, ld, lane, N) : load_obs(Y, lane_bytes);
    const double c = (double)c0;
    Filler fill{c0};
    auto obs = [&](float v) { return FILL ? fill(v) : v; };
    double A[F];
#pragma unroll
    for (int u = 0; u < F; ++u) A[u] = 0.0;
    double yy = 0.0;
    // Trend sum Tr = sum_t (t+1) d_t, with t + 1 = F b + u + 1 for row u of block
    // b: Tr = F sum_b b (block sum) + sum_u (u+1) A[u]; Wb = sum_t b d_t needs one
    // FMA per row against the block index held in a register.
    double Wb = 0.0, bidx = 0.0;
    // max |y| over the history as an unsigned maximum of the magnitude bits
    // (their order is the order of the magnitudes; NaN pixels are flagged anyway).
    uint32_t ymax_bits = 0;
    auto hist = [&](int u, int t, float v) {
        const double d = (double)v - c;
        yy = fma(d, d, yy);
        A[u] += d;
        Wb = fma(bidx, d, Wb);
        ymax_bits = max(ymax_bits, __float_as_uint(v) & 0x7fffffffu);
        (void)t;
    };
    auto hist_pre = [&](int tb, int, int) { bidx = (double)(tb / F); };
    // Rows from a block boundary at or before n - H also go to the ring, so that
    // it holds the last H history rows when the history ends.
    const int B = ((n - H) / F) * F;
    stream_aligned<F>(BlockCursorT<T>(Y, ld, lane), 0, B,
                      [&](int u, int t, float v) { hist(u, t, obs(v)); }, hist_pre);
    int slot = B % H;  // ring slot of the next row: t mod H
    stream_aligned<F>(
        BlockCursorT<T>(Y + (int64_t)B * ld, ld, lane), B, n,
        [&](int u, int t, float v) {
            v = obs(v);
            hist(u, t, v);
            myring[slot * kPeriodicBlock] = v;
            slot = slot + 1 == H ? 0 : slot + 1;
        },
        hist_pre);

    // ---- fit: g = X~_n' d from the phase sums, b' = R^-T g ----
    double g[NP];
    double g0 = 0.0;
#pragma unroll
    for (int u = 0; u < F; ++u) g0 += A[u];
    double Tr = (double)F * Wb;
#pragma unroll
    for (int u = 0; u < F; ++u) Tr = fma((double)(u + 1), A[u], Tr);
    g[0] = g0;
    g[1] = (Tr - 0.5 * (double)(n + 1) * g0) / (double)n;
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < F; ++u) s = fma(hh[u * NH + j], A[u], s);
        g[2 + j] = s;
    }
    double bq[NP], beta[NP];
    double rss = yy;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k <= i; ++k) s = fma(rt[i * NP + k], g[k], s);
        bq[i] = s;
        rss = fma(-s, s, rss);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        double s = 0.0;
#pragma unroll
        for (int k = i; k < NP; ++k) s = fma(ri[i * NP + k], bq[k], s);
        beta[i] = s;
    }
    const double tc = 0.5 * (double)(n + 1);
    // High signal-to-noise: explicit history residuals and one refinement step
    // for the lanes whose RSS the Gram identity cannot resolve (wave-uniform).
    const bool refine = rss < kRefineRatio * yy;
    if (__ballot(refine) != 0) {
        double dg[NP], rr = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) dg[j] = 0.0;
        Filler fill2{c0};
        history_residual_sums<K, F>(BlockCursorT<T>(Y, ld, lane), 0, n, n, c,
                                    [&](float v) { return FILL ? fill2(v) : v; }, hh, beta, dg, rr);
        refine_apply<NP>(rt, ri, dg, rr, refine, beta, rss);
    }
    const double sig = sqrt(fmax(rss, 0.0) * a.inv_dof);
    const double scale = sig * a.sqrt_n;
    const double qnan = __builtin_nan("");
    const bool hist_bad = !isfinite(yy);
    const bool degenerate = sig <= kSigmaRelTol * (double)__uint_as_float(ymax_bits);
    // The fit's outputs are written now, so that the coefficients need not stay
    // live through the monitoring loop; a non-finite monitoring value found later
    // turns them into NaN.
    auto write_fit = [&](bool bad) {
        if (a.sigma) put_out(a.sigma, pix, bad ? qnan : sig, a.out_f64);
        if (a.beta) {
            // beta~ is in the centred-trend basis of the centred series; map it
            // to the basis of Eq. 2: tau = (t - (n+1)/2)/n.
            for (int j = 0; j < NP; ++j) {
                double v = beta[j];
                if (j == 0) v = beta[0] - (tc / (double)n) * beta[1] + c;
                if (j == 1) v = beta[1] / (double)n;
                put_out(a.beta, (int64_t)j * a.P + pix, bad ? qnan : v, a.out_f64);
            }
        }
    };
    if (active) write_fit(hist_bad);

    // ---- window sums of fitted values: Lc + gamma (t+1) + Pw[t mod F] ----
    double Pw[F];
#pragma unroll
    for (int u = 0; u < F; ++u) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NH; ++j) s = fma(wh[u * NH + j], beta[2 + j], s);
        Pw[u] = s;
    }
    const double Hd = (double)H;
    const double gamma = beta[1] * Hd / (double)n;
    const double Lc = Hd * beta[0] - beta[1] * Hd * (0.5 * (Hd - 1.0) + tc) / (double)n;

    // Window sum over the last H history rows (all ring slots), minus the trend
    // part at t = n - 1.
    double S = 0.0;
    for (int s = 0; s < H; ++s) S += (double)myring[s * kPeriodicBlock] - c;
    double Sp = S - Lc - gamma * (double)n;

    // ---- monitoring period (Eq. 3, Eq. 4) ----
    double hi = -INFINITY, lo = INFINITY;
    int brk = INT_MAX;  // rows ascend, so the first crossing is the smallest m
    float vo[F];
    int s0 = slot;
    // The window is at least F rows long, so a block's ring reads precede its
    // writes and can be issued together.
    auto pre = [&](int, int lo_, int hi_) {
        s0 = slot;
#pragma unroll
        for (int u = 0; u < F; ++u) {
            if (u >= lo_ && u < hi_) {
                int s = s0 + (u - lo_);
                s -= s >= H ? H : 0;
                vo[u] = myring[s * kPeriodicBlock];
            }
        }
        slot = s0 + (hi_ - lo_);
        slot -= slot >= H ? H : 0;
    };
    // Ring writes: row t goes to slot t mod H.  Within a block, the first row
    // handed over has slot s0 and the rows follow in order.
    int wslot = 0;
    auto pre_w = [&](int tb, int lo_, int hi_) {
        pre(tb, lo_, hi_);
        wslot = s0;
    };
    auto row = [&](int u, int t, float v, double thr) {
        v = obs(v);
        myring[wslot * kPeriodicBlock] = v;
        wslot = wslot + 1 == H ? 0 : wslot + 1;
        Sp += ((double)v - (double)vo[u]) - gamma;
        const double num = Sp - Pw[u];
        const int m = t - n;
        brk = fabs(num) > thr ? min(brk, m) : brk;
        hi = max_num(hi, num);
        lo = min_num(lo, num);
        if (EXPORT && a.mosum && active)
            put_out(a.mosum, (int64_t)m * a.P + lane, num / scale, a.out_f64);
    };
    // Eq. 4 is flat (b_t = lambda) while t/n <= e; blocks entirely in that part
    // use one threshold, the rest read b_t per row.
    const int t_flat = n + a.m_flat;
    const int tA = t_flat >= N ? N : (t_flat / F) * F > n ? (t_flat / F) * F : n;
    const double thr_flat = a.lambda * scale;
    stream_aligned<F>(BlockCursorT<T>(Y + (int64_t)n * ld, ld, lane), n, tA,
                      [&](int u, int t, float v) { row(u, t, v, thr_flat); }, pre_w);
    stream_aligned<F>(BlockCursorT<T>(Y + (int64_t)tA * ld, ld, lane), tA, N,
                      [&](int u, int t, float v) { row(u, t, v, bnd[t - n] * scale); }, pre_w);

    const bool bad = hist_bad || !isfinite(Sp);
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
                float v = to_float(Y[(int64_t)t * ld + pix]);
                if (FILL) v = rfill(v);
                if (!bad) {
                    const int ph = t % F;
                    r = (double)v - c - beta[0] -
                        beta[1] * ((double)(t + 1) - tc) / (double)n;
                    for (int j = 0; j < NH; ++j) r = fma(-hh[ph * NH + j], beta[2 + j], r);
                }
                put_out(a.resid, (int64_t)t * a.P + pix, r, a.out_f64);
            }
        }
        if (a.mosum && st != BFM_ST_OK)
            for (int m = 0; m < N - n; ++m) put_out(a.mosum, (int64_t)m * a.P + pix, qnan, a.out_f64);
    }
}

// Time-split form for tiles too small to fill the device: NS waves of one
// workgroup share 64 pixels and each streams a contiguous share of the history
// blocks and of the monitoring blocks, so a pixel's rows are worked on NS at a
// time.  The history sums (phase sums A, yy, Wb, max |y|) add up over the
// shares: every wave leaves its partial sums in LDS and wave 0 adds them in wave
// order, fits (the same arithmetic as periodic_kernel) and leaves the per-pixel
// quantities the monitoring needs in LDS.  Each wave rebuilds the window at the
// start of its monitoring share from the H rows before it (Eq. 3 needs only
// them), runs the same per-row recursion, and the first crossing, max and min
// are combined over the waves at the end.
//
// LDS (bytes): max(NS (F + 3) 512, (F + NP + 5) 512 + NS H 256,
// (F + NP + 5 + (NS + 1)(NP + 1)) 512).
template <int K, int F, int NS, bool EXPORT, typename T>
__global__ __launch_bounds__(kPlainBlock * NS) void periodic_split_kernel(PeriodicArgs a)
{
    constexpr int NP = 2 + 2 * K;
    constexpr int NH = 2 * K;
    constexpr int NB = F + NP + 5;  // broadcast doubles per lane: Pw, beta, gamma, Lc, scale, c, sig
    extern __shared__ double lds[];
    const int tid = threadIdx.x % kPlainBlock;
    const int w = threadIdx.x / kPlainBlock;  // wave index: its share of the rows
    const int64_t pix = (int64_t)blockIdx.x * kPlainBlock + tid;
    const bool active = pix < a.P;
    const uint32_t lane = (uint32_t)(active ? pix : a.P - 1);
    const uint32_t lane_bytes = lane * (uint32_t)sizeof(T);
    const int n = a.n, N = a.N, H = a.H;
    const int64_t ld = a.ld;
    const T* __restrict__ Y = static_cast<const T*>(a.Y);
    const ctab rt = as_const(a.tab);
    const ctab ri = rt + NP * NP;
    const ctab hh = ri + NP * NP;
    const ctab wh = hh + F * NH;
    const ctab bnd = wh + F * NH;
    double* const part = lds + tid;               // [NS][F + 3][64]
    double* const bc = lds + tid;                  // [NB][64] after the combine
    // refinement: beta and flag [NP + 1][64], then [NS][NP + 1][64] partial sums
    double* const rf = lds + NB * kPlainBlock + tid;
    float* const myring = reinterpret_cast<float*>(lds + NB * kPlainBlock) + w * H * kPlainBlock + tid;

    // ---- this wave's share of the history blocks ----
    const double c = (double)load_obs(Y, lane_bytes);
    const int nbh = (n + F - 1) / F;
    const int h0 = (nbh * w / NS) * F;
    const int h1 = min((nbh * (w + 1) / NS) * F, n);
    double A[F];
#pragma unroll
    for (int u = 0; u < F; ++u) A[u] = 0.0;
    double yy = 0.0, Wb = 0.0, bidx = 0.0;
    uint32_t ymax_bits = 0;
    if (h0 < h1)
        stream_aligned<F>(
            BlockCursorT<T>(Y + (int64_t)h0 * ld, ld, lane), h0, h1,
            [&](int u, int, float v) {
                const double d = (double)v - c;
                yy = fma(d, d, yy);
                A[u] += d;
                Wb = fma(bidx, d, Wb);
                ymax_bits = max(ymax_bits, __float_as_uint(v) & 0x7fffffffu);
            },
            [&](int tb, int, int) { bidx = (double)(tb / F); });
#pragma unroll
    for (int u = 0; u < F; ++u) part[((w * (F + 3)) + u) * kPlainBlock] = A[u];
    part[(w * (F + 3) + F) * kPlainBlock] = yy;
    part[(w * (F + 3) + F + 1) * kPlainBlock] = Wb;
    part[(w * (F + 3) + F + 2) * kPlainBlock] = __longlong_as_double((long long)ymax_bits);
    __syncthreads();

    const double tc = 0.5 * (double)(n + 1);
    const double qnan = __builtin_nan("");
    bool hist_bad = false, degenerate = false;
    double beta[NP];
    double rss = 0.0;
    if (w == 0) {
        // ---- sum of the shares (in wave order) and the fit ----
        for (int v = 1; v < NS; ++v) {
#pragma unroll
            for (int u = 0; u < F; ++u) A[u] += part[(v * (F + 3) + u) * kPlainBlock];
            yy += part[(v * (F + 3) + F) * kPlainBlock];
            Wb += part[(v * (F + 3) + F + 1) * kPlainBlock];
            ymax_bits = max(ymax_bits,
                            (uint32_t)__double_as_longlong(part[(v * (F + 3) + F + 2) * kPlainBlock]));
        }
        double g[NP];
        double g0 = 0.0;
#pragma unroll
        for (int u = 0; u < F; ++u) g0 += A[u];
        double Tr = (double)F * Wb;
#pragma unroll
        for (int u = 0; u < F; ++u) Tr = fma((double)(u + 1), A[u], Tr);
        g[0] = g0;
        g[1] = (Tr - 0.5 * (double)(n + 1) * g0) / (double)n;
#pragma unroll
        for (int j = 0; j < NH; ++j) {
            double sj = 0.0;
#pragma unroll
            for (int u = 0; u < F; ++u) sj = fma(hh[u * NH + j], A[u], sj);
            g[2 + j] = sj;
        }
        double bq[NP];
        rss = yy;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            double sv = 0.0;
#pragma unroll
            for (int k = 0; k <= i; ++k) sv = fma(rt[i * NP + k], g[k], sv);
            bq[i] = sv;
            rss = fma(-sv, sv, rss);
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            double sv = 0.0;
#pragma unroll
            for (int k = i; k < NP; ++k) sv = fma(ri[i * NP + k], bq[k], sv);
            beta[i] = sv;
        }
        // the coefficients and the refinement flag, for every wave (past the
        // broadcast rows, which wave 0 writes below while the others may still
        // read these)
#pragma unroll
        for (int j = 0; j < NP; ++j) rf[j * kPlainBlock] = beta[j];
        rf[NP * kPlainBlock] = rss < kRefineRatio * yy ? 1.0 : 0.0;
    }
    __syncthreads();
    // High signal-to-noise (the same 64 flags in every wave): each wave sums the
    // residuals of its history share, wave 0 adds the shares in wave order and
    // refines the lanes whose RSS the Gram identity cannot resolve.
    const bool refine = rf[NP * kPlainBlock] != 0.0;
    if (__ballot(refine) != 0) {
        double dg[NP], rr = 0.0, bt[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            dg[j] = 0.0;
            bt[j] = rf[j * kPlainBlock];
        }
        if (h0 < h1)
            history_residual_sums<K, F>(BlockCursorT<T>(Y + (int64_t)h0 * ld, ld, lane), h0, h1, n, c,
                                        [](float v) { return v; }, hh, bt, dg, rr);
        double* const rp = rf + (size_t)(1 + w) * (NP + 1) * kPlainBlock;
#pragma unroll
        for (int j = 0; j < NP; ++j) rp[j * kPlainBlock] = dg[j];
        rp[NP * kPlainBlock] = rr;
        __syncthreads();
        if (w == 0) {
            for (int v = 1; v < NS; ++v) {
                const double* q = rf + (size_t)(1 + v) * (NP + 1) * kPlainBlock;
#pragma unroll
                for (int j = 0; j < NP; ++j) dg[j] += q[j * kPlainBlock];
                rr += q[NP * kPlainBlock];
            }
            refine_apply<NP>(rt, ri, dg, rr, refine, beta, rss);
        }
        __syncthreads();  // the refinement area is free again
    }
    if (w == 0) {
        const double sig = sqrt(fmax(rss, 0.0) * a.inv_dof);
        hist_bad = !isfinite(yy);
        degenerate = sig <= kSigmaRelTol * (double)__uint_as_float(ymax_bits);
        const double Hd = (double)H;
        // per-pixel quantities of the monitoring, for every wave
#pragma unroll
        for (int u = 0; u < F; ++u) {
            double sv = 0.0;
#pragma unroll
            for (int j = 0; j < NH; ++j) sv = fma(wh[u * NH + j], beta[2 + j], sv);
            bc[u * kPlainBlock] = sv;
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) bc[(F + j) * kPlainBlock] = beta[j];
        bc[(F + NP) * kPlainBlock] = beta[1] * Hd / (double)n;  // gamma
        bc[(F + NP + 1) * kPlainBlock] = Hd * beta[0] - beta[1] * Hd * (0.5 * (Hd - 1.0) + tc) / (double)n;
        bc[(F + NP + 2) * kPlainBlock] = sig * a.sqrt_n;  // scale
        bc[(F + NP + 4) * kPlainBlock] = sig;
    }
    __syncthreads();
    double Pw[F];
#pragma unroll
    for (int u = 0; u < F; ++u) Pw[u] = bc[u * kPlainBlock];
#pragma unroll
    for (int j = 0; j < NP; ++j) beta[j] = bc[(F + j) * kPlainBlock];
    const double gamma = bc[(F + NP) * kPlainBlock];
    const double Lc = bc[(F + NP + 1) * kPlainBlock];
    const double scale = bc[(F + NP + 2) * kPlainBlock];
    const double sig = bc[(F + NP + 4) * kPlainBlock];
    if (w == 0 && active) {
        if (a.sigma) put_out(a.sigma, pix, hist_bad ? qnan : sig, a.out_f64);
        if (a.beta)
            for (int j = 0; j < NP; ++j) {
                double v = beta[j];
                if (j == 0) v = beta[0] - (tc / (double)n) * beta[1] + c;
                if (j == 1) v = beta[1] / (double)n;
                put_out(a.beta, (int64_t)j * a.P + pix, hist_bad ? qnan : v, a.out_f64);
            }
    }

    // ---- this wave's share of the monitoring blocks ----
    const int mb0 = n / F, nbm = (N - 1) / F - mb0 + 1;
    const int m0 = max(n, (mb0 + nbm * w / NS) * F);
    const int m1 = min(N, (mb0 + nbm * (w + 1) / NS) * F);
    double hi = -INFINITY, lo = INFINITY;
    int brk = INT_MAX;
    bool mon_bad = false;
    if (m0 < m1) {
        // the window that ends at row m0 - 1: its H rows go to this wave's ring
        // (row t in slot t mod H) and their sum starts the recursion
        double Sy = 0.0;
        int slot = (m0 - H) % H;
        stream_aligned<F>(
            BlockCursorT<T>(Y + (int64_t)(m0 - H) * ld, ld, lane), m0 - H, m0,
            [&](int, int, float v) {
                myring[slot * kPlainBlock] = v;
                slot = slot + 1 == H ? 0 : slot + 1;
                Sy += (double)v - c;
            },
            [](int, int, int) {});
        double Sp = Sy - Lc - gamma * (double)m0;
        float vo[F];
        int s0 = slot, wslot = 0;
        auto pre_w = [&](int, int lo_, int hi_) {
            s0 = slot;
#pragma unroll
            for (int u = 0; u < F; ++u) {
                if (u >= lo_ && u < hi_) {
                    int sl = s0 + (u - lo_);
                    sl -= sl >= H ? H : 0;
                    vo[u] = myring[sl * kPlainBlock];
                }
            }
            slot = s0 + (hi_ - lo_);
            slot -= slot >= H ? H : 0;
            wslot = s0;
        };
        auto row = [&](int u, int t, float v, double thr) {
            myring[wslot * kPlainBlock] = v;
            wslot = wslot + 1 == H ? 0 : wslot + 1;
            Sp += ((double)v - (double)vo[u]) - gamma;
            const double num = Sp - Pw[u];
            const int m = t - n;
            brk = fabs(num) > thr ? min(brk, m) : brk;
            hi = max_num(hi, num);
            lo = min_num(lo, num);
            if (EXPORT && a.mosum && active)
                put_out(a.mosum, (int64_t)m * a.P + lane, num / scale, a.out_f64);
        };
        const int t_flat = n + a.m_flat;
        const double thr_flat = a.lambda * scale;
        const int mA = min(max(t_flat, m0), m1);
        if (m0 < mA)
            stream_aligned<F>(BlockCursorT<T>(Y + (int64_t)m0 * ld, ld, lane), m0, mA,
                              [&](int u, int t, float v) { row(u, t, v, thr_flat); }, pre_w);
        if (mA < m1)
            stream_aligned<F>(BlockCursorT<T>(Y + (int64_t)mA * ld, ld, lane), mA, m1,
                              [&](int u, int t, float v) { row(u, t, v, bnd[t - n] * scale); }, pre_w);
        mon_bad = !isfinite(Sp);
    }

    // ---- combine the shares ----
    __syncthreads();  // every wave is past its reads of the broadcast area
    lds[(0 * NS + w) * kPlainBlock + tid] = hi;
    lds[(1 * NS + w) * kPlainBlock + tid] = lo;
    lds[(2 * NS + w) * kPlainBlock + tid] = __longlong_as_double((long long)brk | ((long long)mon_bad << 32));
    __syncthreads();
    if (w != 0) return;
    bool bad = hist_bad;
    for (int v = 0; v < NS; ++v) {
        hi = fmax(hi, lds[(0 * NS + v) * kPlainBlock + tid]);
        lo = fmin(lo, lds[(1 * NS + v) * kPlainBlock + tid]);
        const long long e = __double_as_longlong(lds[(2 * NS + v) * kPlainBlock + tid]);
        brk = min(brk, (int)(e & 0xffffffffll));
        bad = bad || ((e >> 32) & 1);
    }
    const uint8_t st = bad ? BFM_ST_NONFINITE : degenerate ? BFM_ST_DEGENERATE_SIGMA : BFM_ST_OK;
    if (!active) return;
    double mag = qnan;
    if (st == BFM_ST_OK) mag = (hi >= -lo ? hi : lo) / scale;
    if (st != BFM_ST_OK || brk == INT_MAX) brk = -1;
    a.brk[pix] = brk;
    if (a.mag) put_out(a.mag, pix, mag, a.out_f64);
    if (a.status) a.status[pix] = st;
    if (bad && !hist_bad) {
        if (a.sigma) put_out(a.sigma, pix, qnan, a.out_f64);
        if (a.beta)
            for (int j = 0; j < NP; ++j) put_out(a.beta, (int64_t)j * a.P + pix, qnan, a.out_f64);
    }
    if (EXPORT) {
        if (a.resid) {
            for (int t = 0; t < N; ++t) {
                double r = qnan;
                if (st != BFM_ST_NONFINITE) {
                    const int ph = t % F;
                    r = (double)to_float(Y[(int64_t)t * ld + pix]) - c - beta[0] -
                        beta[1] * ((double)(t + 1) - tc) / (double)n;
                    for (int j = 0; j < NH; ++j) r = fma(-hh[ph * NH + j], beta[2 + j], r);
                }
                put_out(a.resid, (int64_t)t * a.P + pix, r, a.out_f64);
            }
        }
        if (a.mosum && st != BFM_ST_OK)
            for (int m = 0; m < N - n; ++m) put_out(a.mosum, (int64_t)m * a.P + pix, qnan, a.out_f64);
    }
}

// LDS bytes of periodic_split_kernel for these sizes.
__host__ __device__ constexpr size_t split_lds_bytes(int F, int NP, int NS, int H)
{
    const size_t partials = (size_t)NS * (F + 3) * kPlainBlock * 8;
    const size_t refine = ((size_t)(F + NP + 5) + (size_t)(NS + 1) * (NP + 1)) * kPlainBlock * 8;
    const size_t monitor = (size_t)(F + NP + 5) * kPlainBlock * 8 + (size_t)NS * H * kPlainBlock * 4;
    const size_t combine = (size_t)3 * NS * kPlainBlock * 8;
    size_t m = partials > monitor ? partials : monitor;
    m = m > refine ? m : refine;
    return m > combine ? m : combine;
}

// The time-split launches (float32 series, no per-row exports): one
// translation unit per split factor instantiates them.
template <int NS>
hipError_t launch_split_ns(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    const dim3 grid((unsigned)((a.P + kPlainBlock - 1) / kPlainBlock));
    const size_t lds = split_lds_bytes(F, 2 + 2 * order, NS, a.H);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, grid, dim3(kPlainBlock * NS), lds, stream, a);
        return hipGetLastError();
    };
#define BFM_SPLIT_CASE(K, FF) \
    if (order == K && F == FF) return go(periodic_split_kernel<K, FF, NS, false, float>);
#define BFM_SPLIT_F(FF) BFM_SPLIT_CASE(0, FF) BFM_SPLIT_CASE(1, FF) BFM_SPLIT_CASE(2, FF) \
    BFM_SPLIT_CASE(3, FF) BFM_SPLIT_CASE(4, FF)
    BFM_SPLIT_F(12) BFM_SPLIT_F(23) BFM_SPLIT_F(24)
#undef BFM_SPLIT_F
#undef BFM_SPLIT_CASE
    return hipErrorInvalidValue;
}

template <int K, int F, typename T, bool FILL>
hipError_t launch_kf(const PeriodicArgs& a, hipStream_t stream)
{
    const dim3 grid((unsigned)((a.P + kPeriodicBlock - 1) / kPeriodicBlock));
    const size_t lds = (size_t)a.H * kPeriodicBlock * sizeof(float);
    if (a.resid || a.mosum)
        hipLaunchKernelGGL((periodic_kernel<K, F, true, T, FILL>), grid, dim3(kPeriodicBlock), lds, stream, a);
    else
        hipLaunchKernelGGL((periodic_kernel<K, F, false, T, FILL>), grid, dim3(kPeriodicBlock), lds, stream, a);
    return hipGetLastError();
}

template <int F, typename T, bool FILL>
hipError_t launch_f(const PeriodicArgs& a, int order, hipStream_t stream)
{
    switch (order) {
    case 0: return launch_kf<0, F, T, FILL>(a, stream);
    case 1: return launch_kf<1, F, T, FILL>(a, stream);
    case 2: return launch_kf<2, F, T, FILL>(a, stream);
    case 3: return launch_kf<3, F, T, FILL>(a, stream);
    case 4: return launch_kf<4, F, T, FILL>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, bool FILL = false>
hipError_t launch_t(const PeriodicArgs& a, int order, int F, hipStream_t stream)
{
    switch (F) {
    case 12: return launch_f<12, T, FILL>(a, order, stream);
    case 23: return launch_f<23, T, FILL>(a, order, stream);
    case 24: return launch_f<24, T, FILL>(a, order, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace bfm
