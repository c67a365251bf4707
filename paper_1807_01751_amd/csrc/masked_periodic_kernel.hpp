// Period-blocked masked kernel of BFAST Monitor for gfx950 (FP64 arithmetic):
// pixels with missing observations when f is an integer number of rows F.
//
// Same reading of missing values as the general masked kernel: observed values
// in time order form the series, design rows keep their original time, and the
// window, the normaliser and the boundary use compacted counts (H = floor(h
// n_v), sqrt(n_v), u/n_v).  With f = F rows the harmonic regressors of Eq. 2
// repeat every F rows, so for row t = F b + r (phase r, block b) every entry of
// the per-pixel Gram matrix sum_t w_t x~_t x~_t' follows from two integers per
// phase, W_r (observed rows) and Q_r (sum of their block indices), and one per
// pixel, sum w_t b_t^2: one packed integer add per row replaces the 2 + 6k
// masked FP64 sums of the general kernel.  The right-hand side needs one FP64
// sum per phase, A_r = sum w_t (y_t - c), plus sum w_t b_t (y_t - c).
//
// The series may be stored as float32, BF16 or FP16 (template parameter T); the
// arithmetic is the same.  This header holds the kernel template;
// masked_periodic_kernel.hip (float32), masked_periodic_kernel_bf16.hip and
// masked_periodic_kernel_f16.hip instantiate it, and
// masked_periodic_kernel_m32.hip / masked_periodic_kernel_m32_f16.hip its FP32
// MOSUM form (BFM_PREC_FP32).
//
// One lane owns one pixel and streams its series once, time-major, in blocks
// of F rows aligned to multiples of F, so a row's phase is a compile-time
// register index:
//   history        W_r, Q_r, A_r, yy; (t, y_t) of each observed row goes to a
//                  per-lane LDS ring.
//   fit            Gram matrix from the phase sums (products of harmonics by
//                  product-to-sum identities), Cholesky, beta, RSS = yy - ||z||^2.
//   window start   the last H observed history values become residuals.
//   monitoring     r_t = y_t - (P_r + gamma b): one FP64 subtract per row, with
//                  P_r the fitted value at phase r in block 0 (constant, trend
//                  and harmonics) and gamma the trend step per block; the ring
//                  gives back the residual H observations earlier; boundary
//                  test of Eq. 4 at the compacted position.
#pragma once

#include <climits>
#include <cmath>
#include <type_traits>

#include "bfm_internal.hpp"
#include "device_common.hpp"
#include "masked_common.hpp"

// Every fused multiply-add below is written out: the template variants (with or
// without exports, NaN or explicit masks) then round identically.
#pragma clang fp contract(off)

namespace bfm {
namespace {

using namespace dev;

constexpr int kBlock = 64;           // pixels per workgroup (one wave, or `split` waves)
constexpr uint32_t kCountBits = 12;  // acc_r = W_r + (Q_r << 12)
constexpr uint32_t kCountMask = (1u << kCountBits) - 1;


// Boundary test of Eq. 4 past e for one lane: |S| > lambda scale sqrt(ln(u/n_v)),
// squared: S^2 > thr2 ln(u/n_v).  Called only for rows where some lane of the
// wave may be past e; cross_flat (|S| > lambda scale) is necessary for a
// crossing.  The hardware log2 in FP32 decides every case whose margin exceeds
// 1e-5 (its error is below 1e-6 of ln(u/n_v) >= 1); the rest take the FP64
// logarithm.
__device__ __noinline__ bool cross_past_e(bool cross_flat, double S, double thr2, int u, int ue, int nv,
                                          float l2nv)
{
    if (!cross_flat || u <= ue) return cross_flat;
    const double s2 = S * S;
    const double tl = thr2 * (double)((__log2f((float)u) - l2nv) * 0.69314718f);
    if (s2 > tl * (1.0 + 1e-5)) return true;
    if (!(s2 > tl * (1.0 - 1e-5))) return false;
    return s2 > thr2 * log((double)u / (double)nv);
}

// Ring slots of the blocked kernel for the general kernel's ring capacity (the
// longest window plus one): the longest window, at least one.
__host__ __device__ constexpr int ring_slots(int cap) { return cap > 2 ? cap - 1 : 1; }

// A residual in a 6-byte ring slot: the low 16 of its 52 mantissa bits are
// cleared (relative change below 2^-36) and the value stored is the value
// returned, the one the MOSUM adds.
__device__ __forceinline__ double ring_store(uint32_t* hi, uint16_t* mid, int slot, double r)
{
    const uint64_t b = (uint64_t)__double_as_longlong(r) & ~(uint64_t)0xffff;
    hi[slot * kBlock] = (uint32_t)(b >> 32);
    mid[slot * kBlock] = (uint16_t)(b >> 16);
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ double ring_value(uint32_t hi, uint16_t mid)
{
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | ((uint64_t)mid << 16)));
}

__device__ __forceinline__ bool observed(float v) { return isfinite(v); }
__device__ __forceinline__ bool observed(FlaggedObs o) { return o.ok != 0; }
__device__ __forceinline__ float missing(float) { return __builtin_nanf(""); }
__device__ __forceinline__ FlaggedObs missing(FlaggedObs o) { return {o.y, 0u}; }
__device__ __forceinline__ float value(float v) { return v; }
__device__ __forceinline__ float value(FlaggedObs o) { return o.y; }

// Streams rows [t0, t1) in blocks of F rows aligned to multiples of F, one
// block ahead of the arithmetic in two register buffers used in turn.  Every
// block runs the same unrolled code: a row of the block outside [t0, t1) reads
// the nearest row inside, is replaced by a missing value before the rows run,
// and is passed with in = false.  init(buf) sees the first block before any row
// of it runs; pre(tb) runs before the rows of block tb.
template <int F, typename At, typename Body, typename Pre, typename Init>
__device__ __forceinline__ void stream_blocks(At at, int t0, int t1, Body&& body, Pre&& pre, Init&& init)
{
    using V = typename decltype(at(0))::value_type;
    if (t0 >= t1) return;
    auto load = [&](V* buf, int tb) {
        const auto cur = at(tb);
        const int first = t0 - tb, last = t1 - 1 - tb;
#pragma unroll
        for (int u = 0; u < F; ++u) buf[u] = cur.load(u < first ? first : (u < last ? u : last));
    };
    auto run = [&](V* buf, int tb) {
        pre(tb);
        const int lo = t0 - tb > 0 ? t0 - tb : 0, hi = t1 - tb < F ? t1 - tb : F;
        const uint32_t in = ((1u << hi) - 1u) & ~((1u << lo) - 1u);  // rows of the block in range
        // In a partial block (wave-uniform branch, once per block) the rows
        // outside the range become missing, so that a row's observed() alone
        // decides whether it takes part: whole blocks test nothing per row.
        if (lo > 0 || hi < F) {
#pragma unroll
            for (int u = 0; u < F; ++u)
                if (((in >> u) & 1u) == 0) buf[u] = missing(buf[u]);
        }
#pragma unroll
        for (int u = 0; u < F; ++u) body(u, tb + u, buf[u], ((in >> u) & 1u) != 0);
    };
    // Whole blocks in a straight-line loop with the next block in flight (the
    // compiler keeps its loads outstanding: no branch between a block's loads
    // and the previous block's rows); a partial first block runs alone, and
    // the last blocks go through the general form below.
    auto load_full = [&](V* buf, int tb) {
        const auto cur = at(tb);
#pragma unroll
        for (int u = 0; u < F; ++u) buf[u] = cur.load(u);
    };
    auto run_full = [&](V* buf, int tb) {
        pre(tb);
#pragma unroll
        for (int u = 0; u < F; ++u) body(u, tb + u, buf[u], true);
    };
    V a[F], b[F];
    int tb = t0 - t0 % F;
    load(a, tb);
    init(static_cast<const V*>(a));
    if (tb < t0 || tb + F > t1) {
        run(a, tb);
        tb += F;
        if (tb >= t1) return;
        load(a, tb);
    }
    for (; tb + 3 * F <= t1; tb += 2 * F) {
        load_full(b, tb + F);
        run_full(a, tb);
        load_full(a, tb + 2 * F);
        run_full(b, tb + F);
    }
    // a holds the block at tb; at most two more blocks follow.
    if (tb + F < t1) load(b, tb + F);
    run(a, tb);
    tb += F;
    if (tb >= t1) return;
    if (tb + F < t1) load(a, tb + F);
    run(b, tb);
    tb += F;
    if (tb >= t1) return;
    run(a, tb);
}

// Rows tb, tb + 1, ... of the series from one buffer resource based at row tb:
// row u of the block is at byte offset u * ld * sizeof(T) (a scalar offset), the
// lane's pixel at lane * sizeof(T).  The host keeps F rows of offsets below 2^31.
template <typename T>
struct ObsBlock {
    using value_type = float;
    __amdgpu_buffer_rsrc_t y;
    uint32_t ldb, lane_bytes;
    __device__ __forceinline__ value_type load(int u) const
    {
        return load_at(static_cast<const T*>(nullptr), y, lane_bytes, (uint32_t)u * ldb);
    }
};

// The same with the caller's validity flags (one byte per pixel and row).
template <typename T>
struct FlaggedBlock {
    using value_type = FlaggedObs;
    __amdgpu_buffer_rsrc_t y, f;
    uint32_t ldb, ldv, lane;
    __device__ __forceinline__ value_type load(int u) const
    {
        return {load_at(static_cast<const T*>(nullptr), y, lane * (uint32_t)sizeof(T), (uint32_t)u * ldb),
                __builtin_amdgcn_raw_buffer_load_b8(f, (int)lane, (int)((uint32_t)u * ldv), kLoadNT)};
    }
};

template <bool EXPLICIT, typename T>
struct CursorOf {
    using type = ObsBlock<T>;
    __device__ static type at(const MaskedArgs& a, int t, uint32_t lane)
    {
        return type{row_rsrc(static_cast<const T*>(a.Y) + (int64_t)t * a.ld),
                    (uint32_t)a.ld * (uint32_t)sizeof(T), lane * (uint32_t)sizeof(T)};
    }
};
template <typename T>
struct CursorOf<true, T> {
    using type = FlaggedBlock<T>;
    __device__ static type at(const MaskedArgs& a, int t, uint32_t lane)
    {
        return type{row_rsrc(static_cast<const T*>(a.Y) + (int64_t)t * a.ld),
                    row_rsrc(a.valid + (int64_t)t * a.ldv), (uint32_t)a.ld * (uint32_t)sizeof(T),
                    (uint32_t)a.ldv, lane};
    }
};

// LDS is what limits residency (one ring slot per window position and lane),
// so the kernel may use up to 256 VGPRs without losing waves.
//
// History split (a.split = S > 1 waves per 64 pixels, for tiles with few
// pixels): wave w streams its share of the history blocks and keeps its own
// sums and ring.  The history sums add up over the shares (the per-pixel sum
// of squared block indices by parts with a cross term for the observations of
// the earlier shares), so the waves hand their partial sums on in wave order
// through LDS; the last wave then also takes the observations its window needs
// from the rings of the earlier shares, fits, and monitors alone.
//
// M32 (BFM_PREC_FP32): the MOSUM in FP32.  The fit, sigma and each residual are
// computed in FP64 as above; the residual is then rounded to float, kept in the
// ring's 32-bit word (no 16-bit word: one LDS write and one read per row), and
// the window sum, its extremes and the boundary test run in FP32 (the paper's
// own MOSUM kernel computes in float).
template <int K, int F, bool EXPORT, bool EXPLICIT, typename T, bool M32>
__global__ __launch_bounds__(kBlock * kMaskedMaxSplit) __attribute__((amdgpu_waves_per_eu(2))) void
masked_periodic_kernel(MaskedArgs a)
{
    using Acc = typename std::conditional<M32, float, double>::type;  // MOSUM arithmetic
    using Gk = Gram<K>;
    using Cur = CursorOf<EXPLICIT, T>;
    using V = typename Cur::type::value_type;
    constexpr int NP = Gk::NP, NG = Gk::NG, NL = Gk::NL;
    constexpr int NT = 4 * K;  // phase-table row: sin, cos of m w (t+1), m = 1..2k
    // Window ring, cap slots x kBlock lanes of 6 bytes: a 32-bit high word and a
    // 16-bit middle word.  History slots hold (y_t as float bits, t); monitoring
    // slots hold a residual kept to 36 mantissa bits (the low 16 bits cleared
    // before it enters the MOSUM, so it leaves the sum exactly as it entered).
    extern __shared__ uint32_t ring_hi[];
    const int tid = threadIdx.x & (kBlock - 1);
    const int NS = (int)(blockDim.x / kBlock);                              // waves per 64 pixels
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kBlock));  // this wave's share
    const int64_t pix = (int64_t)blockIdx.x * kBlock + tid;
    const bool active = pix < a.P;
    const uint32_t lane = (uint32_t)(active ? pix : a.P - 1);
    const int n = a.n, N = a.N;
    const int cap = ring_slots(a.cap);  // the longest window: rows are written only when observed
    const ctab ph = as_const(a.ph);
    // Rings of the S waves: high words, then the 16-bit middle words.
    uint32_t* const rhi = ring_hi + (w * cap) * kBlock + tid;
    uint16_t* const rmid0 = reinterpret_cast<uint16_t*>(ring_hi + NS * cap * kBlock) + tid;
    uint16_t* const rmid = rmid0 + (w * cap) * kBlock;
    // The history blocks of this wave's share (the host keeps S <= blocks).
    const int nblk = (n + F - 1) / F;
    const int b0 = nblk * w / NS, b1 = nblk * (w + 1) / NS;
    const int h0 = b0 * F, h1 = min(b1 * F, n);
    const double c0 = 0.5 * (double)(n - 1);  // tau_t = (t - c0) / n for 0-based t

    // ---- history rows: per-phase counts and sums ----
    uint32_t acc[F];
    double A[F];
#pragma unroll
    for (int r = 0; r < F; ++r) {
        acc[r] = 0u;
        A[r] = 0.0;
    }
    double yy = 0.0, Bd = 0.0;
    uint32_t cnt = 0u, zs = 0u, ymaxb = 0u;
    bool bad = false;
    int wp = 0;  // next ring slot
    uint32_t inc = 1u;
    double bd = 0.0;
    // Centring constant c: the first observed history value, found in the first
    // block as it arrives; only a wave with a lane that has nothing observed
    // there scans further blocks.
    float cf = 0.0f;
    double c = 0.0;
    auto first_observed = [&](const V* buf, int t0, bool have) {
        const int lim = n - 1 - t0;
        float first = 0.0f;
        bool any = false;
#pragma unroll
        for (int u = F - 1; u >= 0; --u) {
            const bool ok = u <= lim && observed(buf[u]);
            first = ok ? value(buf[u]) : first;
            any = any || ok;
        }
        cf = have ? cf : first;
        return have || any;
    };
    auto init = [&](const V* buf) {
        bool have;
        if (h0 == 0) {
            have = first_observed(buf, 0, false);
        } else {  // a later share: every wave finds the same first observation
            const typename Cur::type cc = Cur::at(a, 0, lane);
            const int lim = n - 1;
            V first[F];
#pragma unroll
            for (int u = 0; u < F; ++u) first[u] = cc.load(u < lim ? u : lim);
            have = first_observed(first, 0, false);
        }
        for (int t0 = F; t0 < n && !__all(have); t0 += F) {
            const typename Cur::type cc = Cur::at(a, t0, lane);
            const int lim = n - 1 - t0;
            V more[F];
#pragma unroll
            for (int u = 0; u < F; ++u) more[u] = cc.load(u < lim ? u : lim);
            have = first_observed(more, t0, have);
        }
        c = (double)cf;
    };
    stream_blocks<F>(
        [&](int t) { return Cur::at(a, t, lane); }, h0, h1,
        [&](int u, int t, V val, bool) {
            const bool ok = observed(val);  // rows outside the range arrive missing
            const float v = value(val);
            if (EXPLICIT) bad = bad || (ok && !isfinite(v));
            // Lanes whose row is missing sit this one out (execution mask, no selects).
            if (ok) {
                const double d = (double)v - c;
                A[u] += d;
                yy = fma(d, d, yy);
                Bd = fma(bd, d, Bd);
                acc[u] += inc;
                ++cnt;
                ymaxb = max(ymaxb, __float_as_uint(v) & 0x7fffffffu);
                rhi[wp * kBlock] = __float_as_uint(v);
                rmid[wp * kBlock] = (uint16_t)t;
                wp = wp + 1 == cap ? 0 : wp + 1;
            }
        },
        [&](int tb) {
            const uint32_t b = (uint32_t)(tb / F);
            // sum over observed rows of b^2 by parts: (B-1)^2 n_v - sum_b (2b-1) C_b,
            // C_b the count before block b.
            if (b > 0) zs += (2u * b - 1u) * cnt;
            inc = 1u + (b << kCountBits);
            bd = (double)b;
        },
        init);

    // ---- history split: partial sums handed on in wave order ----
    const uint32_t cnt_own = cnt;  // observations in this wave's share (its ring)
    if (NS > 1) {
        // Staging after the rings: per lane, A[F], yy, Bd (FP64), then acc[F],
        // cnt, zs, ymax, bad, then every wave's (count, next slot).
        double* const sd = reinterpret_cast<double*>(ring_hi + NS * cap * kBlock * 3 / 2) + tid;
        uint32_t* const su = reinterpret_cast<uint32_t*>(sd - tid + (F + 2) * kBlock) + tid;
        uint32_t* const meta = su + (F + 4) * kBlock;
        meta[(2 * w) * kBlock] = cnt_own;
        meta[(2 * w + 1) * kBlock] = (uint32_t)wp;
        // Sum of (2b - 1) over this share's blocks b >= 1: the weight of the
        // earlier shares' count in the sum of squared block indices by parts.
        const uint32_t bw0 = (uint32_t)(b0 > 0 ? b0 - 1 : 0), bw1 = (uint32_t)(b1 - 1);
        const uint32_t zs_weight = bw1 * bw1 - bw0 * bw0;
        auto take = [&]() {  // add the sums of the earlier shares
#pragma unroll
            for (int r = 0; r < F; ++r) {
                A[r] = sd[r * kBlock] + A[r];
                acc[r] += su[r * kBlock];
            }
            yy = sd[F * kBlock] + yy;
            Bd = sd[(F + 1) * kBlock] + Bd;
            const uint32_t cprev = su[F * kBlock];
            zs += su[(F + 1) * kBlock] + cprev * zs_weight;
            cnt += cprev;
            ymaxb = max(ymaxb, su[(F + 2) * kBlock]);
            bad = bad || su[(F + 3) * kBlock] != 0u;
        };
        for (int k = 0; k < NS - 1; ++k) {
            if (w == k) {
                if (k > 0) take();
#pragma unroll
                for (int r = 0; r < F; ++r) {
                    sd[r * kBlock] = A[r];
                    su[r * kBlock] = acc[r];
                }
                sd[F * kBlock] = yy;
                sd[(F + 1) * kBlock] = Bd;
                su[F * kBlock] = cnt;
                su[(F + 1) * kBlock] = zs;
                su[(F + 2) * kBlock] = ymaxb;
                su[(F + 3) * kBlock] = bad ? 1u : 0u;
            }
            __syncthreads();
        }
        if (w != NS - 1) return;  // the last wave fits and monitors
        take();
    }

    // ---- Gram matrix and right-hand side from the phase sums (Eq. 5-6) ----
    const int nv = (int)cnt;
    const uint32_t blast = (uint32_t)((n - 1) / F);
    const uint32_t zsum = blast * blast * cnt - zs;  // sum w_t b_t^2 (exact below 2^32)
    double gs[NG], bq[NP];
#pragma unroll
    for (int i = 0; i < NG; ++i) gs[i] = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) bq[j] = 0.0;
    double s_t = 0.0, s_tt = 0.0, s_rA = 0.0;
#pragma unroll
    for (int r = 0; r < F; ++r) {
        const double w = (double)(acc[r] & kCountMask);
        const double q = (double)(acc[r] >> kCountBits);
        const double rc = (double)r - c0;
        const double U = fma(rc, w, (double)F * q);  // sum over phase r of w (t - c0)
        s_t += U;
        s_tt = fma(rc * rc, w, fma(2.0 * F * rc, q, s_tt));
        bq[0] += A[r];
        s_rA = fma(rc, A[r], s_rA);
#pragma unroll
        for (int m = 1; m <= 2 * K; ++m) {
            gs[1 + m] = fma(w, ph[r * NT + 2 * (m - 1)], gs[1 + m]);
            gs[1 + 2 * K + m] = fma(w, ph[r * NT + 2 * (m - 1) + 1], gs[1 + 2 * K + m]);
        }
#pragma unroll
        for (int j = 1; j <= K; ++j) {
            const double sj = ph[r * NT + 2 * (j - 1)], cj = ph[r * NT + 2 * (j - 1) + 1];
            gs[1 + 4 * K + j] = fma(U, sj, gs[1 + 4 * K + j]);
            gs[1 + 5 * K + j] = fma(U, cj, gs[1 + 5 * K + j]);
            bq[2 * j] = fma(A[r], sj, bq[2 * j]);
            bq[2 * j + 1] = fma(A[r], cj, bq[2 * j + 1]);
        }
    }
    const double inv_n = 1.0 / (double)n;
    s_tt = fma((double)F * (double)F, (double)zsum, s_tt);
    gs[0] = s_t * inv_n;
    gs[1] = s_tt * (inv_n * inv_n);
#pragma unroll
    for (int j = 1; j <= K; ++j) {
        gs[1 + 4 * K + j] *= inv_n;
        gs[1 + 5 * K + j] *= inv_n;
    }
    bq[1] = fma((double)F, Bd, s_rA) * inv_n;

    // ---- fit on the observed history ----
    const int H = a.h_window > 0 ? a.h_window : (int)floor(a.h_frac * (double)nv);
    uint8_t st = BFM_ST_OK;
    if (bad)
        st = BFM_ST_NONFINITE;
    else if (nv <= NP || H < 1 || H > nv)
        st = BFM_ST_INSUFFICIENT;
    double L[NL];
    Gk::assemble(gs, (double)nv, L);
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
    // a second pass (wave-uniform), r_t = (y_t - c) - x~_t' beta~, RSS = sum r_t^2
    // - ||L^-1 X~' r||^2 and one refinement step beta~ += L^-T L^-1 X~' r.
    double rss = yy - zz;
    const bool refine = fitted && rss < kRefineRatio * yy;
    if (__ballot(refine) != 0) {
        // Design rows from the table of the general kernel (the same basis:
        // tau = (t - c0) / n, harmonics at 1-based time), rows streamed in
        // chunks of eight: a lean loop, so that the factor L can stay live.
        double dq[NP], rr = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) dq[j] = 0.0;
        const ctab x = as_const(a.x);
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
        const T* const Yt = static_cast<const T*>(a.Y);
        if (EXPLICIT)
            stream_rows_lean<8>(FlaggedCursorT<T>{Yt, a.valid, a.ld, a.ldv, lane}, 0, n,
                                [&](int t, FlaggedObs o) { row2(t, o.y, o.ok != 0); });
        else
            stream_rows_lean<8>(ObsCursorT<T>{Yt, a.ld, lane * (uint32_t)sizeof(T)}, 0, n,
                                [&](int t, float v) { row2(t, v, isfinite(v)); });
        rss = refine ? rr - Gk::refine(L, dq, beta, refine) : rss;
    }
    const double sig = sqrt(fmax(rss, 0.0) / (double)(nv - NP));
    const double scale = sig * sqrt((double)nv);
    if (st == BFM_ST_OK && sig <= kSigmaRelTol * (double)__uint_as_float(ymaxb))
        st = BFM_ST_DEGENERATE_SIGMA;
    const bool monitor = st == BFM_ST_OK;

    // Fitted value at row t = F b + r: P_r + gamma b (the centring constant included).
    double Pw[F];
#pragma unroll
    for (int r = 0; r < F; ++r) {
        double v = fma(beta[1], ((double)r - c0) * inv_n, beta[0] + c);
#pragma unroll
        for (int j = 1; j <= K; ++j) {
            v = fma(beta[2 * j], ph[r * NT + 2 * (j - 1)], v);
            v = fma(beta[2 * j + 1], ph[r * NT + 2 * (j - 1) + 1], v);
        }
        Pw[r] = v;
    }
    const double gamma = beta[1] * (double)F * inv_n;

    // ---- outputs of the fit, written before the monitoring loop ----
    const double qnan = __builtin_nan("");
    if (active && a.beta) {
        // beta~ is in the centred-trend basis of the centred series; map it to
        // the basis of Eq. 2: tau = (t - (n+1)/2)/n with t the 1-based time.
        const bool have_fit = fitted && !bad;
        const double tc = 0.5 * (double)(n + 1);
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            double v = beta[j];
            if (j == 0) v = beta[0] - (tc / (double)n) * beta[1] + c;
            if (j == 1) v = beta[1] / (double)n;
            put_out(a.beta, (int64_t)j * a.P + pix, have_fit ? v : qnan, a.out_f64);
        }
    }

    // ---- history split: the window's observations from earlier shares ----
    // A lane whose share holds fewer than H observations copies the ones before
    // them, oldest first, from the earlier shares' rings into the free slots
    // before its own entries, so that its window lies in its ring in time order.
    if (NS > 1) {
        const uint32_t* const meta = reinterpret_cast<const uint32_t*>(
            reinterpret_cast<const double*>(ring_hi + NS * cap * kBlock * 3 / 2) + (F + 2) * kBlock) +
            (F + 4) * kBlock + tid;
        auto cnt_of = [&](int v) { return (int)meta[(2 * v) * kBlock]; };
        auto wp_of = [&](int v) { return (int)meta[(2 * v + 1) * kBlock]; };
        const int want = monitor && (int)cnt_own < H ? H - (int)cnt_own : 0;
        int most = want;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) most = max(most, __shfl_xor(most, o));
        most = __builtin_amdgcn_readfirstlane(most);
        if (most > 0) {
            int sw = NS - 2, need = want;
            while (sw > 0 && cnt_of(sw) < need) {
                need -= cnt_of(sw);
                --sw;
            }
            int ss = wp_of(sw) - need;
            ss += ss < 0 ? cap : 0;
            int rem = need;
            int d = wp - H;
            d += d < 0 ? cap : 0;
            for (int i = 0; i < most; ++i) {
                if (i < want) {
                    const int src = (sw * cap + ss) * kBlock;
                    rhi[d * kBlock] = ring_hi[src + tid];
                    rmid[d * kBlock] = rmid0[src];
                    d = d + 1 == cap ? 0 : d + 1;
                    ss = ss + 1 == cap ? 0 : ss + 1;
                    if (--rem == 0 && i + 1 < want) {
                        do {
                            ++sw;
                        } while (cnt_of(sw) == 0);
                        rem = cnt_of(sw);
                        ss = wp_of(sw) - rem;
                        ss += ss < 0 ? cap : 0;
                    }
                }
            }
        }
    }

    // ---- the last H observed history values become residuals ----
    // Four slots per step, so that their phase-table gathers are in flight
    // together; the wave stops at its largest window.
    Acc S = 0;
    int hmax = monitor ? H : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) hmax = max(hmax, __shfl_xor(hmax, o));
    hmax = __builtin_amdgcn_readfirstlane(hmax);
    for (int i0 = 0; i0 < hmax; i0 += 4) {
        int slot[4], t[4];
        float y[4];
        double hr[4][2 * K + 1];
#pragma unroll
        for (int k = 0; k < 4; ++k) {  // slots past the lane's window read slot 0, unused
            slot[k] = wp - H + i0 + k;
            slot[k] += slot[k] < 0 ? cap : 0;
            slot[k] = monitor && i0 + k < H ? slot[k] : 0;
            y[k] = __uint_as_float(rhi[slot[k] * kBlock]);
            t[k] = rmid[slot[k] * kBlock];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double* row = a.ph + (t[k] % F) * NT;
#pragma unroll
            for (int j = 0; j < 2 * K; ++j) hr[k][j] = row[j];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (monitor && i0 + k < H) {
                double pr = fma(beta[1], ((double)t[k] - c0) * inv_n, beta[0] + c);
#pragma unroll
                for (int j = 1; j <= K; ++j) {
                    pr = fma(beta[2 * j], hr[k][2 * (j - 1)], pr);
                    pr = fma(beta[2 * j + 1], hr[k][2 * (j - 1) + 1], pr);
                }
                if constexpr (M32) {
                    const float rf = (float)((double)y[k] - pr);
                    rhi[slot[k] * kBlock] = __float_as_uint(rf);
                    S += rf;
                } else {
                    S += ring_store(rhi, rmid, slot[k], (double)y[k] - pr);
                }
            }
        }
    }

    // ---- monitoring period (Eq. 3 and Eq. 4 at compacted positions) ----
    int rp = wp - H;  // slot of the residual that leaves the window next
    rp += rp < 0 ? cap : 0;
    const double thr_flat = a.lambda * scale;
    const double thr2 = thr_flat * thr_flat;
    const float l2nv = __log2f((float)nv);
    // Largest compacted count m with m / n_v <= e: up to there log+ is 1.
    int ue = (int)floor(M_E * (double)nv);
    while (ue > 0 && (double)ue / (double)nv > M_E) --ue;
    while ((double)(ue + 1) / (double)nv <= M_E) ++ue;
    // Rows before t_split cannot take any lane of the wave past ue (one
    // observation per row at most): the boundary there is lambda.
    int room = monitor ? ue - nv : INT_MAX;  // lanes that do not monitor do not count
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) room = min(room, __shfl_xor(room, o));
    room = __builtin_amdgcn_readfirstlane(room);  // the same in every lane: keep it scalar
    const int t_split = room >= N - n ? N : n + (room > 0 ? room : 0);
    int u1 = nv;  // compacted (1-based) position of the latest observation
    Acc hi = -INFINITY, lo = INFINITY;
    const Acc thr_acc = (Acc)thr_flat;
    int brk = INT_MAX;
    double Gb = 0.0;
    const double rscale = 1.0 / scale;
    auto pre = [&](int tb) { Gb = gamma * (double)(tb / F); };
    // The residual leaving the window is read one observation ahead (after the
    // previous write, so the window still holds exactly the last H residuals):
    // its LDS latency overlaps the rest of the row.
    uint32_t old_hi = rhi[rp * kBlock];
    uint16_t old_mid = M32 ? 0 : rmid[rp * kBlock];
    stream_blocks<F>(
        [&](int t) { return Cur::at(a, t, lane); }, n, N,
        [&](int u, int t, V val, bool in) {
            const bool ok = observed(val);  // rows outside the range arrive missing
            const float v = value(val);
            if (EXPLICIT) bad = bad || (ok && !isfinite(v));
            if (ok) {  // lanes whose row is missing sit this one out
                if constexpr (M32) {
                    const float r = (float)((double)v - (Pw[u] + Gb));
                    rhi[wp * kBlock] = __float_as_uint(r);
                    S += r - __uint_as_float(old_hi);
                } else {
                    const double r = ring_store(rhi, rmid, wp, (double)v - (Pw[u] + Gb));
                    S += r - ring_value(old_hi, old_mid);
                }
                wp = wp + 1 == cap ? 0 : wp + 1;
                rp = rp + 1 == cap ? 0 : rp + 1;
                old_hi = rhi[rp * kBlock];
                if (!M32) old_mid = rmid[rp * kBlock];
                hi = max_num(hi, S);
                lo = min_num(lo, S);
                ++u1;
                bool cross = fabs(S) > thr_acc;
                if (t >= t_split)  // wave-uniform; not reached while every u/n_v stays below e
                    cross = cross_past_e(cross, (double)S, thr2, u1, ue, nv, l2nv);
                brk = cross ? min(brk, t - n) : brk;
            }
            if (EXPORT && a.mosum && active && in)
                put_out(a.mosum, (int64_t)(t - n) * a.P + lane, monitor && ok ? (double)S * rscale : qnan,
                        a.out_f64);
        },
        pre, [](const V*) {});

    if (bad) st = BFM_ST_NONFINITE;
    if (st == BFM_ST_OK && u1 == nv) st = BFM_ST_NO_MONITOR;
    if (!active) return;

    const bool have_fit = fitted && st != BFM_ST_NONFINITE;
    double mag = qnan;
    if (st == BFM_ST_OK) mag = (double)(hi >= -lo ? hi : lo) * rscale;
    if (st != BFM_ST_OK || brk == INT_MAX) brk = -1;
    a.brk[pix] = brk;
    if (a.mag) put_out(a.mag, pix, mag, a.out_f64);
    if (a.status) a.status[pix] = st;
    if (a.sigma) put_out(a.sigma, pix, have_fit ? sig : qnan, a.out_f64);
    if (EXPORT) {
        if (a.resid) {
            for (int tb = 0; tb < N; tb += F) {
                const double g = gamma * (double)(tb / F);
#pragma unroll
                for (int u = 0; u < F; ++u) {
                    const int t = tb + u;
                    if (t < N) {
                        const float v = to_float(static_cast<const T*>(a.Y)[(int64_t)t * a.ld + pix]);
                        const bool ok = EXPLICIT ? a.valid[(int64_t)t * a.ldv + pix] != 0 : isfinite(v);
                        const double r = have_fit && ok ? (double)v - (Pw[u] + g) : qnan;
                        put_out(a.resid, (int64_t)t * a.P + pix, r, a.out_f64);
                    }
                }
            }
        }
        if (a.mosum && st != BFM_ST_OK)
            for (int m = 0; m < N - n; ++m) put_out(a.mosum, (int64_t)m * a.P + pix, qnan, a.out_f64);
    }
}

template <int K, int F, bool EXPLICIT, typename T, bool M32>
hipError_t launch_kf(const MaskedArgs& a, hipStream_t stream)
{
    const dim3 grid((unsigned)((a.P + kBlock - 1) / kBlock));
    const int split = a.split > 0 ? a.split : 1;
    // The rings, and with a split the staging after them (host-checked sizes).
    const size_t lds = (size_t)split * ring_slots(a.cap) * kBlock * 6 +
                       (split > 1 ? (size_t)kBlock * (8 * (F + 2) + 4 * (F + 4) + 8 * split) : 0);
    if (a.n >= 65536) return hipErrorInvalidValue;  // history rows are kept as 16-bit indices
    if (split > kMaskedMaxSplit || split > (a.n + F - 1) / F) return hipErrorInvalidValue;  // a block per wave
    const dim3 block((unsigned)(kBlock * split));
    if (a.resid || a.mosum)
        hipLaunchKernelGGL((masked_periodic_kernel<K, F, true, EXPLICIT, T, M32>), grid, block, lds, stream,
                           a);
    else
        hipLaunchKernelGGL((masked_periodic_kernel<K, F, false, EXPLICIT, T, M32>), grid, block, lds, stream,
                           a);
    return hipGetLastError();
}

template <int K, bool EXPLICIT, typename T, bool M32>
hipError_t launch_k(const MaskedArgs& a, hipStream_t stream)
{
    switch (a.F) {
    case 12: return launch_kf<K, 12, EXPLICIT, T, M32>(a, stream);
    case 23: return launch_kf<K, 23, EXPLICIT, T, M32>(a, stream);
    case 24: return launch_kf<K, 24, EXPLICIT, T, M32>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

template <bool EXPLICIT, typename T, bool M32>
hipError_t launch_mode(const MaskedArgs& a, int order, hipStream_t stream)
{
    switch (order) {
    case 0: return launch_k<0, EXPLICIT, T, M32>(a, stream);
    case 1: return launch_k<1, EXPLICIT, T, M32>(a, stream);
    case 2: return launch_k<2, EXPLICIT, T, M32>(a, stream);
    case 3: return launch_k<3, EXPLICIT, T, M32>(a, stream);
    case 4: return launch_k<4, EXPLICIT, T, M32>(a, stream);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, bool M32 = false>
hipError_t launch_t(const MaskedArgs& a, int order, int mask_mode, hipStream_t stream)
{
    return mask_mode == BFM_MASK_EXPLICIT ? launch_mode<true, T, M32>(a, order, stream)
                                          : launch_mode<false, T, M32>(a, order, stream);
}

}  // namespace
}  // namespace bfm
