// Host-side construction of the shared operators of the plain path (FP64).
//
// Section 3 of the paper observes that the pseudo-inverse of the history
// design, M = (X_n X_n')^-1 X_n (Eq. 7), is the same for every pixel, so the
// per-pixel fit collapses to one contraction with Y (Eq. 8).  This file builds
// the orthonormal form of that operator once per parameter set:
//
//   x~_t  design row of Eq. 2 with the trend written (t - tc) / ts, which
//         spans the same column space as (1, t) and keeps the factorisation
//         well conditioned (tc = (n+1)/2, ts = n for t = 1..N; with
//         observation times, the same frame from the history's first and last
//         times);
//   X~_n = Q R (Householder, rows t = 1..n).  For history rows q_t is row t
//         of the explicitly formed Q (orthonormal to rounding whatever the
//         conditioning); for monitoring rows q_t = R^-T x~_t, the same map
//         extended past the history.  Q' y_n = sum_t q_t y_t gives coordinates
//         b' with yhat_t = q_t' b' and RSS = ||y_n||^2 - ||b'||^2;
//   w_t   sum of q_s over the MOSUM window of monitoring time t, so the window
//         sum of fitted values in Eq. 3 is w_t' b';
//   bnd   the boundary of Eq. 4 at each monitoring time;
//   bmap  maps b' back to beta in the basis of Eq. 2.
#include <cmath>
#include <cstring>

#include "bfm_internal.hpp"

namespace bfm {

int window_length(const bfm_params& prm, int count)
{
    if (prm.h_window > 0) return prm.h_window;
    return (int)std::floor(prm.h_frac * (double)count);
}

// Time of the observation with 1-based index t: the index itself, or the
// given observation time (Section 4 uses day numbers for an unevenly sampled
// series).  Windows, the history and the boundary stay counts of observations.
static double time_at(const bfm_params& prm, int t)
{
    return prm.times ? prm.times[t - 1] : (double)t;
}

void trend_frame(const bfm_params& prm, double* tc, double* ts)
{
    const int n = prm.n_hist;
    if (!prm.times) {
        *tc = 0.5 * (double)(n + 1);
        *ts = (double)n;
        return;
    }
    const double t1 = prm.times[0], tn = prm.times[n - 1];
    *tc = 0.5 * (t1 + tn);
    *ts = n > 1 ? (tn - t1) * (double)n / (double)(n - 1) : 1.0;
}

// Design row of Eq. 2 in the centred-trend basis at time t.  The angle is
// reduced exactly (fmod is exact in IEEE arithmetic) before scaling by 2 pi/f.
static void design_row_centred(double t, double tc, double ts, int k, double f, double* x)
{
    x[0] = 1.0;
    x[1] = (t - tc) / ts;
    for (int j = 1; j <= k; ++j) {
        double ang = (2.0 * M_PI / f) * std::fmod((double)j * t, f);
        x[2 * j] = std::sin(ang);
        x[2 * j + 1] = std::cos(ang);
    }
}

static double log_plus(double x) { return x <= M_E ? 1.0 : std::log(x); }

bool build_plain_ops(const bfm_params& prm, PlainOps* ops)
{
    const int N = prm.n_obs, n = prm.n_hist, k = prm.order, p = 2 + 2 * k;
    const int M = N - n;
    const int H = window_length(prm, n);
    ops->N = N;
    ops->n = n;
    ops->p = p;
    ops->H = H;
    ops->rank_ok = false;
    ops->q.assign((size_t)N * p, 0.0);
    ops->w.assign((size_t)M * p, 0.0);
    ops->bnd.assign(M, 0.0);
    ops->bmap.assign((size_t)p * p, 0.0);
    ops->R.assign((size_t)p * p, 0.0);
    for (int m = 0; m < M; ++m)
        ops->bnd[m] = prm.lambda * std::sqrt(log_plus((double)(n + 1 + m) / (double)n));
    // log+ is exactly 1 up to t/n = e, and t/n increases with m.
    while (ops->m_flat < M && (double)(n + 1 + ops->m_flat) / (double)n <= M_E) ++ops->m_flat;
    if (n <= p) return true;  // every pixel INSUFFICIENT; no factorisation
    double tc, ts;
    trend_frame(prm, &tc, &ts);

    // Householder QR of X~_n (n x p, column-major copy).
    std::vector<double> A((size_t)n * p), x(p);
    for (int t = 1; t <= n; ++t) {
        design_row_centred(time_at(prm, t), tc, ts, k, prm.freq, x.data());
        for (int j = 0; j < p; ++j) A[(size_t)j * n + (t - 1)] = x[j];
    }
    std::vector<double> R((size_t)p * p, 0.0);
    const double tol = kRankTol * std::sqrt((double)n);
    bool ok = true;
    for (int j = 0; j < p && ok; ++j) {
        double* a = &A[(size_t)j * n];
        double nrm = 0.0;
        for (int i = j; i < n; ++i) nrm += a[i] * a[i];
        nrm = std::sqrt(nrm);
        if (nrm <= tol) {
            ok = false;
            break;
        }
        double rjj = a[j] > 0 ? -nrm : nrm;
        a[j] -= rjj;
        double vv = 0.0;
        for (int i = j; i < n; ++i) vv += a[i] * a[i];
        for (int c = j + 1; c < p; ++c) {
            double* b = &A[(size_t)c * n];
            double d = 0.0;
            for (int i = j; i < n; ++i) d += a[i] * b[i];
            d = 2.0 * d / vv;
            for (int i = j; i < n; ++i) b[i] -= d * a[i];
            R[(size_t)j * p + c] = b[j];
        }
        R[(size_t)j * p + j] = rjj;
    }
    if (!ok) return true;  // rank deficient: every pixel RANK_DEFICIENT
    ops->rank_ok = true;
    ops->R = R;

    // History rows: Q = H_0 H_1 ... H_{p-1} [I_p; 0], reflectors stored in A
    // below the diagonal (v_j = A[j.., j], H_j = I - 2 v v' / v'v).
    for (int c = 0; c < p; ++c) {
        std::vector<double> e(n, 0.0);
        e[c] = 1.0;
        for (int j = p - 1; j >= 0; --j) {
            const double* a = &A[(size_t)j * n];
            double vv = 0.0, d = 0.0;
            for (int i = j; i < n; ++i) {
                vv += a[i] * a[i];
                d += a[i] * e[i];
            }
            d = 2.0 * d / vv;
            for (int i = j; i < n; ++i) e[i] -= d * a[i];
        }
        for (int t = 0; t < n; ++t) ops->q[(size_t)t * p + c] = e[t];
    }
    // Monitoring rows: q_t = R^-T x~_t (forward substitution with R').
    for (int t = n + 1; t <= N; ++t) {
        design_row_centred(time_at(prm, t), tc, ts, k, prm.freq, x.data());
        double* qt = &ops->q[(size_t)(t - 1) * p];
        for (int j = 0; j < p; ++j) {
            double s = x[j];
            for (int c = 0; c < j; ++c) s -= R[(size_t)c * p + j] * qt[c];
            qt[j] = s / R[(size_t)j * p + j];
        }
    }
    // w_t: window of Eq. 3 ending at monitoring time t (0-based t = n + m).
    for (int m = 0; m < M; ++m) {
        int t = n + m;
        double* wt = &ops->w[(size_t)m * p];
        for (int s = t - H + 1; s <= t; ++s)
            for (int j = 0; j < p; ++j) wt[j] += ops->q[(size_t)s * p + j];
    }
    // bmap = T' R^-1, where x~ = T x: beta~ = R^-1 b', beta = T' beta~.
    std::vector<double> Ri((size_t)p * p, 0.0);
    for (int c = 0; c < p; ++c) {  // column c of R^-1 solves R z = e_c
        for (int j = p - 1; j >= 0; --j) {
            double s = (j == c) ? 1.0 : 0.0;
            for (int l = j + 1; l < p; ++l) s -= R[(size_t)j * p + l] * Ri[(size_t)l * p + c];
            Ri[(size_t)j * p + c] = s / R[(size_t)j * p + j];
        }
    }
    for (int c = 0; c < p; ++c) {
        for (int j = 0; j < p; ++j) ops->bmap[(size_t)j * p + c] = Ri[(size_t)j * p + c];
        ops->bmap[0 * p + c] = Ri[0 * p + c] - (tc / ts) * Ri[1 * p + c];
        ops->bmap[1 * p + c] = Ri[1 * p + c] / ts;
    }
    return true;
}

int periodic_period(const bfm_params& prm, const PlainOps& ops)
{
    if (prm.times || !ops.rank_ok || ops.n <= ops.p || prm.order > kPeriodicMaxOrder) return 0;
    for (int F : kPeriods)
        if (prm.freq == (double)F && ops.H >= F) return F;
    return 0;
}

void build_periodic_ops(const bfm_params& prm, const PlainOps& ops, int F, PeriodicOps* out)
{
    const int p = ops.p, k = prm.order, n = ops.n, H = ops.H;
    out->F = F;
    out->rt.assign((size_t)p * p, 0.0);
    out->ri.assign((size_t)p * p, 0.0);
    // R^-1 column by column (R z = e_c); R^-T is its transpose.
    for (int c = 0; c < p; ++c) {
        for (int j = p - 1; j >= 0; --j) {
            double s = (j == c) ? 1.0 : 0.0;
            for (int l = j + 1; l < p; ++l) s -= ops.R[(size_t)j * p + l] * out->ri[(size_t)l * p + c];
            out->ri[(size_t)j * p + c] = s / ops.R[(size_t)j * p + j];
        }
    }
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) out->rt[(size_t)i * p + j] = out->ri[(size_t)j * p + i];
    // Harmonics at phase r = t mod F (0-based t, paper time t+1), exact reduction.
    auto harm = [&](long t1, int j, bool cosine) {
        double ang = (2.0 * M_PI / prm.freq) * std::fmod((double)j * (double)t1, prm.freq);
        return cosine ? std::cos(ang) : std::sin(ang);
    };
    out->hh.assign((size_t)F * 2 * k, 0.0);
    out->wh.assign((size_t)F * 2 * k, 0.0);
    for (int r = 0; r < F; ++r) {
        for (int j = 1; j <= k; ++j) {
            out->hh[(size_t)r * 2 * k + 2 * (j - 1)] = harm(r + 1, j, false);
            out->hh[(size_t)r * 2 * k + 2 * (j - 1) + 1] = harm(r + 1, j, true);
            // window of H rows ending at a time t with t mod F = r (take t >= H)
            long t = r + (long)F * ((H + F) / F);
            double ws = 0.0, wc = 0.0;
            for (long s = t - H + 1; s <= t; ++s) {
                ws += harm(s + 1, j, false);
                wc += harm(s + 1, j, true);
            }
            out->wh[(size_t)r * 2 * k + 2 * (j - 1)] = ws;
            out->wh[(size_t)r * 2 * k + 2 * (j - 1) + 1] = wc;
        }
    }
    (void)n;
}

bool build_masked_ops(const bfm_params& prm, MaskedOps* ops)
{
    const int N = prm.n_obs, n = prm.n_hist, k = prm.order, p = 2 + 2 * k;
    const int ng = 2 + 6 * k;
    ops->N = N;
    ops->n = n;
    ops->p = p;
    ops->ng = ng;
    ops->Hmax = window_length(prm, n);
    // One spare slot: the slot about to be written never holds a live entry.
    ops->cap = (ops->Hmax > 0 ? ops->Hmax : 0) + 1;
    ops->x.assign((size_t)N * p, 0.0);
    ops->g.assign((size_t)n * ng, 0.0);
    trend_frame(prm, &ops->tc, &ops->ts);
    std::vector<double> x(p);
    for (int t = 1; t <= N; ++t) {
        design_row_centred(time_at(prm, t), ops->tc, ops->ts, k, prm.freq, x.data());
        for (int j = 0; j < p; ++j) ops->x[(size_t)(t - 1) * p + j] = x[j];
    }
    for (int t = 1; t <= n; ++t) {
        double* gr = &ops->g[(size_t)(t - 1) * ng];
        const double tv = time_at(prm, t);
        const double tau = (tv - ops->tc) / ops->ts;
        gr[0] = tau;
        gr[1] = tau * tau;
        for (int m = 1; m <= 2 * k; ++m) {
            double ang = (2.0 * M_PI / prm.freq) * std::fmod((double)m * tv, prm.freq);
            gr[1 + m] = std::sin(ang);
            gr[1 + 2 * k + m] = std::cos(ang);
        }
        for (int j = 1; j <= k; ++j) {
            gr[1 + 4 * k + j] = tau * gr[1 + j];
            gr[1 + 5 * k + j] = tau * gr[1 + 2 * k + j];
        }
    }
    ops->F = 0;
    ops->ph.clear();
    if (!prm.times && k <= kMaskedMaxOrder && n <= kMaskedPeriodicMaxHist)
        for (int F : kPeriods)
            if (prm.freq == (double)F) ops->F = F;
    if (ops->F > 0) {
        const int F = ops->F;
        ops->ph.assign((size_t)F * 4 * k, 0.0);
        for (int r = 0; r < F; ++r)
            for (int m = 1; m <= 2 * k; ++m) {
                double ang = (2.0 * M_PI / prm.freq) * std::fmod((double)m * (double)(r + 1), prm.freq);
                ops->ph[(size_t)r * 4 * k + 2 * (m - 1)] = std::sin(ang);
                ops->ph[(size_t)r * 4 * k + 2 * (m - 1) + 1] = std::cos(ang);
            }
    }
    return true;
}

}  // namespace bfm
