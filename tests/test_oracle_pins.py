"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each checks a closed form, an
invariant, a special case that reduces to a textbook result, LAPACK least
squares, or brute force, so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def design(orc, N, order, freq):
    return np.stack([orc.design_row(t, order, freq) for t in range(1, N + 1)])


def noisy(N, P, order=3, freq=23.0, seed=0, f64=True):
    rng = np.random.default_rng(seed)
    t = np.arange(1, N + 1)[:, None]
    y = 0.5 + 5e-4 * t + np.zeros((N, P))
    for j in range(1, order + 1):
        y += rng.uniform(0, 0.2, P) * np.sin(2 * np.pi * j * t / freq + rng.uniform(0, 2 * np.pi, P))
    y += rng.normal(0, 0.02, (N, P))
    return y if f64 else y.astype(np.float32)


# ---------------------------------------------------------------- Eq. 2 ----
def test_design_row_special_values(orc):
    """Eq. 2 at quarter and full periods: sin/cos take exact textbook values."""
    f = 24.0
    x = orc.design_row(6, 3, f)  # 2 pi j 6/24 = j pi/2
    assert x[0] == 1.0 and x[1] == 6.0
    np.testing.assert_allclose(x[2:], [1, 0, 0, -1, -1, 0], atol=1e-15)
    x = orc.design_row(24, 2, f)  # full period: sin 0, cos 1
    np.testing.assert_allclose(x[2:], [0, 1, 0, 1], atol=1e-14)
    x = orc.design_row(17, 4, 23.0)
    for j in range(4):
        assert abs(x[2 + 2 * j] ** 2 + x[3 + 2 * j] ** 2 - 1) < 1e-15
    # the j-th harmonic at t equals the first harmonic at j*t (same frequency ladder)
    assert abs(orc.design_row(17, 4, 23.0)[6] - orc.design_row(51, 1, 23.0)[2]) < 1e-13


# ---------------------------------------------------------------- Eq. 4 ----
def test_boundary_closed_form(orc):
    lam = 2.5
    for r in (1.0, 1.5, 2.0, math.e):
        assert orc.boundary(lam, r) == lam  # log+ x = 1 for x <= e
    for r in (3.0, 5.0, 10.0):
        assert abs(orc.boundary(lam, r) - lam * math.sqrt(math.log(r))) < 1e-15
    # continuous at x = e
    assert abs(orc.boundary(lam, math.e * (1 + 1e-12)) - lam) < 1e-10


# ------------------------------------------------------- Eq. 5 / Eq. 6 ----
def test_exact_trend_series_zero_residuals(orc):
    """y in the column space (dyadic intercept and slope, exact in FP32)."""
    N, n = 96, 48
    t = np.arange(1, N + 1, dtype=np.float64)
    y = (0.5 + t * 2.0 ** -10)[:, None].astype(np.float32)
    r = orc.fit_monitor(y, n=n, order=2)
    assert np.abs(r["resid"]).max() <= 1e-12 * np.abs(y).max()
    np.testing.assert_allclose(r["beta"][:, 0], [0.5, 2.0 ** -10, 0, 0, 0, 0], atol=1e-12)
    assert r["status"][0] == orc.DEGENERATE_SIGMA and r["brk"][0] == -1 and np.isnan(r["mag"][0])


def test_exact_harmonic_series_recovers_beta(orc):
    N, n, K = 120, 60, 3
    X = design(orc, N, K, 23.0)
    beta0 = np.array([0.4, 1e-3, 0.1, -0.05, 0.02, 0.07, -0.03, 0.01])
    y = (X @ beta0)[:, None]
    r = orc.fit_monitor(y, n=n, order=K)
    np.testing.assert_allclose(r["beta"][:, 0], beta0, rtol=0, atol=1e-12)
    assert np.abs(r["resid"]).max() < 1e-13
    assert r["status"][0] == orc.DEGENERATE_SIGMA


def test_column_space_invariance(orc):
    """r(y + X c) = r(y) and sigma, MO unchanged: only the column space matters."""
    N, n, K, P = 160, 80, 2, 6
    X = design(orc, N, K, 23.0)
    y = noisy(N, P, order=K, seed=3)
    c = np.random.default_rng(4).normal(0, 0.3, (2 + 2 * K, P))
    a = orc.fit_monitor(y, n=n, order=K, h=0.3)
    b = orc.fit_monitor(y + X @ c, n=n, order=K, h=0.3)
    np.testing.assert_allclose(b["resid"], a["resid"], atol=1e-12)
    np.testing.assert_allclose(b["sigma"], a["sigma"], rtol=1e-11)
    np.testing.assert_allclose(b["mosum"], a["mosum"], atol=1e-9)
    np.testing.assert_allclose(b["beta"], a["beta"] + c, atol=1e-10)
    np.testing.assert_array_equal(b["brk"], a["brk"])


def test_normal_equations_hold(orc):
    """X_n' r_n = 0; with the intercept column the history residuals sum to 0."""
    N, n, K, P = 200, 100, 3, 5
    X = design(orc, N, K, 23.0)
    y = noisy(N, P, seed=5)
    r = orc.fit_monitor(y, n=n, order=K)
    g = X[:n].T @ r["resid"][:n]
    assert np.abs(g / (np.linalg.norm(X[:n], axis=0)[:, None] * np.linalg.norm(y[:n], axis=0))).max() < 1e-13
    assert np.abs(r["resid"][:n].sum(axis=0)).max() < 1e-12


def test_order_zero_is_simple_linear_regression(orc):
    """K = 0: textbook slope and intercept of y on t."""
    N, n, P = 80, 40, 4
    rng = np.random.default_rng(6)
    y = rng.normal(0, 1, (N, P)) + 0.03 * np.arange(1, N + 1)[:, None]
    r = orc.fit_monitor(y, n=n, order=0, h=0.5)
    t = np.arange(1, n + 1, dtype=np.float64)
    tb = t.mean()
    for i in range(P):
        yb = y[:n, i].mean()
        slope = ((t - tb) * (y[:n, i] - yb)).sum() / ((t - tb) ** 2).sum()
        icpt = yb - slope * tb
        np.testing.assert_allclose(r["beta"][:, i], [icpt, slope], rtol=1e-12, atol=1e-14)
        rss = ((y[:n, i] - icpt - slope * t) ** 2).sum()
        assert abs(r["sigma"][i] - math.sqrt(rss / (n - 2))) < 1e-13 * math.sqrt(rss)


def test_matches_lapack_lstsq(orc):
    N, n, K, P = 228, 114, 3, 8
    X = design(orc, N, K, 23.0)
    y = noisy(N, P, seed=7)
    r = orc.fit_monitor(y, n=n, order=K)
    beta, res, rank, _ = np.linalg.lstsq(X[:n], y[:n], rcond=None)
    assert rank == 8
    np.testing.assert_allclose(r["beta"], beta, rtol=1e-9, atol=1e-12)
    resid = y - X @ beta
    np.testing.assert_allclose(r["resid"], resid, atol=1e-12)
    np.testing.assert_allclose(r["sigma"], np.sqrt(res / (n - 8)), rtol=1e-11)


def test_sigma_scale_equivariance(orc):
    N, n, P = 150, 75, 3
    y = noisy(N, P, seed=8)
    a = orc.fit_monitor(y, n=n)
    b = orc.fit_monitor(-3.0 * y, n=n)
    np.testing.assert_allclose(b["sigma"], 3.0 * a["sigma"], rtol=1e-12)
    np.testing.assert_allclose(b["mosum"], -a["mosum"], atol=1e-11)  # MO(a y) = sign(a) MO(y)
    np.testing.assert_allclose(b["mag"], -a["mag"], rtol=1e-11)
    np.testing.assert_array_equal(b["brk"], a["brk"])


# ---------------------------------------------------------------- Eq. 3 ----
def _recurrence_mosum(resid, sigma, n, H):
    """The running-sum update of the paper's kernel listing, from residuals."""
    N = resid.shape[0]
    out = np.empty(N - n)
    s = resid[n - H + 1:n + 1].sum()  # window of t = n+1 (1-based): s = n+2-H..n+1
    out[0] = s
    for j in range(1, N - n):
        s = s - resid[n - H + j] + resid[n + j]
        out[j] = s
    return out / (sigma * math.sqrt(n))


@pytest.mark.parametrize("N,n,h,hw", [(228, 114, 0.25, 0), (200, 100, 0.5, 0), (60, 30, 0.0, 30),
                                      (400, 50, 0.1, 0), (51, 50, 0.0, 1)])
def test_mosum_windows_match_recurrence_and_prefix(orc, N, n, h, hw):
    y = noisy(N, 3, seed=9)
    r = orc.fit_monitor(y, n=n, h=h, h_window=hw)
    H = hw if hw else int(math.floor(h * n))
    for i in range(3):
        ref = _recurrence_mosum(r["resid"][:, i], r["sigma"][i], n, H)
        np.testing.assert_allclose(r["mosum"][:, i], ref, rtol=1e-10, atol=1e-12)
        c = np.concatenate([[0.0], np.cumsum(r["resid"][:, i])])
        t = np.arange(n + 1, N + 1)
        pre = (c[t] - c[t - H]) / (r["sigma"][i] * math.sqrt(n))
        np.testing.assert_allclose(r["mosum"][:, i], pre, rtol=1e-9, atol=1e-11)
        # a window one longer or shorter does not match
        if H < n:
            bad = _recurrence_mosum(r["resid"][:, i], r["sigma"][i], n, H + 1)
            assert np.abs(bad - r["mosum"][:, i]).max() > 1e-6


def test_break_and_magnitude_follow_the_mosum(orc):
    """brk is the first strict boundary crossing, mag the extreme MO value."""
    N, n = 400, 100
    y = noisy(N, 16, seed=10)
    y[250:, :8] -= 0.15
    r = orc.fit_monitor(y, n=n, lam=2.5)  # N/n = 4 > e: the ln branch is used
    for i in range(16):
        mo = r["mosum"][:, i]
        t = np.arange(n + 1, N + 1)
        b = np.array([orc.boundary(2.5, x / n) for x in t])
        assert b[-1] > 2.5 and b[0] == 2.5
        hit = np.nonzero(np.abs(mo) > b)[0]
        assert r["brk"][i] == (hit[0] if len(hit) else -1)
        hi, lo = mo.max(), mo.min()
        assert r["mag"][i] == (hi if hi >= -lo else lo)
    assert (r["brk"][:8] >= 0).all()


# ----------------------------------------- planted step, closed form ----
def _planted(orc, N, n, H, K, s, d, tau, f=23.0):
    """y = X beta0 + e + step with e orthogonal to col(X_n), zero after n+1-H.

    Then sigma = s exactly, every window before tau sums to 0, and after tau the
    window sum is -d * min(H, t - tau + 1).
    """
    X = design(orc, N, K, f)
    L = n + 1 - H
    z = np.random.default_rng(11).normal(size=L)
    Q, _ = np.linalg.qr(X[:L])
    e = z - Q @ (Q.T @ z)
    e *= s * math.sqrt(n - (2 + 2 * K)) / np.linalg.norm(e)
    beta0 = np.linspace(0.3, -0.2, 2 + 2 * K) * np.r_[1, 1e-3, np.ones(2 * K)]
    y = X @ beta0
    y[:L] += e
    y[tau - 1:] -= d
    return y[:, None]


@pytest.mark.parametrize("N,n,H,K,s,d,tau,lam", [
    (228, 114, 28, 3, 0.02, 0.3, 140, 2.5),
    (400, 200, 50, 3, 0.02, 0.1, 260, 2.5),
    (200, 100, 50, 2, 0.05, 0.2, 150, 2.1),
    (500, 100, 25, 1, 0.03, 0.1, 300, 2.5),  # N/n = 5: boundary above lambda
])
def test_planted_step_closed_form(orc, N, n, H, K, s, d, tau, lam):
    y = _planted(orc, N, n, H, K, s, d, tau)
    r = orc.fit_monitor(y, n=n, order=K, h_window=H, lam=lam)
    assert r["status"][0] == orc.OK
    assert abs(r["sigma"][0] - s) < 1e-12
    scale = s * math.sqrt(n)
    brk = -1
    for t in range(tau, N + 1):
        mo = d * min(H, t - tau + 1) / scale
        b = lam * math.sqrt(max(1.0, math.log(t / n)) if t / n > math.e else 1.0)
        if mo > b:
            brk = t - n - 1
            break
    assert brk >= 0 and r["brk"][0] == brk
    if tau + H - 1 <= N:
        assert abs(r["mag"][0] - (-d * H / scale)) < 1e-9
    mo = r["mosum"][:, 0]
    assert np.abs(mo[: tau - n - 1]).max() < 1e-10


def test_planted_step_index_formula_flat_boundary(orc):
    """At N/n <= e: brk = tau + j* - n - 2 with j* = floor(lam s sqrt(n)/d) + 1."""
    N, n, H, K, s, d, tau, lam = 228, 114, 28, 3, 0.02, 0.3, 150, 2.5
    r = orc.fit_monitor(_planted(orc, N, n, H, K, s, d, tau), n=n, order=K, h_window=H, lam=lam)
    jstar = math.floor(lam * s * math.sqrt(n) / d) + 1
    assert r["brk"][0] == tau + jstar - n - 2
    assert abs(abs(r["mag"][0]) - d * H / (s * math.sqrt(n))) < 1e-9


def test_noisy_planted_steps_are_flagged(orc):
    """The generator's -0.3 step (15 noise sigmas) is flagged at or soon after tau."""
    N, n, P = 228, 114, 64
    rng = np.random.default_rng(12)
    y = noisy(N, P, seed=12)
    tau = rng.integers(n + 1, N - 10, P)
    has = np.arange(P) < 32
    for i in range(32):
        y[tau[i] - 1:, i] -= 0.3
    r = orc.fit_monitor(y, n=n)
    assert (r["status"] == orc.OK).all()
    brk_t = r["brk"][:32] + n + 1  # 1-based time of the first crossing
    assert (r["brk"][:32] >= 0).all()
    assert (brk_t >= tau[:32] - 1).all() and (brk_t <= tau[:32] + 6).all()
    assert (r["mag"][:32] < 0).all()
    assert (r["brk"][~has] == -1).mean() > 0.8


# -------------------------------------------------------- missing values ----
def test_all_valid_mask_equals_plain(orc):
    N, n, P = 200, 100, 5
    y = noisy(N, P, seed=13)
    a = orc.fit_monitor(y, n=n)
    b = orc.fit_monitor(y, n=n, mask_mode=orc.MASK_NAN)
    c = orc.fit_monitor(y, n=n, mask_mode=orc.MASK_EXPLICIT, valid=np.ones((N, P), np.uint8))
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
        np.testing.assert_array_equal(a[k], c[k])


def test_nan_equals_explicit_mask(orc):
    N, n, P = 200, 100, 6
    y = noisy(N, P, seed=14)
    miss = np.random.default_rng(15).random((N, P)) < 0.2
    yn = y.copy()
    yn[miss] = np.nan
    a = orc.fit_monitor(yn, n=n, mask_mode=orc.MASK_NAN)
    yg = y.copy()
    yg[miss] = 1e6  # garbage the explicit mask must hide
    b = orc.fit_monitor(yg, n=n, mask_mode=orc.MASK_EXPLICIT, valid=(~miss).astype(np.uint8))
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("N,n,K,P,h,lam", [(120, 60, 2, 5, 0.25, 2.5), (400, 100, 2, 24, 0.25, 2.0)])
def test_masked_compaction_brute_force(orc, N, n, K, P, h, lam):
    """Masked result = a plain fit on the valid subsequence at its original t.

    The second shape has N/n = 4 > e, so the boundary's compacted position u/n_v
    matters; small late steps make the crossing index sensitive to it."""
    y = noisy(N, P, order=K, seed=16)
    rng = np.random.default_rng(17)
    miss = rng.random((N, P)) < 0.25
    y[miss] = np.nan
    y[90:, 0] -= 0.3
    for i in range(1, P, 2):
        y[int(rng.integers(int(0.7 * N), N - 20)):, i] -= 0.03
    r = orc.fit_monitor(y, n=n, order=K, h=h, lam=lam, mask_mode=orc.MASK_NAN)
    X = design(orc, N, K, 23.0)
    for i in range(P):
        v = np.nonzero(~miss[:, i])[0]
        vh = v[v < n]
        nv = len(vh)
        beta = np.linalg.lstsq(X[vh], y[vh, i], rcond=None)[0]
        e = y[v, i] - X[v] @ beta
        sig = math.sqrt((e[:nv] ** 2).sum() / (nv - (2 + 2 * K)))
        H = int(math.floor(h * nv))
        mo = np.array([e[u - H + 1:u + 1].sum() for u in range(nv, len(v))]) / (sig * math.sqrt(nv))
        np.testing.assert_allclose(r["beta"][:, i], beta, rtol=1e-9, atol=1e-11)
        assert abs(r["sigma"][i] - sig) < 1e-11
        np.testing.assert_allclose(r["mosum"][v[nv:] - n, i], mo, atol=1e-10)
        assert np.isnan(r["mosum"][:, i]).sum() == (N - n) - (len(v) - nv)
        u1 = np.arange(nv + 1, len(v) + 1) / nv
        b = lam * np.sqrt(np.where(u1 <= math.e, 1.0, np.log(np.maximum(u1, 1.0))))
        hit = np.nonzero(np.abs(mo) > b)[0]
        assert r["brk"][i] == (v[nv + hit[0]] - n if len(hit) else -1)
    assert r["brk"][0] >= 0


# ------------------------------------------------------ degenerate cases ----
def test_status_codes(orc):
    N, n, K = 60, 20, 3
    y = noisy(N, 6, order=K, seed=18)
    y[5, 0] = np.nan                      # NaN without a mask
    y[:, 1] = 0.25                        # constant: sigma = 0
    y[:13, 2] = np.nan                    # only 7 valid history obs <= p = 8
    y[n:, 3] = np.nan                     # no monitor observation
    r0 = orc.fit_monitor(y, n=n, order=K)
    assert r0["status"][0] == orc.NONFINITE and r0["brk"][0] == -1 and np.isnan(r0["mag"][0])
    assert r0["status"][1] == orc.DEGENERATE_SIGMA
    r1 = orc.fit_monitor(y, n=n, order=K, mask_mode=orc.MASK_NAN)
    assert r1["status"][0] == orc.OK
    assert r1["status"][2] == orc.INSUFFICIENT and np.isnan(r1["sigma"][2])
    assert r1["status"][3] == orc.NO_MONITOR and np.isfinite(r1["sigma"][3])
    assert (r1["status"][4:] == orc.OK).all()
    # f = 2 aliases the first harmonic: sin(pi t) = 0 for integer t
    r2 = orc.fit_monitor(noisy(N, 2, order=1, seed=19), n=n, order=1, freq=2.0)
    assert (r2["status"] == orc.RANK_DEFICIENT).all()
    # window longer than the masked history
    y4 = noisy(N, 1, order=1, seed=20)
    y4[:15] = np.nan
    r3 = orc.fit_monitor(y4, n=n, order=1, h_window=10, mask_mode=orc.MASK_NAN)
    assert r3["status"][0] == orc.INSUFFICIENT


def test_rejects_bad_parameters(orc):
    y = noisy(40, 2, seed=21)
    for kw in (dict(n=40), dict(n=0), dict(n=20, h=0.0), dict(n=20, h=1.5), dict(n=20, lam=0.0),
               dict(n=20, order=-1), dict(n=20, freq=0.0), dict(n=20, h_window=21)):
        with pytest.raises(ValueError):
            orc.fit_monitor(y, **kw)


def test_threads_do_not_change_results(orc):
    y = noisy(228, 300, seed=22, f64=False)
    a = orc.fit_monitor(y, n=114, threads=1)
    b = orc.fit_monitor(y, n=114, threads=4)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


# ------------------------------------- irregular time (Section 4, Chile) ----
def acquisition_days(N, seed=0):
    """Day numbers of N acquisitions: gaps of 8 to 48 days (revisits of 8 or 16
    days, some lost to clouds), strictly increasing, starting at day 18."""
    rng = np.random.default_rng(seed)
    return 18.0 + np.concatenate([[0.0], np.cumsum(rng.choice([8.0, 16.0, 16.0, 16.0, 32.0, 48.0], N - 1))])


def seasonal_in_time(days, P, order=3, seed=0, noise=0.02):
    rng = np.random.default_rng(seed)
    t = days[:, None]
    y = 0.5 + 2e-5 * t + np.zeros((len(days), P))
    for j in range(1, order + 1):
        y += rng.uniform(0, 0.2, P) * np.sin(2 * np.pi * j * t / 365.0 + rng.uniform(0, 2 * np.pi, P))
    return y + rng.normal(0, noise, y.shape)


def test_times_equal_to_the_index_give_the_regular_path(orc):
    """times = 1..N is the regular series: every output identical."""
    y = noisy(150, 40, seed=30)
    y[np.random.default_rng(31).random(y.shape) < 0.2] = np.nan
    idx = np.arange(1, 151, dtype=np.float64)
    for mode in (orc.MASK_NONE, orc.MASK_NAN):
        a = orc.fit_monitor(y, n=75, mask_mode=mode)
        b = orc.fit_monitor(y, n=75, mask_mode=mode, times=idx)
        for k in a:
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_exact_series_in_irregular_time_recovers_beta(orc):
    """A noise-free season-trend series in day numbers (f = 365): the fit
    recovers the coefficients of Eq. 2 that built it."""
    N, n, k = 288, 144, 3
    days = acquisition_days(N, seed=32)
    beta = np.array([0.4, 3e-5, 0.1, -0.05, 0.03, 0.02, -0.01, 0.015])
    X = np.column_stack([np.ones(N), days] + [f(2 * np.pi * j * days / 365.0)
                                                for j in range(1, k + 1) for f in (np.sin, np.cos)])
    y = (X @ beta)[:, None]
    r = orc.fit_monitor(y, n=n, order=k, freq=365.0, h_window=72, times=days)
    np.testing.assert_allclose(r["beta"][:, 0], beta, rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(r["resid"][:, 0], 0.0, atol=1e-12)
    assert r["status"][0] == orc.DEGENERATE_SIGMA


@pytest.mark.parametrize("shift,scale", [(365.0 * 3, 1.0), (17.3, 1.0), (0.0, 1.0 / 365.0)])
def test_time_origin_and_unit_do_not_change_the_monitor(orc, shift, scale):
    """Shifting every time (the trend and harmonic columns span the same space)
    or changing the unit together with f leaves the fitted values, sigma, the
    MOSUM and the break unchanged."""
    N, n = 288, 144
    days = acquisition_days(N, seed=33)
    y = seasonal_in_time(days, 30, seed=34)
    y[200:, ::3] -= 0.2
    a = orc.fit_monitor(y, n=n, order=3, freq=365.0, h_window=72, times=days)
    b = orc.fit_monitor(y, n=n, order=3, freq=365.0 * scale, h_window=72,
                        times=(days + shift) * scale)
    np.testing.assert_array_equal(a["brk"], b["brk"])
    for key in ("sigma", "mag", "mosum", "resid"):
        np.testing.assert_allclose(a[key], b[key], rtol=1e-9, atol=1e-10, err_msg=key)
    assert (a["brk"][::3] >= 0).all()


def test_irregular_time_with_gaps_brute_force(orc):
    """Dropped observations in irregular time: LAPACK least squares on the
    valid history at the observations' day numbers, windows summed by brute
    force, boundary at compacted positions."""
    N, n, k, H, lam = 288, 144, 3, 72, 2.5
    days = acquisition_days(N, seed=35)
    P = 12
    y = seasonal_in_time(days, P, seed=36)
    rng = np.random.default_rng(37)
    miss = rng.random((N, P)) < 0.2
    y[miss] = np.nan
    y[220:, ::2] -= 0.15
    r = orc.fit_monitor(y, n=n, order=k, freq=365.0, h_window=H, lam=lam,
                        mask_mode=orc.MASK_NAN, times=days)
    X = np.column_stack([np.ones(N), days] + [f(2 * np.pi * j * days / 365.0)
                                                for j in range(1, k + 1) for f in (np.sin, np.cos)])
    for i in range(P):
        v = np.nonzero(~miss[:, i])[0]
        vh = v[v < n]
        nv = len(vh)
        beta = np.linalg.lstsq(X[vh], y[vh, i], rcond=None)[0]
        e = y[v, i] - X[v] @ beta
        sig = math.sqrt((e[:nv] ** 2).sum() / (nv - (2 + 2 * k)))
        mo = np.array([e[u - H + 1:u + 1].sum() for u in range(nv, len(v))]) / (sig * math.sqrt(nv))
        np.testing.assert_allclose(r["beta"][:, i], beta, rtol=1e-7, atol=1e-11)
        assert abs(r["sigma"][i] - sig) < 1e-11
        np.testing.assert_allclose(r["mosum"][v[nv:] - n, i], mo, atol=1e-9)
        u1 = np.arange(nv + 1, len(v) + 1) / nv
        b = lam * np.sqrt(np.where(u1 <= math.e, 1.0, np.log(np.maximum(u1, 1.0))))
        hit = np.nonzero(np.abs(mo) > b)[0]
        assert r["brk"][i] == (v[nv + hit[0]] - n if len(hit) else -1)
    assert (r["brk"][::2] >= 0).all()


def test_rejects_times_that_do_not_increase(orc):
    y = noisy(40, 2, seed=38)
    t = np.arange(1.0, 41.0)
    for bad in (t[::-1].copy(), np.where(t == 10, 9.0, t), np.where(t == 5, np.nan, t)):
        with pytest.raises(ValueError):
            orc.fit_monitor(y, n=20, times=bad)


# ------------------------------------ filling (footnote of Section 3) ----
def test_fill_is_forward_then_backward_fill(orc):
    """MASK_FILL equals the plain path on the series filled by pandas (ffill,
    then bfill for the leading gap), bit for bit."""
    pd = pytest.importorskip("pandas")
    N, n, P = 200, 100, 40
    y = noisy(N, P, seed=39)
    rng = np.random.default_rng(40)
    y[rng.random((N, P)) < 0.1] = np.nan
    for i in range(0, P, 4):                       # runs, leading and trailing gaps
        a = int(rng.integers(0, N - 10))
        y[a:a + int(rng.integers(2, 10)), i] = np.nan
    y[:7, 1] = np.nan
    y[-5:, 2] = np.nan
    y[3, 5] = np.inf
    filled = pd.DataFrame(np.where(np.isfinite(y), y, np.nan)).ffill().bfill().to_numpy()
    assert np.isfinite(filled).all()
    a = orc.fit_monitor(y, n=n, mask_mode=orc.MASK_FILL)
    b = orc.fit_monitor(filled, n=n, mask_mode=orc.MASK_NONE)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_fill_special_cases(orc):
    N, n = 60, 30
    y = noisy(N, 4, seed=41)
    complete = orc.fit_monitor(y, n=n)
    r = orc.fit_monitor(y, n=n, mask_mode=orc.MASK_FILL)
    for k in r:                                     # nothing missing: the plain path
        np.testing.assert_array_equal(r[k], complete[k], err_msg=k)
    y[:, 1] = np.nan                                # nothing to fill from
    y[:n, 2] = np.nan                               # history backward-filled: constant
    y[[0, 1, 2, 40], 3] = np.nan                    # leading gap takes y[3]
    r = orc.fit_monitor(y, n=n, mask_mode=orc.MASK_FILL)
    assert r["status"][1] == orc.INSUFFICIENT and r["brk"][1] == -1
    assert r["status"][2] == orc.DEGENERATE_SIGMA
    assert r["status"][3] == orc.OK
    y3 = y[:, 3].copy()
    y3[:3] = y3[3]
    y3[40] = y3[39]
    ref = orc.fit_monitor(y3[:, None], n=n)
    for k in ref:
        np.testing.assert_array_equal(r[k][..., 3:4], ref[k], err_msg=k)


# ------------------------------------------ high signal-to-noise ratio ----

_LD = np.longdouble
_EXT_CACHE = {}


def _extended_reference(Y, N, n, K, f, H):
    """sigma and MO of Algorithm 1 in x87 extended precision (64-bit mantissa):
    design rows of Eq. 2 with a long-double pi and sinl/cosl, least squares by
    classical Gram-Schmidt applied twice, residuals, their scale and brute-force
    windows.  Independent of the oracle; its own rounding is ~2048 times below
    FP64's, so it stands for the exact result."""
    pi = _LD("3.141592653589793238462643383279502884")
    t = np.arange(1, N + 1).astype(_LD)
    cols = [np.ones(N, _LD), t / _LD(n)]
    for j in range(1, K + 1):
        a = 2 * pi * j * t / _LD(f)
        cols += [np.sin(a), np.cos(a)]
    X = np.stack(cols, 1)
    p = X.shape[1]
    Q = np.zeros((n, p), _LD)
    R = np.zeros((p, p), _LD)
    for j in range(p):
        v = X[:n, j].copy()
        for _ in range(2):
            c = Q[:, :j].T @ v
            v = v - Q[:, :j] @ c
            R[:j, j] += c
        R[j, j] = np.sqrt(v @ v)
        Q[:, j] = v / R[j, j]
    Yl = Y.astype(_LD)
    b = Q.T @ Yl[:n]
    beta = np.zeros_like(b)
    for i in range(p - 1, -1, -1):
        beta[i] = (b[i] - R[i, i + 1:] @ beta[i + 1:]) / R[i, i]
    r = Yl - X @ beta
    sig = np.sqrt((r[:n] ** 2).sum(0) / (n - p))
    C = np.vstack([np.zeros((1, Y.shape[1]), _LD), np.cumsum(r, 0)])
    tt = np.arange(n + 1, N + 1)
    mo = (C[tt] - C[tt - H]) / (sig * np.sqrt(_LD(n)))
    return sig.astype(np.float64), mo.astype(np.float64)


@pytest.mark.parametrize("noise,mo_bound", [(1e-5, 2e-10), (1.5e-6, 1e-9)])
def test_high_snr_matches_extended_precision(orc, noise, mo_bound):
    """Near the DEGENERATE_SIGMA threshold (sigma <= 1e-6 max|y|) the MOSUM is a
    small difference of large window sums, so rounding in the design rows or in
    the fit shows.  Against the extended-precision result: sigma within 1e-10
    and MO (normwise per pixel) within the bounds here, at noise 1e-5 and 1.5e-6
    on series of level 0.5-1.2 stored as float32."""
    if np.finfo(_LD).eps > 1e-18:
        pytest.skip("long double is not an extended type on this platform")
    N, n, K, f, H, P = 400, 200, 3, 23.0, 50, 64
    key = (noise,)
    if key not in _EXT_CACHE:
        rng = np.random.default_rng(4)
        t = np.arange(1, N + 1)[:, None]
        y = 0.5 + 5e-4 * t + np.zeros((N, P))
        for j in range(1, K + 1):
            y += rng.uniform(0, 0.2, P) * np.sin(2 * np.pi * j * t / f + rng.uniform(0, 2 * np.pi, P))
        y = (y + rng.normal(0, noise, (N, P))).astype(np.float32)
        _EXT_CACHE[key] = (y,) + _extended_reference(y, N, n, K, f, H)
    y, sig, mo = _EXT_CACHE[key]
    r = orc.fit_monitor(y, n=n, order=K, freq=f, h_window=H, lam=2.5)
    assert (r["status"] == 0).all()
    assert np.abs(r["sigma"] / sig - 1).max() < 1e-10
    err = np.abs(r["mosum"] - mo).max(0) / np.abs(mo).max(0)
    assert err.max() < mo_bound, err.max()
