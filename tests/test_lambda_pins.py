"""Pins of the lambda-by-simulation oracle (oracle/lambda_sim.py) against what
the mathematics fixes: numpy's own Philox4x64-10 bit generator, the normal
distribution of the Box-Muller output, closed-form covariances of the MOSUM
under no change, the closed-form critical value of a single monitoring point,
and brute force on tiny inputs.  ``lam`` is the module under test (a mutated
copy in test_lambda_mutants)."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def lam():
    from oracle import lambda_sim
    return lambda_sim


def test_philox_matches_numpy_bit_generator(lam):
    """numpy's Philox raises the counter by one before each block, so its first
    block from counter c is the block of counter c + 1 (with carry)."""
    for seed, j, p in ((0, 1, 0), (7, 5, 3), (2 ** 63 + 11, 1000, 123456), (3, 0, 9)):
        c0 = [j - 1, p, 0, 0] if j > 0 else [2 ** 64 - 1, p - 1, 0, 0]
        bg = np.random.Philox(key=np.array([seed, 0], np.uint64), counter=np.array(c0, np.uint64))
        ref = bg.random_raw(4)
        got = lam.philox4x64([np.uint64(j), np.uint64(p), np.uint64(0), np.uint64(0)],
                             (np.uint64(seed), np.uint64(0)))
        assert [int(x) for x in got] == [int(x) for x in ref], (seed, j, p)


def test_normals_are_standard_normal(lam):
    stats = pytest.importorskip("scipy.stats")
    z = lam.normals(5, np.arange(400), 1000).ravel()
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    zz = lam.normals(5, np.arange(400), 1000)
    for lag in (1, 2, 3, 4):                       # within and across Box-Muller pairs
        r = (zz[lag:] * zz[:-lag]).mean()
        assert abs(r) < 5 / math.sqrt(zz[lag:].size), lag
    # distinct paths and seeds draw different numbers
    assert not np.array_equal(lam.normals(5, [0], 8), lam.normals(5, [1], 8))
    assert not np.array_equal(lam.normals(5, [0], 8), lam.normals(6, [0], 8))


def _cov_closed_form(n, H, a, b):
    """n Cov(M_a, M_b) for windows A = (a-H, a], B = (b-H, b] of unit-variance
    steps minus (H/n) times the history sum."""
    A, B, hist = set(range(a - H + 1, a + 1)), set(range(b - H + 1, b + 1)), set(range(1, n + 1))
    h = H / n
    return len(A & B) - h * len(A & hist) - h * len(B & hist) + h * h * n


def test_mosum_covariance_matches_closed_form(lam):
    n, N, H, paths = 40, 100, 10, 40000
    M = lam.mosum_paths(n, N, H, 9, np.arange(paths))
    ks = [n + 1, n + 5, n + H, n + H + 7, N]
    for a in ks:
        for b in ks:
            c = _cov_closed_form(n, H, a, b) / n
            va, vb = _cov_closed_form(n, H, a, a) / n, _cov_closed_form(n, H, b, b) / n
            emp = np.mean(M[a - n - 1] * M[b - n - 1])
            assert abs(emp - c) < 5 * math.sqrt((va * vb + c * c) / paths), (a, b, emp, c)


@pytest.mark.parametrize("n,H,alpha", [(50, 12, 0.05), (80, 20, 0.1), (40, 40, 0.05)])
def test_single_monitoring_point_closed_form(lam, n, H, alpha):
    """With one monitoring step (N = n + 1) the boundary is flat and M is normal
    with variance (H - (H^2 - 2H)/n)/n: lambda is its two-sided quantile."""
    stats = pytest.importorskip("scipy.stats")
    paths = 100000
    got = lam.critical_value(alpha, n, n + 1, H, paths, seed=13)
    var = (H - (H * H - 2 * H) / n) / n
    ref = stats.norm.ppf(1 - alpha / 2) * math.sqrt(var)
    assert abs(got - ref) < 0.02 * ref, (got, ref)


def test_sup_statistic_brute_force(lam):
    """Horizon past e (boundary growing): loops over the definition."""
    n, N, H = 30, 120, 9
    paths = [0, 17, 4242]
    S = lam.sup_statistic(n, N, H, 21, paths)
    z = lam.normals(21, paths, N)
    for c in range(len(paths)):
        best = 0.0
        hist = sum(z[i - 1, c] for i in range(1, n + 1))
        for k in range(n + 1, N + 1):
            win = sum(z[i - 1, c] for i in range(k - H + 1, k + 1))
            m = (win - H / n * hist) / math.sqrt(n)
            r = k / n
            b = math.sqrt(1.0 if r <= math.e else math.log(r))
            best = max(best, abs(m) / b)
        assert abs(S[c] - best) < 1e-12 * best


def test_critical_value_is_the_quantile(lam):
    n, N, H, paths, alpha = 50, 150, 12, 3000, 0.05
    S = lam.sup_statistic(n, N, H, 3, np.arange(paths))
    got = lam.critical_value(alpha, n, N, H, paths, seed=3, chunk=1000)
    assert (S > got).mean() <= alpha < (S >= got).mean()
    assert lam.quantile_rank(0.05, 1000) == 950 and lam.quantile_rank(0.5, 3) == 2


def test_lambda_grows_with_confidence_and_horizon(lam):
    n, H, paths = 40, 10, 20000
    l1 = lam.critical_value(0.10, n, 2 * n, H, paths, seed=1)
    l2 = lam.critical_value(0.05, n, 2 * n, H, paths, seed=1)
    l3 = lam.critical_value(0.05, n, 4 * n, H, paths, seed=1)
    assert l1 < l2 and l2 < l3 + 0.02


def _sup_sample(lam, n, paths, chunk=5000, seed=20180704):
    """S of ``paths`` simulated paths at resolution n (N = 2n, H = n/2), on
    normals from numpy's SFC64 generator (one stream per chunk, in threads): the
    statistic and the quantile are the oracle's, only the normal source is a
    faster library one."""
    from concurrent.futures import ThreadPoolExecutor

    N, H = 2 * n, n // 2
    seqs = np.random.SeedSequence(seed).spawn(paths // chunk)

    def one(ss):
        z = np.random.Generator(np.random.SFC64(ss)).standard_normal((chunk, N))
        return lam.sup_of_normals(n, N, H, z.T)

    with ThreadPoolExecutor(8) as ex:
        return np.sort(np.concatenate(list(ex.map(one, seqs))))


def test_critical_value_matches_section_4_3(lam):
    """Section 4.3 prints the boundary 2.39 for alpha = 0.05, h = 72/144 = 1/2 and
    N/n = 288/144 = 2 (where Eq. 4 is flat, so the boundary is lambda).

    Bound, derived:
      - Monte Carlo: with m = 2e5 paths the true (1 - alpha) quantile of the
        simulated S lies between the order statistics of rank
        r -/+ 3 sqrt(m alpha (1 - alpha)) (binomial 3-sigma band, free of the
        distribution of S).
      - Resolution: the printed value is itself a simulated quantile of the
        same process at a resolution the paper does not state.  The discrete
        sup over n steps per unit of time falls short of the continuous one by
        rho = 0.5826 sqrt(2/n) (Siegmund's corrected diffusion approximation;
        the constant is -zeta(1/2)/sqrt(2 pi) for a random walk, whose steps
        have variance 2/n here), with a remainder of order 1/n taken as at most
        c2 = 0.003 at n >= 500.  So any resolution from n = 2000 up to the
        continuum gives a value between the band at n = 2000 and that band
        raised by rho.
      - The printed value stands for [2.385, 2.395] (tests/golden).
    The printed interval must meet [band_lo(2000) - c2, band_hi(2000) + rho +
    c2].  The correction itself is checked: the corrected bands at n = 500 and
    n = 2000 must overlap."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                    "critical_value_section_4_3.json")))
    half = 0.5 * 10.0 ** -g["printed_decimals"]
    printed_lo, printed_hi = g["lambda_printed"] - half, g["lambda_printed"] + half
    assert (g["alpha"], g["h_over_n"], g["N_over_n"]) == (0.05, 0.5, 2.0)
    alpha, m, c2 = 0.05, 200_000, 0.003
    r = lam.quantile_rank(alpha, m)
    d = math.ceil(3 * math.sqrt(m * alpha * (1 - alpha)))
    siegmund = 1.4603545088095868 / math.sqrt(2 * math.pi)  # -zeta(1/2) / sqrt(2 pi)
    bands = {}
    for n in (500, 2000):
        S = _sup_sample(lam, n, m)
        bands[n] = (S[r - 1 - d], S[r - 1], S[r - 1 + d], siegmund * math.sqrt(2.0 / n))
    print("lambda(0.05, h=1/2, N/n=2) bands (lo, mid, hi, rho):", bands)
    lo, mid, hi, rho = bands[2000]
    assert lo - c2 <= printed_hi and hi + rho + c2 >= printed_lo, bands
    lo5, _, hi5, rho5 = bands[500]
    assert lo5 + rho5 - c2 <= hi + rho and lo + rho - c2 <= hi5 + rho5, bands
    assert abs(mid - g["lambda_printed"]) < 0.02 and abs(mid + rho - g["lambda_printed"]) < 0.02, bands
