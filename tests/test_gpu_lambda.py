"""GPU parity of the simulated critical value (bfm_mosum_null_sup,
bfm_critical_value) against the numpy oracle (oracle/lambda_sim.py): the same
counter-based normals on both sides, so every path's statistic is compared."""
import math
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_01751_amd import bfm as b
    b.load()
    return b


@pytest.fixture(scope="module")
def lam():
    from oracle import lambda_sim
    return lambda_sim


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("n,N,H,seed", [(200, 400, 50, 7), (100, 300, 25, 1), (60, 61, 60, 3),
                                        (37, 230, 11, 2 ** 63 + 5)])
def test_sup_parity(bfm, lam, n, N, H, seed):
    """M is a window sum minus (H/n) times the history sum, both of size about
    sqrt(n) before the division by sqrt(n): they may nearly cancel (H = n with
    one monitoring step leaves z_{n+1} - z_1), so the rounding of either side is
    bounded relative to the scale of the sums, |S| or 1, not to S itself."""
    say(f"case null sup n={n} N={N} H={H} seed={seed} paths=6000")
    g = bfm.mosum_null_sup(n=n, N=N, h_window=H, seed=seed, paths=6000).cpu().numpy()
    o = lam.sup_statistic(n, N, H, seed, np.arange(6000))
    err = np.abs(g - o) / np.maximum(o, 1.0)
    say(f"max err {err.max():.3g}")
    assert err.max() < 1e-12


def test_paths_do_not_depend_on_the_split(bfm):
    a = bfm.mosum_null_sup(n=200, N=400, h_window=50, seed=9, paths=20000).cpu().numpy()
    b = bfm.mosum_null_sup(n=200, N=400, h_window=50, seed=9, path0=12345, paths=1000).cpu().numpy()
    np.testing.assert_array_equal(a[12345:13345], b)


@pytest.mark.parametrize("alpha,paths", [(0.05, 20000), (0.01, 777), (0.5, 1), (0.1, 2)])
def test_critical_value_selects_the_rank(bfm, lam, alpha, paths):
    """The device selection returns exactly the rank's order statistic of the
    device statistics, which equals the oracle's lambda."""
    say(f"case critical value alpha={alpha} paths={paths}")
    n, N, H = 100, 300, 25
    got = bfm.critical_value(alpha, n=n, N=N, h_window=H, paths=paths, seed=4)
    g = np.sort(bfm.mosum_null_sup(n=n, N=N, h_window=H, seed=4, paths=paths).cpu().numpy())
    assert got == g[lam.quantile_rank(alpha, paths) - 1]
    ref = lam.critical_value(alpha, n, N, H, paths, seed=4)
    assert abs(got - ref) <= 1e-12 * ref


def test_million_paths_sampled(bfm, lam):
    """One million paths at n = 200, N = 400, H = 50 (the monitoring
    configuration of the 1024x1024 tile): sampled paths against the oracle and
    the defining property of lambda."""
    say("case critical value 1M paths n=200 N=400 H=50")
    n, N, H, P = 200, 400, 50, 1 << 20
    sup = bfm.mosum_null_sup(n=n, N=N, h_window=H, seed=11, paths=P).cpu().numpy()
    got = bfm.critical_value(0.05, n=n, N=N, h_window=H, paths=P, seed=11)
    assert (sup > got).sum() <= 0.05 * P < (sup >= got).sum()
    idx = np.unique(np.r_[np.arange(32), np.arange(P - 32, P),
                          np.random.default_rng(0).integers(0, P, 1500)])
    o = lam.sup_statistic(n, N, H, 11, idx)
    assert (np.abs(sup[idx] - o) / np.maximum(o, 1.0)).max() < 1e-12
    say(f"lambda(alpha=0.05, h=0.25, N/n=2) = {got:.6f}")


def test_single_point_closed_form(bfm):
    """One monitoring step: lambda is the two-sided normal quantile of M."""
    stats = pytest.importorskip("scipy.stats")
    n, H = 200, 50
    got = bfm.critical_value(0.05, n=n, N=n + 1, h_window=H, paths=1 << 20, seed=5)
    ref = stats.norm.ppf(0.975) * math.sqrt((H - (H * H - 2 * H) / n) / n)
    assert abs(got - ref) < 0.005 * ref, (got, ref)


def test_rejects_bad_arguments(bfm):
    for kw in (dict(alpha=0.0), dict(alpha=1.0), dict(paths=0)):
        args = dict(alpha=0.05, n=50, N=100, h_window=10, paths=10)
        args.update(kw)
        with pytest.raises(bfm.BfmError) as e:
            bfm.critical_value(args.pop("alpha"), **args)
        assert e.value.code == bfm.E_INVAL
