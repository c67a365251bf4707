"""GPU parity of the method variants: observation times in place of the index
(Section 4, the Chile scene: day numbers, f = 365) and filling of missing
observations (footnote of Section 3), against the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

from parity import compare, to_numpy

pytestmark = pytest.mark.gpu

ALL = ("brk", "mag", "sigma", "status", "beta", "resid", "mosum")
LEAN = ("brk", "mag", "sigma", "status")


@pytest.fixture(scope="module")
def bfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_01751_amd import bfm as b
    b.load()
    return b


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def bnd_of(N, n, lam):
    t = np.arange(n + 1, N + 1) / n
    return lam * np.sqrt(np.where(t <= np.e, 1.0, np.log(np.maximum(t, 1.0))))


def chile_like(P, N=288, n=144, seed=0, miss=0.0):
    """Series at the acquisition days of an unevenly sampled scene (N = 288
    images, history n = 144, k = 3, f = 365 days)."""
    from paper_1807_01751_amd.synth import (acquisition_days, apply_missing, make_missing,
                                            make_series, split_rate)
    days = acquisition_days(N, seed=seed)
    Y, _ = make_series(P, N, n, 3, freq=365.0, times=days, trend=2e-5, seed=seed + 1,
                       device="cuda")
    if miss > 0:
        r = split_rate(miss)
        Y = apply_missing(Y, make_missing(N, P, iid=r, runs=r, seed=seed + 2, device="cuda"))
    return Y, days


# ------------------------------------------------------------ times ----
def test_times_plain_parity(bfm, orc):
    say("case times plain P=3000 N=288 n=144 f=365 h=72")
    Y, days = chile_like(3000, seed=1)
    g = to_numpy(bfm.fit_monitor(Y, n=144, order=3, freq=365.0, h_window=72, times=days,
                                 outputs=ALL))
    o = orc.fit_monitor(Y.cpu().numpy(), n=144, order=3, freq=365.0, h_window=72, times=days,
                        threads=0)
    rep = compare(g, o, bnd=bnd_of(288, 144, 2.5))
    say(rep)
    assert rep["not_ok"] == 0 and (g["brk"] >= 0).mean() > 0.1


@pytest.mark.parametrize("mode", ["nan", "explicit"])
def test_times_masked_parity(bfm, orc, mode):
    from test_gpu_masked import check, hist_count
    say(f"case times masked {mode} P=2000 N=288 n=144 miss=0.2")
    Y, days = chile_like(2000, seed=3, miss=0.2)
    kw = dict(n=144, order=3, freq=365.0, h_window=72, times=days)
    if mode == "nan":
        g = to_numpy(bfm.fit_monitor(Y, mask_mode=bfm.MASK_NAN, outputs=ALL, **kw))
        o = orc.fit_monitor(Y.cpu().numpy(), mask_mode=orc.MASK_NAN, threads=0, **kw)
        used = hist_count(Y, 144)
    else:
        valid = torch.isfinite(Y).to(torch.uint8)
        Yg = torch.where(valid.bool(), Y, torch.full_like(Y, 5.0))
        g = to_numpy(bfm.fit_monitor(Yg, mask_mode=bfm.MASK_EXPLICIT, valid=valid, outputs=ALL, **kw))
        o = orc.fit_monitor(Yg.cpu().numpy(), mask_mode=orc.MASK_EXPLICIT,
                            valid=valid.cpu().numpy(), threads=0, **kw)
        used = hist_count(Yg, 144, valid)
    say(check(g, o, 2.5, used))


def test_index_times_match_the_oracle(bfm, orc):
    """times = 1..N with f = 23 (table-driven kernels instead of the
    period-blocked ones) against the oracle's index time."""
    from paper_1807_01751_amd.synth import make_series
    say("case times=index P=2000 N=228 n=114")
    Y, _ = make_series(2000, 228, 114, 3, seed=5, device="cuda")
    idx = np.arange(1, 229, dtype=np.float64)
    g = to_numpy(bfm.fit_monitor(Y, n=114, times=idx, outputs=ALL))
    o = orc.fit_monitor(Y.cpu().numpy(), n=114, threads=0)
    say(compare(g, o, bnd=bnd_of(228, 114, 2.5)))


def test_times_operator_cache_follows_the_times(bfm, orc):
    """Two calls with the same parameters and different times each get the
    operators of their own times (the context caches per time vector)."""
    say("case times cache P=1000")
    Y, days = chile_like(1000, seed=7)
    for tv in (days, days * 1.5 + 3.0, days):
        g = to_numpy(bfm.fit_monitor(Y, n=144, order=3, freq=365.0, h_window=72, times=tv,
                                     outputs=ALL))
        o = orc.fit_monitor(Y.cpu().numpy(), n=144, order=3, freq=365.0, h_window=72, times=tv,
                            threads=0)
        compare(g, o, bnd=bnd_of(288, 144, 2.5))


def test_times_unsupported_and_rejected(bfm):
    Y, days = chile_like(64, seed=9)
    with pytest.raises(bfm.BfmError) as e:
        bfm.fit_monitor(Y.to(torch.float16), n=144, freq=365.0, h_window=72, times=days)
    assert e.value.code == bfm.E_UNSUPPORTED
    with pytest.raises(bfm.BfmError) as e:
        bfm.fit_monitor(Y, n=144, freq=365.0, h_window=72, times=days[::-1].copy())
    assert e.value.code == bfm.E_INVAL


# ------------------------------------------------------------- fill ----
def gappy(P, N, n, seed, freq=23.0, order=3):
    """Series with 10% missing observations: iid gaps and cloud runs, leading
    and trailing gaps, an all-missing pixel, Inf values and a pixel observed only
    after the history."""
    from paper_1807_01751_amd.synth import apply_missing, make_missing, make_series, split_rate
    Y, _ = make_series(P, N, n, order, freq=freq, seed=seed, device="cuda")
    r = split_rate(0.1)
    Y = apply_missing(Y, make_missing(N, P, iid=r, runs=r, seed=seed + 1, device="cuda"))
    Y[:9, 1] = float("nan")
    Y[-4:, 2] = float("nan")
    Y[:, 3] = float("nan")
    Y[7, 4] = float("inf")
    Y[50, 5] = -float("inf")
    Y[:n, 6] = float("nan")
    Y[:, P - 1] = float("nan")           # the last lane of the last wave
    return Y


@pytest.mark.parametrize("freq,order,N,n", [(23.0, 3, 228, 114), (12.0, 2, 150, 72),
                                            (24.0, 4, 400, 100), (22.5, 3, 228, 114),
                                            (23.0, 6, 300, 150)])
def test_fill_parity(bfm, orc, freq, order, N, n):
    """f in {12, 23, 24} takes the period-blocked kernel, f = 22.5 and k = 6 the
    table-driven one; both with and without the per-row exports."""
    say(f"case fill f={freq} k={order} N={N} n={n} P=2500")
    Y = gappy(2500, N, n, seed=11 + order, freq=freq, order=order)
    o = orc.fit_monitor(Y.cpu().numpy(), n=n, order=order, freq=freq,
                        mask_mode=orc.MASK_FILL, threads=0)
    assert o["status"][3] == orc.INSUFFICIENT and o["status"][6] == orc.DEGENERATE_SIGMA
    g = to_numpy(bfm.fit_monitor(Y, n=n, order=order, freq=freq, mask_mode=bfm.MASK_FILL,
                                 outputs=ALL))
    rep = compare(g, o, bnd=bnd_of(N, n, 2.5))
    say(rep)
    lean = to_numpy(bfm.fit_monitor(Y, n=n, order=order, freq=freq, mask_mode=bfm.MASK_FILL,
                                    outputs=LEAN))
    for k in LEAN:
        np.testing.assert_array_equal(lean[k], g[k], err_msg=k)
    assert (o["status"] == 0).mean() > 0.99


def test_fill_of_a_complete_series_is_the_plain_path(bfm):
    from paper_1807_01751_amd.synth import make_series
    say("case fill complete P=3000 N=228")
    Y, _ = make_series(3000, 228, 114, 3, seed=21, device="cuda")
    a = to_numpy(bfm.fit_monitor(Y, n=114, outputs=ALL))
    b = to_numpy(bfm.fit_monitor(Y, n=114, mask_mode=bfm.MASK_FILL, outputs=ALL))
    for k in ALL:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_fill_with_times(bfm, orc):
    say("case fill + times P=2000 N=288")
    Y, days = chile_like(2000, seed=23, miss=0.1)
    kw = dict(n=144, order=3, freq=365.0, h_window=72, times=days)
    g = to_numpy(bfm.fit_monitor(Y, mask_mode=bfm.MASK_FILL, outputs=ALL, **kw))
    o = orc.fit_monitor(Y.cpu().numpy(), mask_mode=orc.MASK_FILL, threads=0, **kw)
    say(compare(g, o, bnd=bnd_of(288, 144, 2.5)))


def test_fill_degenerate_parameters(bfm, orc):
    """A rank-deficient shared design (f = 2, k = 1) fills status only; an
    all-missing pixel is INSUFFICIENT there too."""
    from paper_1807_01751_amd.synth import make_series
    Y, _ = make_series(100, 60, 30, 1, seed=25, device="cuda")
    Y[:, 4] = float("nan")
    Y[3, 5] = float("nan")
    g = to_numpy(bfm.fit_monitor(Y, n=30, order=1, freq=2.0, mask_mode=bfm.MASK_FILL,
                                 outputs=("brk", "status")))
    o = orc.fit_monitor(Y.cpu().numpy(), n=30, order=1, freq=2.0, mask_mode=orc.MASK_FILL)
    np.testing.assert_array_equal(g["status"], o["status"])
    assert g["status"][4] == bfm.ST_INSUFFICIENT and (g["brk"] == -1).all()


def test_fill_16bit_unsupported(bfm):
    Y = gappy(128, 228, 114, seed=27).to(torch.bfloat16)
    with pytest.raises(bfm.BfmError) as e:
        bfm.fit_monitor(Y, n=114, mask_mode=bfm.MASK_FILL)
    assert e.value.code == bfm.E_UNSUPPORTED


def test_fill_full_tile_sampled(bfm, orc):
    """1024x1024 pixels, N=400, n=200, k=3 with 10% missing, filled: sampled
    parity at the full size."""
    say("case fill full tile P=1048576 N=400 n=200")
    P, N, n = 1 << 20, 400, 200
    Y = gappy(P, N, n, seed=29)
    g = to_numpy(bfm.fit_monitor(Y, n=n, mask_mode=bfm.MASK_FILL, outputs=LEAN))
    rng = np.random.default_rng(5)
    idx = np.unique(np.r_[np.arange(64), np.arange(P - 64, P), rng.integers(0, P, 3000)])
    Ys = Y[:, torch.as_tensor(idx, device="cuda")].cpu().numpy()
    o = orc.fit_monitor(Ys, n=n, mask_mode=orc.MASK_FILL, threads=0)
    gs = {k: v[idx] for k, v in g.items()}
    say("fill full tile sample", compare(gs, o, bnd=bnd_of(N, n, 2.5)))
