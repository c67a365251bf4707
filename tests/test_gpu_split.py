"""GPU parity of the time-split plain kernel (tile-shape tuning): each group of
64 pixels gets 1, 2, 4 or 8 waves that stream consecutive shares of its rows.
Every split is pinned in turn (bfm_tune_set) and checked against the oracle;
bfm_autotune is checked to pick a split that then gives the same results."""
import sys

import numpy as np
import pytest
import torch

from parity import compare, to_numpy

pytestmark = pytest.mark.gpu

LEAN = ("brk", "mag", "sigma", "status", "beta")


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


@pytest.mark.parametrize("split", [1, 2, 4, 8])
@pytest.mark.parametrize("P,N,n,order,freq,h", [
    (4096, 228, 114, 3, 23.0, 0.25),   # the small latency tile
    (1000, 300, 100, 2, 12.0, 0.25),   # ragged wave, N/n = 3 > e: log boundary
    (777, 250, 97, 4, 24.0, 0.25),     # history ends inside a period
    (130, 120, 60, 0, 23.0, 0.4),      # k = 0, fewer monitoring blocks than waves
])
def test_split_parity(bfm, orc, split, P, N, n, order, freq, h):
    from paper_1807_01751_amd.synth import make_series
    say(f"case split={split} P={P} N={N} n={n} k={order} f={freq} h={h}")
    Y, _ = make_series(P, N, n, max(order, 1), freq=freq, seed=P + split, device="cuda")
    bfm.tune_set(Y, split, n=n, order=order, freq=freq, h=h)
    g = to_numpy(bfm.fit_monitor(Y, n=n, order=order, freq=freq, h=h, outputs=LEAN))
    o = orc.fit_monitor(Y.cpu().numpy(), n=n, order=order, freq=freq, h=h, threads=0)
    rep = compare(g, o, bnd=bnd_of(N, n, 2.5))
    say(rep)
    assert rep["not_ok"] == 0


def test_autotune_picks_a_split(bfm):
    from paper_1807_01751_amd.synth import make_series
    say("case autotune P=4096 N=228")
    Y, _ = make_series(4096, 228, 114, 3, seed=77, device="cuda")
    split, times = bfm.autotune(Y, n=114)
    say("autotune", split, times)
    assert split in (1, 2, 4, 8) and split in times and times[split] == min(times.values())
    a = to_numpy(bfm.fit_monitor(Y, n=114, outputs=LEAN))
    bfm.tune_set(Y, 1, n=114)
    b = to_numpy(bfm.fit_monitor(Y, n=114, outputs=LEAN))
    np.testing.assert_array_equal(a["status"], b["status"])
    np.testing.assert_allclose(a["mag"], b["mag"], rtol=1e-12)
    assert (a["brk"] == b["brk"]).mean() > 0.999
    with pytest.raises(bfm.BfmError) as e:
        bfm.tune_set(Y, 3, n=114)
    assert e.value.code == bfm.E_INVAL
    with pytest.raises(bfm.BfmError) as e:
        bfm.tune_set(Y, 2, n=114, freq=22.5)
    assert e.value.code == bfm.E_UNSUPPORTED


@pytest.mark.parametrize("mode", ["plain", "fill"])
def test_default_split_on_a_long_series_over_few_pixels(bfm, orc, mode):
    """4096 pixels x 1000 rows with no tuning: the default rule gives the plain
    path eight waves per 64 pixels (a tile of at most one wave per compute unit
    over N >= 512); filling always streams one wave per 64 pixels.  Both match
    the oracle."""
    from paper_1807_01751_amd.synth import apply_missing, make_missing, make_series, split_rate
    say(f"case default split {mode} P=4096 N=1000 n=500 h=0.1")
    P, N, n, h = 4096, 1000, 500, 0.1
    Y, _ = make_series(P, N, n, 3, seed=91, device="cuda")
    kw = dict(n=n, h=h)
    if mode == "fill":
        r = split_rate(0.1)
        Y = apply_missing(Y, make_missing(N, P, iid=r, runs=r, seed=92, device="cuda"))
        g = to_numpy(bfm.fit_monitor(Y, mask_mode=bfm.MASK_FILL, outputs=LEAN, **kw))
        o = orc.fit_monitor(Y.cpu().numpy(), mask_mode=orc.MASK_FILL, threads=0, **kw)
    else:
        g = to_numpy(bfm.fit_monitor(Y, outputs=LEAN, **kw))
        o = orc.fit_monitor(Y.cpu().numpy(), threads=0, **kw)
    rep = compare(g, o, bnd=bnd_of(N, n, 2.5))
    say(rep)
    assert rep["not_ok"] == 0
