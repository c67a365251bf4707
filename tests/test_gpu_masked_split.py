"""GPU parity of the history split of the period-blocked missing-value kernel:
each group of 64 pixels gets 2, 4 or 8 waves that stream consecutive shares of
the history blocks; the last wave adds up the shares' sums, takes the window's
observations from the earlier shares' rings and monitors.  Every split is
pinned in turn (bfm_tune_set) and checked against the oracle at the FP64 bar,
and against the unsplit kernel; bfm_autotune is checked on the NaN mode."""
import sys

import numpy as np
import pytest
import torch

from parity import compare, to_numpy, used_history

pytestmark = pytest.mark.gpu

ALL = ("brk", "mag", "sigma", "status", "beta", "mosum")


@pytest.fixture(scope="module")
def bfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_01751_amd import bfm as b
    b.load()
    return b


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def masked_series(P, N, n, order, seed, miss, freq, dtype=torch.float32, tail_gap=0):
    from paper_1807_01751_amd.synth import apply_missing, make_missing, make_series, split_rate
    Y, _ = make_series(P, N, n, max(order, 1), freq=freq, seed=seed, device="cuda")
    r = split_rate(miss)
    m = make_missing(N, P, iid=r, runs=r, seed=seed + 100, device="cuda")
    if tail_gap:
        # Every pixel misses the last `tail_gap` history rows: the last shares
        # hold few observations and the window reaches into earlier shares.
        m[n - tail_gap:n] = True
    return apply_missing(Y, m).to(dtype), m


CASES = [
    # P, N, n, order, freq, h, miss, dtype, tail_gap, mode
    (1000, 400, 200, 3, 23.0, 0.25, 0.25, torch.float32, 0, "nan"),
    (777, 300, 199, 4, 24.0, 0.25, 0.25, torch.float32, 0, "explicit"),  # history ends inside a block
    (1500, 400, 200, 2, 12.0, 0.25, 0.4, torch.float32, 60, "nan"),      # window reaches back past a gap
    (2000, 400, 200, 3, 23.0, 0.25, 0.25, torch.float16, 0, "nan"),
    (130, 250, 190, 0, 23.0, 0.25, 0.1, torch.float32, 0, "nan"),        # k = 0, 9 history blocks
    (1000, 400, 200, 3, 23.0, 0.1, 0.25, torch.float32, 30, "nan"),      # short windows: 8 waves fit
    (900, 300, 240, 2, 24.0, 0.08, 0.3, torch.float32, 40, "explicit"),
]


def lds_bytes(split, H, F):
    """LDS of the period-blocked missing-value kernel: the rings of every wave
    (6 bytes per slot and lane) and, with a split, the staging of the sums."""
    return split * H * 64 * 6 + (64 * (8 * (F + 2) + 4 * (F + 4) + 8 * split) if split > 1 else 0)


@pytest.mark.parametrize("split", [2, 4, 8])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_masked_split_parity(bfm, orc, split, case):
    P, N, n, order, freq, h, miss, dtype, gap, mode = CASES[case]
    say(f"case masked split={split} P={P} N={N} n={n} k={order} f={freq} h={h} miss={miss} {dtype} "
        f"gap={gap} {mode}")
    Y, m = masked_series(P, N, n, order, 300 + case, miss, freq, dtype, gap)
    kw = dict(n=n, order=order, freq=freq, h=h)
    if mode == "nan":
        mm, valid = bfm.MASK_NAN, None
    else:
        mm, valid = bfm.MASK_EXPLICIT, (~m).to(torch.uint8)
        Y = torch.where(m, torch.zeros_like(Y), Y)  # flagged rows hold finite values
    bfm.tune_set(Y, 1, mask_mode=mm, **kw)
    one = to_numpy(bfm.fit_monitor(Y, mask_mode=mm, valid=valid, outputs=ALL, **kw))
    if lds_bytes(split, int(h * n), int(freq)) > 160 * 1024:
        # More LDS than a workgroup has: the split is refused, the tuning kept.
        with pytest.raises(bfm.BfmError) as e:
            bfm.tune_set(Y, split, mask_mode=mm, **kw)
        assert e.value.code == bfm.E_UNSUPPORTED
        return
    bfm.tune_set(Y, split, mask_mode=mm, **kw)
    g = to_numpy(bfm.fit_monitor(Y, mask_mode=mm, valid=valid, outputs=ALL, **kw))
    torch.cuda.synchronize()
    Yh = Y.float().cpu().numpy()
    vh = None if valid is None else valid.cpu().numpy()
    o = orc.fit_monitor(Yh, n=n, order=order, freq=freq, h=h, mask_mode=mm, valid=vh, threads=0)
    rep = compare(g, o, lam=2.5, n_v=used_history(Yh, n, vh))
    say("vs oracle", rep)
    assert (o["status"] == 0).mean() > 0.9
    # The split changes only the order of the history sums.
    np.testing.assert_array_equal(g["status"], one["status"])
    ok = one["status"] == 0
    np.testing.assert_allclose(g["sigma"][ok], one["sigma"][ok], rtol=1e-11)
    np.testing.assert_allclose(g["mag"][ok], one["mag"][ok], rtol=1e-9)
    bfm.tune_set(Y, 1, mask_mode=mm, **kw)


def test_masked_autotune_and_limits(bfm, orc):
    say("case masked autotune P=4096 N=228 n=114 miss=0.25")
    Y, _ = masked_series(4096, 228, 114, 3, 310, 0.25, 23.0)
    split, times = bfm.autotune(Y, n=114, mask_mode=bfm.MASK_NAN)
    say("masked autotune", split, times)
    # 114 history rows are 5 blocks of 23: splits 1, 2 and 4 fit, 8 does not.
    assert sorted(times) == [1, 2, 4] and times[split] == min(times.values())
    g = to_numpy(bfm.fit_monitor(Y, n=114, mask_mode=bfm.MASK_NAN, outputs=("brk", "mag", "sigma", "status")))
    Yh = Y.cpu().numpy()
    o = orc.fit_monitor(Yh, n=114, mask_mode=orc.MASK_NAN, threads=0)
    say("tuned vs oracle", compare(g, o, lam=2.5, n_v=used_history(Yh, 114)))
    with pytest.raises(bfm.BfmError) as e:
        bfm.tune_set(Y, 8, n=114, mask_mode=bfm.MASK_NAN)
    assert e.value.code == bfm.E_UNSUPPORTED
    with pytest.raises(bfm.BfmError) as e:
        bfm.tune_set(Y, 3, n=114, mask_mode=bfm.MASK_NAN)
    assert e.value.code == bfm.E_INVAL
    with pytest.raises(bfm.BfmError) as e:  # the general missing-value kernel has no split
        bfm.tune_set(Y, 2, n=114, freq=22.5, mask_mode=bfm.MASK_NAN)
    assert e.value.code == bfm.E_UNSUPPORTED
    with pytest.raises(bfm.BfmError) as e:  # no validity mask to time with
        bfm.autotune(Y, n=114, mask_mode=bfm.MASK_EXPLICIT)
    assert e.value.code == bfm.E_UNSUPPORTED
    bfm.tune_set(Y, 1, n=114, mask_mode=bfm.MASK_NAN)


@pytest.mark.parametrize("split", [2, 4])
def test_masked_split_bf16_storage(bfm, orc, split):
    """BF16 storage: the values decode exactly, so the FP64 bar holds."""
    say(f"case masked split={split} bf16 P=1200 N=400 n=200")
    Y, _ = masked_series(1200, 400, 200, 3, 330, 0.25, 23.0, torch.bfloat16)
    kw = dict(n=200, order=3, freq=23.0)
    bfm.tune_set(Y, split, mask_mode=bfm.MASK_NAN, **kw)
    g = to_numpy(bfm.fit_monitor(Y, mask_mode=bfm.MASK_NAN, outputs=ALL, **kw))
    bfm.tune_set(Y, 1, mask_mode=bfm.MASK_NAN, **kw)
    Yh = Y.float().cpu().numpy()
    o = orc.fit_monitor(Yh, n=200, order=3, mask_mode=orc.MASK_NAN, threads=0)
    say("bf16 vs oracle", compare(g, o, lam=2.5, n_v=used_history(Yh, 200)))


def test_masked_split_fp32_mosum(bfm, orc):
    """BFM_PREC_FP32 with a history split, at the FP32 bar against the oracle."""
    from test_gpu_fp32 import check32
    say("case masked split=4 fp32 MOSUM P=1500 N=400 n=200")
    Y, _ = masked_series(1500, 400, 200, 3, 331, 0.25, 23.0)
    kw = dict(n=200, order=3, freq=23.0)
    bfm.tune_set(Y, 4, mask_mode=bfm.MASK_NAN, **kw)
    g = to_numpy(bfm.fit_monitor(Y, mask_mode=bfm.MASK_NAN, outputs=("brk", "mag", "sigma", "status", "mosum"),
                                 precision="fp32", **kw))
    bfm.tune_set(Y, 1, mask_mode=bfm.MASK_NAN, **kw)
    Yh = Y.cpu().numpy()
    o = orc.fit_monitor(Yh, n=200, order=3, mask_mode=orc.MASK_NAN, threads=0)
    say("fp32 split vs oracle", check32(g, o, 2.5, used_history(Yh, 200)))
