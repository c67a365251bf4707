"""GPU parity: libbfm (through its C ABI) against the FP64 CPU oracle.

Every case prints its name, seed and shape before touching the device.
"""
import math
import sys

import numpy as np
import pytest
import torch

from parity import compare, to_numpy

pytestmark = pytest.mark.gpu

ALL = ("brk", "mag", "sigma", "status", "beta", "resid", "mosum")


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


def run_both(bfm, orc, Y, *, n, order=3, freq=23.0, h=0.25, h_window=0, lam=2.5,
             outputs=ALL, out_dtype=torch.float64, **kw):
    g = bfm.fit_monitor(Y, n=n, order=order, freq=freq, h=h, h_window=h_window, lam=lam,
                        outputs=outputs, out_dtype=out_dtype, **kw)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy() if Y.stride(1) == 1 else Y.t().cpu().numpy()
    o = orc.fit_monitor(Yh, n=n, order=order, freq=freq, h=h, h_window=h_window, lam=lam,
                        threads=0)
    return to_numpy(g), o


def series(P, N, n, order=3, seed=0, **kw):
    from paper_1807_01751_amd.synth import make_series
    Y, _ = make_series(P, N, n, order, seed=seed, device="cuda", **kw)
    return Y


def test_config1_latency_tile_full_parity(bfm, orc):
    """64x64 pixels, N=228, n=114, k=3 (p=8), h=0.25, lambda=2.5, 20% steps."""
    say("case config1 seed=1 P=4096 N=228 n=114")
    Y = series(4096, 228, 114, seed=1)
    g, o = run_both(bfm, orc, Y, n=114)
    rep = compare(g, o, bnd=bnd_of(228, 114, 2.5))
    say("config1", rep)
    assert rep["not_ok"] == 0
    assert (o["brk"] >= 0).mean() > 0.15  # the planted steps are found


def test_lean_and_export_kernels_agree_bitwise(bfm):
    """The same kernel with and without per-row exports (the time split, which
    only lean calls take, is pinned to one wave so both run the same kernel)."""
    say("case lean-vs-export seed=2 P=3000 N=228")
    Y = series(3000, 228, 114, seed=2)
    bfm.tune_set(Y, 1, n=114)
    a = to_numpy(bfm.fit_monitor(Y, n=114, outputs=("brk", "mag", "sigma", "status")))
    b = to_numpy(bfm.fit_monitor(Y, n=114, outputs=ALL))
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("P,N,n,order,h,hw,lam,freq", [
    (1, 40, 20, 1, 0.5, 0, 2.5, 23.0),          # one pixel
    (63, 100, 50, 3, 0.25, 0, 2.5, 23.0),       # less than a wave
    (65, 101, 57, 2, 0.3, 0, 2.0, 23.0),        # ragged wave, odd lengths
    (1000, 400, 100, 3, 0.25, 0, 2.5, 23.0),    # N/n = 4 > e: log boundary
    (777, 228, 114, 0, 0.25, 0, 2.5, 23.0),     # k = 0: intercept + trend
    (500, 300, 150, 8, 0.25, 0, 2.5, 23.0),     # k = 8 (p = 18, largest)
    (300, 200, 100, 3, 0.0, 1, 2.5, 23.0),      # window of one observation
    (300, 200, 100, 3, 0.0, 100, 2.5, 23.0),    # window = whole history
    (257, 288, 144, 3, 0.0, 72, 2.39, 365.0),   # Chile-shaped parameters
    (129, 200, 100, 3, 0.5, 0, 2.5, 23.0),      # the paper's artificial workload shape
    (64, 37, 20, 2, 0.25, 0, 2.5, 23.0),        # fewer rows than one prefetch chunk
])
def test_shapes_and_parameters(bfm, orc, P, N, n, order, h, hw, lam, freq):
    say(f"case shapes P={P} N={N} n={n} k={order} h={h} hw={hw} lam={lam} f={freq}")
    Y = series(P, N, n, order=min(order, 3) if order else 1, seed=P + N)
    g, o = run_both(bfm, orc, Y, n=n, order=order, h=h if h else 0.25, h_window=hw, lam=lam,
                    freq=freq)
    rep = compare(g, o, bnd=bnd_of(N, n, lam))
    say(rep)


def test_strided_and_transposed_layouts(bfm, orc):
    say("case layout seed=3 P=500 ld=640 N=150")
    N, n, P = 150, 75, 500
    big = series(640, N, n, seed=3)
    Y = big[:, :P]  # ld = 640
    assert Y.stride() == (640, 1)
    g, o = run_both(bfm, orc, Y, n=n)
    compare(g, o, bnd=bnd_of(N, n, 2.5))
    gt = to_numpy(bfm.fit_monitor(Y.t(), n=n, outputs=ALL))  # the (P, N) view
    for k in g:
        np.testing.assert_array_equal(gt[k], g[k])


def test_float32_outputs(bfm, orc):
    say("case out_dtype=f32 seed=4 P=1000 N=228")
    Y = series(1000, 228, 114, seed=4)
    g = to_numpy(bfm.fit_monitor(Y, n=114, outputs=ALL, out_dtype=torch.float32))
    o = orc.fit_monitor(Y.cpu().numpy(), n=114, threads=0)
    ok = o["status"] == 0
    np.testing.assert_array_equal(g["status"], o["status"])
    np.testing.assert_allclose(g["mag"][ok], o["mag"][ok], rtol=2e-7)
    np.testing.assert_allclose(g["sigma"][ok], o["sigma"][ok], rtol=2e-7)
    np.testing.assert_allclose(g["mosum"][:, ok], o["mosum"][:, ok], rtol=2e-6, atol=2e-7)


def test_degenerate_pixels(bfm, orc):
    say("case degenerate P=256 N=120 n=60")
    N, n, P = 120, 60, 256
    Y = series(P, N, n, seed=5)
    t = torch.arange(1, N + 1, device="cuda", dtype=torch.float32)
    Y[:, 0] = 0.5 + t * 2.0 ** -10          # exact trend: sigma = 0
    Y[:, 1] = 0.25                           # constant
    Y[7, 2] = float("nan")                   # NaN in history
    Y[100, 3] = float("inf")                 # Inf in the monitoring period
    Y[0, 4] = float("nan")                   # the first observation
    Y[n - 1, 5] = -float("inf")              # last history row (also in the first window)
    Y[N - 1, 6] = float("nan")               # last row
    Y[:, 7] = 1e30                           # huge but finite
    g, o = run_both(bfm, orc, Y, n=n)
    assert g["status"][0] == 4 and g["status"][1] == 4
    assert (g["status"][2:7] == 1).all()
    assert (g["brk"][:7] == -1).all() and np.isnan(g["mag"][:7]).all()
    compare(g, o, bnd=bnd_of(N, n, 2.5))


def test_parameter_sets_that_leave_nothing_to_fit(bfm, orc):
    say("case global-degenerate")
    Y = series(100, 40, 8, seed=6)
    Y[3, 5] = float("nan")
    # n = 8 <= p = 8 (k = 3): every pixel INSUFFICIENT, NaN pixel NONFINITE
    g, o = run_both(bfm, orc, Y, n=8, order=3)
    np.testing.assert_array_equal(g["status"], o["status"])
    assert g["status"][5] == 1 and (np.delete(g["status"], 5) == 2).all()
    assert (g["brk"] == -1).all() and np.isnan(g["mag"]).all()
    # f = 2 with k = 1: sin(pi t) vanishes, the shared design is rank deficient
    Y = series(100, 40, 20, seed=7)
    g, o = run_both(bfm, orc, Y, n=20, order=1, freq=2.0)
    np.testing.assert_array_equal(g["status"], o["status"])
    assert (g["status"] == 3).all()
    # h * n < 1: window of zero observations
    g, o = run_both(bfm, orc, Y, n=20, order=1, h=0.04)
    assert (g["status"] == 2).all() and (o["status"] == 2).all()


def test_empty_input(bfm):
    say("case P=0")
    Y = torch.empty(50, 0, device="cuda")
    r = bfm.fit_monitor(Y, n=25)
    torch.cuda.synchronize()
    assert r["brk"].numel() == 0


def test_errors_are_reported(bfm):
    say("case errors")
    Y = series(10, 50, 25, seed=8)
    with pytest.raises(bfm.BfmError) as e:
        bfm.fit_monitor(Y, n=50)
    assert e.value.code == bfm.E_INVAL
    with pytest.raises(bfm.BfmError):
        bfm.fit_monitor(Y, n=25, lam=-1.0)
    with pytest.raises(ValueError):
        bfm.fit_monitor(Y.double(), n=25)


def test_planted_step_closed_form_on_gpu(bfm):
    """Constructed input: sigma = s exactly, known break index and magnitude."""
    say("case planted-closed-form")
    from oracle import oracle as orc_mod
    N, n, H, K, s, d, tau = 228, 114, 28, 3, 0.02, 0.3, 150
    X = np.stack([orc_mod.design_row(t, K, 23.0) for t in range(1, N + 1)])
    L = n + 1 - H
    z = np.random.default_rng(11).normal(size=L)
    Q, _ = np.linalg.qr(X[:L])
    e = z - Q @ (Q.T @ z)
    e *= s * math.sqrt(n - 8) / np.linalg.norm(e)
    y = X @ np.r_[0.5, 5e-4, 0.1, -0.05, 0.02, 0.07, -0.03, 0.01]
    y[:L] += e
    y[tau - 1:] -= d
    Y = torch.tensor(y, dtype=torch.float32, device="cuda")[:, None].repeat(1, 64).contiguous()
    g = to_numpy(bfm.fit_monitor(Y, n=n, h_window=H, outputs=ALL))
    jstar = math.floor(2.5 * s * math.sqrt(n) / d) + 1
    # FP32 rounding of y perturbs sigma slightly; the break index is far from marginal
    assert (g["brk"] == tau + jstar - n - 2).all()
    np.testing.assert_allclose(g["mag"], -d * H / (s * math.sqrt(n)), rtol=1e-4)
    np.testing.assert_allclose(g["sigma"], s, rtol=1e-4)


def test_pixel_permutation_equivariance_and_determinism(bfm):
    say("case permutation seed=9 P=5000")
    Y = series(5000, 228, 114, seed=9)
    perm = torch.randperm(5000, generator=torch.Generator().manual_seed(0)).cuda()
    a = to_numpy(bfm.fit_monitor(Y, n=114, outputs=("brk", "mag", "sigma", "status")))
    b = to_numpy(bfm.fit_monitor(Y[:, perm].contiguous(), n=114,
                                 outputs=("brk", "mag", "sigma", "status")))
    c = to_numpy(bfm.fit_monitor(Y, n=114, outputs=("brk", "mag", "sigma", "status")))
    pn = perm.cpu().numpy()
    for k in a:
        np.testing.assert_array_equal(b[k], a[k][pn])
        np.testing.assert_array_equal(c[k], a[k])


def test_config2_full_size_sampled(bfm, orc):
    """1024x1024 pixels, N=400, n=200, p=8, h=0.25, lambda=2.5: the benchmark launch.

    The whole tile runs in the lean kernel exactly as timed; 8192 sampled pixels
    (first, last and random) are checked against the oracle one by one.
    """
    say("case config2 seed=2 P=1048576 N=400 n=200")
    P, N, n = 1 << 20, 400, 200
    Y = series(P, N, n, seed=2)
    g = to_numpy(bfm.fit_monitor(Y, n=n, outputs=("brk", "mag", "sigma", "status")))
    rng = np.random.default_rng(0)
    idx = np.unique(np.r_[np.arange(64), np.arange(P - 64, P), rng.integers(0, P, 8064)])
    Ys = Y[:, torch.as_tensor(idx, device="cuda")].cpu().numpy()
    o = orc.fit_monitor(Ys, n=n, threads=0)
    gs = {k: v[idx] for k, v in g.items()}
    rep = compare(gs, o, bnd=bnd_of(N, n, 2.5))
    say("config2 sample", rep)
    assert rep["not_ok"] == 0
    brk_rate = (g["brk"] >= 0).mean()
    say("config2 break rate", brk_rate)
    assert 0.15 < brk_rate < 0.35


def test_window_longer_than_the_periodic_workgroup_lds(bfm, orc):
    """f = 23 with H = 180 rows: the period-blocked kernel's workgroup would need
    180 KB of LDS for its window rings, so the table-driven kernel serves it."""
    say("case long window P=3000 N=800 n=400 H=180")
    Y = series(3000, 800, 400, seed=41)
    g = to_numpy(bfm.fit_monitor(Y, n=400, h=0.45, outputs=ALL))
    o = orc.fit_monitor(Y.cpu().numpy(), n=400, h=0.45, threads=0)
    rep = compare(g, o, bnd=bnd_of(800, 400, 2.5))
    say(rep)
    assert rep["not_ok"] == 0
    with pytest.raises(bfm.BfmError) as e:
        bfm.fit_monitor(Y.to(torch.float16), n=400, h=0.45)
    assert e.value.code == bfm.E_UNSUPPORTED
