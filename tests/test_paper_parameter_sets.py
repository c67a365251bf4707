"""The paper's experiment parameter sets (tests/golden/paper_parameter_sets.json):
the oracle reproduces a constructed planted step in closed form at each shape."""
import json
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SETS = json.load(open(os.path.join(HERE, "golden", "paper_parameter_sets.json")))["sets"]


def planted(orc, N, n, H, K, f, s, d, tau):
    X = np.stack([orc.design_row(t, K, f) for t in range(1, N + 1)])
    L = n + 1 - H
    z = np.random.default_rng(5).normal(size=L)
    Q, _ = np.linalg.qr(X[:L])
    e = z - Q @ (Q.T @ z)
    e *= s * math.sqrt(n - (2 + 2 * K)) / np.linalg.norm(e)
    y = X @ (np.linspace(0.4, -0.1, 2 + 2 * K) * np.r_[1, 1e-3, np.ones(2 * K)])
    y[:L] += e
    y[tau - 1:] -= d
    return y[:, None]


# The noise-free-window construction needs room for orthogonal noise before the
# first monitoring window: every shape but h = n (covered by the next test).
ROOMY = [p for p in SETS if p["n"] + 1 - p["h_window"] >= 2 + 2 * p["k"] + 2]


@pytest.mark.parametrize("ps", ROOMY, ids=[p["name"] for p in ROOMY])
def test_planted_step_at_paper_shapes(orc, ps):
    N, n, H, K, f = ps["N"], ps["n"], ps["h_window"], ps["k"], float(ps["f"])
    lam = ps.get("lambda_reported", 2.5)
    s, d = 0.02, 0.11  # lambda s sqrt(n) / d is not an integer: no tie at the boundary
    tau = n + (N - n) // 3
    r = orc.fit_monitor(planted(orc, N, n, H, K, f, s, d, tau), n=n, order=K, freq=f,
                        h_window=H, lam=lam)
    assert r["status"][0] == orc.OK
    assert abs(r["sigma"][0] - s) < 1e-10
    jstar = math.floor(lam * s * math.sqrt(n) / d) + 1
    assert r["brk"][0] == tau + jstar - n - 2
    if tau + H - 1 <= N:
        assert abs(r["mag"][0] + d * H / (s * math.sqrt(n))) < 1e-8


@pytest.mark.parametrize("ps", SETS, ids=[p["name"] for p in SETS])
def test_planted_step_with_history_noise_in_the_windows(orc, ps):
    """Every shape, including h = n (Figure 6's h = 100, where every monitoring
    window reaches back over the whole history): the noise e is orthogonal to the
    history design and spread over all n history rows, scaled so that sigma = s
    exactly, and the monitoring rows are exact fits until a step of -d at tau.
    The residuals are then known (e in the history, 0 then -d in the monitoring
    period), so MO_t is the window sum of that known vector over s sqrt(n) and
    the break index and magnitude follow from it."""
    N, n, H, K, f = ps["N"], ps["n"], ps["h_window"], ps["k"], float(ps["f"])
    lam = ps.get("lambda_reported", 2.5)
    p = 2 + 2 * K
    tau = n + (N - n) // 2
    s = 0.02
    d = 1.7 * lam * s * math.sqrt(n) / min(H, N - tau + 1)  # the step alone reaches 1.7 lambda
    X = np.stack([orc.design_row(t, K, f) for t in range(1, N + 1)])
    z = np.random.default_rng(11 + H).normal(size=n)
    Q, _ = np.linalg.qr(X[:n])
    e = z - Q @ (Q.T @ z)
    e *= s * math.sqrt(n - p) / np.linalg.norm(e)
    r = np.zeros(N)
    r[:n] = e
    r[tau - 1:] -= d
    y = X @ (np.linspace(0.4, -0.1, p) * np.r_[1, 1e-3, np.ones(2 * K)]) + r
    C = np.r_[0.0, np.cumsum(r)]
    t = np.arange(n + 1, N + 1)
    mo = (C[t] - C[t - H]) / (s * math.sqrt(n))
    assert np.abs(np.abs(mo) - lam).min() > 1e-6 * lam  # no tie at the boundary
    cross = np.nonzero(np.abs(mo) > lam)[0]
    res = orc.fit_monitor(y[:, None], n=n, order=K, freq=f, h_window=H, lam=lam)
    assert res["status"][0] == orc.OK
    assert abs(res["sigma"][0] - s) < 1e-10
    assert res["brk"][0] == (cross[0] if cross.size else -1)
    assert cross.size, "the construction should break"
    j = np.argmax(np.abs(mo))
    assert abs(res["mag"][0] - mo[j]) < 1e-8
    # f = 365 over a 144-row history leaves the harmonic columns nearly collinear
    # (condition number ~5e5), which the FP64 fit pays in the last digits
    np.testing.assert_allclose(res["mosum"][:, 0], mo, rtol=0, atol=1e-8)
