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


@pytest.mark.parametrize("ps", SETS, ids=[p["name"] for p in SETS])
def test_planted_step_at_paper_shapes(orc, ps):
    N, n, H, K, f = ps["N"], ps["n"], ps["h_window"], ps["k"], float(ps["f"])
    lam = ps.get("lambda_reported", 2.5)
    s, d = 0.02, 0.11  # lambda s sqrt(n) / d is not an integer: no tie at the boundary
    tau = n + (N - n) // 3
    if n + 1 - H < 2 + 2 * K + 2:
        pytest.skip("window too long to plant the orthogonal noise before it")
    r = orc.fit_monitor(planted(orc, N, n, H, K, f, s, d, tau), n=n, order=K, freq=f,
                        h_window=H, lam=lam)
    assert r["status"][0] == orc.OK
    assert abs(r["sigma"][0] - s) < 1e-10
    jstar = math.floor(lam * s * math.sqrt(n) / d) + 1
    assert r["brk"][0] == tau + jstar - n - 2
    if tau + H - 1 <= N:
        assert abs(r["mag"][0] + d * H / (s * math.sqrt(n))) < 1e-8
