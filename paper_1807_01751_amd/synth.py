"""Seeded synthetic satellite-like series (inputs only).

This module produces the input blocks that both the GPU library and the CPU
oracle are run on.  It holds none of the method's arithmetic (no design matrix,
no fit, no MOSUM); it only draws series of the shape the paper's experiments use:
a season-trend signal with noise, a planted level shift in a fraction of the
pixels, and optionally missing observations written as NaN.

Recipe (per pixel i, time t = 1..N; every draw seeded):
  y_t = 0.5 + 5e-4 t + sum_{j=1..K} a_ij sin(2 pi j t / f + phi_ij) + eps_it
  a_ij ~ U(0, 0.2), phi_ij ~ U(0, 2 pi), eps_it ~ N(0, 0.02^2)
  with probability ``step_frac`` the pixel gets y_t += step for t >= tau_i,
  tau_i ~ U{n+1..N} (a break inside the monitoring period).
Unevenly sampled scenes (Section 4's Landsat stack, f = 365 on day numbers):
``acquisition_days`` draws day numbers with gaps of 8-48 days, and
``make_series(..., times=days, freq=365, trend=2e-5)`` evaluates the same
recipe at those times (t replaced by the day number; the planted shift still
starts at an observation index).
Missing observations: a share ``iid`` of independent Bernoulli gaps plus cloud
runs of length U{3..15} whose starts are a Bernoulli process tuned so the runs
cover a share ``runs`` of the series.  Paper context: Section 4 builds its
artificial series from a sine plus noise with a constant added to half of them
(Eq. 12); the values above make that recipe concrete.
"""
from __future__ import annotations

import math

import torch


def _gen(device, seed):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def acquisition_days(N: int, *, seed: int = 0, start: float = 18.0):
    """Day numbers (float64 numpy array, strictly increasing) of N acquisitions:
    gaps of 8 or 16 days (two sensors' revisits) and 32 or 48 days (scenes lost
    to clouds), starting at day ``start``."""
    import numpy as np
    rng = np.random.default_rng(seed)
    gaps = rng.choice(np.array([8.0, 16.0, 16.0, 16.0, 32.0, 48.0]), N - 1)
    return start + np.concatenate([[0.0], np.cumsum(gaps)])


def make_series(P: int, N: int, n: int, order: int = 3, *, freq: float = 23.0, seed: int = 0,
                step_frac: float = 0.2, step: float = -0.3, noise: float = 0.02,
                times=None, trend: float = 5e-4, device="cpu", chunk_rows: int = 64):
    """Return (Y, truth): Y is a time-major float32 tensor of shape (N, P).

    ``truth`` holds the per-pixel draws: ``has_step`` (bool), ``tau`` (int64, the
    1-based observation index of the planted shift; meaningful where has_step).
    ``times`` (N values) replaces t = 1..N in the signal; ``trend`` is the slope
    per unit of t.
    """
    device = torch.device(device)
    g = _gen(device, seed)
    amp = torch.rand(order, P, generator=g, device=device, dtype=torch.float64) * 0.2
    phase = torch.rand(order, P, generator=g, device=device, dtype=torch.float64) * (2 * math.pi)
    has_step = torch.rand(P, generator=g, device=device) < step_frac
    tau = torch.randint(n + 1, N + 1, (P,), generator=g, device=device)
    Y = torch.empty(N, P, device=device, dtype=torch.float32)
    for t0 in range(0, N, chunk_rows):
        t1 = min(N, t0 + chunk_rows)
        t = torch.arange(t0 + 1, t1 + 1, device=device, dtype=torch.float64)[:, None]
        tv = t if times is None else torch.as_tensor(times[t0:t1], dtype=torch.float64,
                                                     device=device)[:, None]
        y = 0.5 + trend * tv + torch.zeros(t1 - t0, P, device=device, dtype=torch.float64)
        for j in range(order):
            y += amp[j] * torch.sin(2 * math.pi * (j + 1) * tv / freq + phase[j])
        y += noise * torch.randn(t1 - t0, P, generator=g, device=device, dtype=torch.float64)
        y += step * (has_step & (t >= tau)).to(torch.float64)
        Y[t0:t1] = y.to(torch.float32)
    return Y, {"has_step": has_step, "tau": tau}


def make_missing(N: int, P: int, *, iid: float = 0.0, runs: float = 0.0, seed: int = 1,
                 device="cpu", run_min: int = 3, run_max: int = 15):
    """Return a (N, P) bool tensor, True where the observation is missing."""
    device = torch.device(device)
    g = _gen(device, seed)
    miss = torch.rand(N, P, generator=g, device=device) < iid
    if runs > 0:
        mean_len = 0.5 * (run_min + run_max)
        q = -math.log(1.0 - runs) / mean_len
        starts = torch.rand(N, P, generator=g, device=device) < q
        lens = torch.randint(run_min, run_max + 1, (N, P), generator=g, device=device)
        for d in range(run_max):
            hit = starts[: N - d] & (lens[: N - d] > d)
            miss[d:] |= hit
    return miss


def apply_missing(Y: torch.Tensor, miss: torch.Tensor) -> torch.Tensor:
    """Write NaN where ``miss`` is True (in place) and return Y."""
    Y.masked_fill_(miss, float("nan"))
    return Y


def split_rate(total: float) -> float:
    """Per-mechanism rate so iid gaps and runs of equal rate miss ``total`` overall."""
    return 1.0 - math.sqrt(1.0 - total)
