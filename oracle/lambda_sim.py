"""Critical value lambda of the boundary (Eq. 4) by simulation: plain numpy
oracle.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the GPU library never does, and it shares
no code with it.

Section 2.1 chooses lambda so that, when nothing changes, the MOSUM crosses
the boundary lambda sqrt(log+(t/n)) with probability alpha; lambda depends on
alpha, the window h and the horizon N/n and is found by simulation, following
the method the paper cites for it.  This module simulates the MOSUM of Eq. 3
under no change at the resolution of the series, with i.i.d. standard normal
errors z_1..z_N and the intercept-only model:

    M_k = ( sum_{i=k-H+1..k} z_i  -  (H/n) sum_{i=1..n} z_i ) / sqrt(n),
    S   = max_{k=n+1..N} |M_k| / sqrt(log+(k/n)),

and a path crosses lambda sqrt(log+(k/n)) iff S > lambda.  lambda is the
ceil((1 - alpha) * paths)-th smallest S: at most a share alpha of the paths
cross it.

What this lambda is: M is the intercept model's residual MOSUM, whose limit
(t in units of the history length) is W(t) - W(t-h) - h W(1) for a standard
Brownian motion W.  The cited method takes its critical values from that
limiting process, which is also the limit for regressors with a stable
second-moment matrix.  The season-trend model of Eq. 2 is not such a model:
the error of the fitted slope, extrapolated over the monitoring period, adds a
term of order one to its residual MOSUM's limit.  So lambda here is the
method's convention, not an exact level-alpha critical value for Eq. 2.  The
discrete sup over n steps per unit of time falls short of the continuous one
by about 0.5826 sqrt(2/n) (Siegmund's correction for a random walk whose steps
have variance 2/n); with that correction the simulated lambda for alpha =
0.05, h = 1/2, N/n = 2 agrees with the value 2.39 printed in Section 4.3.

Random numbers: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011) with key (seed, 0) and counter
(j, path, 0, 0) gives four 64-bit words per block j; each word w becomes a
uniform u = ((w >> 11) + 1/2) 2^-53 in (0, 1), and the Box-Muller transform turns
(u0, u1) and (u2, u3) into z_{4j+1}, z_{4j+2} = r cos(2 pi u1), r sin(2 pi u1)
with r = sqrt(-2 ln u0), and z_{4j+3}, z_{4j+4} likewise from (u2, u3).
"""
from __future__ import annotations

import math

import numpy as np

M0, M1 = np.uint64(0xD2E7470EE14C6C93), np.uint64(0xCA5A826395121157)  # round multipliers
W0, W1 = np.uint64(0x9E3779B97F4A7C15), np.uint64(0xBB67AE8584CAA73B)  # key increments
_LO = np.uint64(0xFFFFFFFF)
_32 = np.uint64(32)


def _mulhilo(a, b):
    """High and low 64-bit halves of the 128-bit product a * b (uint64 arrays)."""
    a = np.asarray(a, np.uint64)
    b = np.asarray(b, np.uint64)
    a0, a1 = a & _LO, a >> _32
    b0, b1 = b & _LO, b >> _32
    with np.errstate(over="ignore"):
        lo = a * b
        p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
        mid = (p00 >> _32) + (p01 & _LO) + (p10 & _LO)
        hi = p11 + (p01 >> _32) + (p10 >> _32) + (mid >> _32)
    return hi, lo


def philox4x64(counter, key):
    """Philox4x64-10 of the counter words (four uint64 arrays) under the key
    (two uint64 scalars): ten rounds, the key bumped by the Weyl constants
    between rounds.  Returns four uint64 arrays."""
    c = [np.asarray(x, np.uint64) for x in counter]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    for r in range(10):
        if r:
            with np.errstate(over="ignore"):
                k0, k1 = k0 + W0, k1 + W1
        hi0, lo0 = _mulhilo(M0, c[0])
        hi1, lo1 = _mulhilo(M1, c[2])
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def normals(seed: int, paths, count: int) -> np.ndarray:
    """Standard normals z_1..z_count of each path index in ``paths``: an array
    of shape (count, len(paths))."""
    paths = np.asarray(paths, np.uint64)
    nb = (count + 3) // 4
    j = np.repeat(np.arange(nb, dtype=np.uint64)[:, None], len(paths), axis=1)
    p = np.broadcast_to(paths[None, :], j.shape)
    zero = np.zeros_like(j)
    w = philox4x64([j, p, zero, zero], (np.uint64(seed), np.uint64(0)))
    u = [((x >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53 for x in w]
    r0 = np.sqrt(-2.0 * np.log(u[0]))
    r2 = np.sqrt(-2.0 * np.log(u[2]))
    z = np.stack([r0 * np.cos(2 * np.pi * u[1]), r0 * np.sin(2 * np.pi * u[1]),
                  r2 * np.cos(2 * np.pi * u[3]), r2 * np.sin(2 * np.pi * u[3])], axis=1)
    return z.reshape(4 * nb, len(paths))[:count]


def mosum_of_normals(n: int, N: int, H: int, z) -> np.ndarray:
    """M_k for k = n+1..N (rows) of each path (column of ``z``, the normals
    z_1..z_N of the path in its rows), by the definition: window sums of z
    minus (H/n) times the history sum, over sqrt(n)."""
    z = np.asarray(z, np.float64)
    C = np.vstack([np.zeros((1, z.shape[1])), np.cumsum(z, axis=0)])  # C[k] = z_1 + .. + z_k
    k = np.arange(n + 1, N + 1)
    return (C[k] - C[k - H] - (H / n) * C[n]) / math.sqrt(n)


def sup_of_normals(n: int, N: int, H: int, z) -> np.ndarray:
    """S = max_k |M_k| / sqrt(log+(k/n)) of each path (column of ``z``)."""
    M = mosum_of_normals(n, N, H, z)
    t = np.arange(n + 1, N + 1) / n
    b = np.sqrt(np.where(t <= math.e, 1.0, np.log(np.maximum(t, 1.0))))
    return (np.abs(M) / b[:, None]).max(axis=0)


def mosum_paths(n: int, N: int, H: int, seed: int, paths) -> np.ndarray:
    """M_k for k = n+1..N (rows) of each path index (columns), on the normals
    of the counter-based generator above."""
    return mosum_of_normals(n, N, H, normals(seed, paths, N))


def sup_statistic(n: int, N: int, H: int, seed: int, paths) -> np.ndarray:
    """S = max_k |M_k| / sqrt(log+(k/n)) per path index."""
    return sup_of_normals(n, N, H, normals(seed, paths, N))


def quantile_rank(alpha: float, paths: int) -> int:
    """1-based rank of lambda among the sorted S: ceil((1 - alpha) paths)."""
    return max(1, min(paths, math.ceil((1.0 - alpha) * paths - 1e-9)))


def critical_value(alpha: float, n: int, N: int, H: int, paths: int, seed: int = 0,
                   chunk: int = 4096) -> float:
    """lambda for (alpha, h = H/n, N/n) from ``paths`` simulated paths."""
    S = np.concatenate([sup_statistic(n, N, H, seed, np.arange(a, min(paths, a + chunk)))
                        for a in range(0, paths, chunk)])
    return float(np.sort(S)[quantile_rank(alpha, paths) - 1])
