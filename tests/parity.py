"""Parity rules between the GPU library and the FP64 oracle (test helper).

Bars (FP64 arithmetic on both sides):
  - residuals and MOSUM: per-pixel normwise relative error
    ||gpu - orc||_inf / ||orc||_inf <= 1e-9;
  - sigma and the magnitude: elementwise relative error <= 1e-9;
  - status: identical;
  - break index: identical, except on "marginal" pixels whose MOSUM comes within
    a relative margin EPS_MARGIN of the boundary at a monitoring position up to
    the later of the two break indices (there rounding may legitimately decide
    the crossing); marginal pixels are counted and reported.

Every OK pixel is compared on every quantity, marginal ones included: a
different break index changes neither sigma nor the MOSUM nor its extreme.
"""
import numpy as np

RTOL = 1e-9
EPS_MARGIN = 1e-8


def _rel_norm(a, b):
    den = np.nanmax(np.abs(b), axis=0)
    num = np.nanmax(np.abs(a - b), axis=0)
    den = np.where(den > 0, den, 1.0)
    return num / den


def boundary_at(mosum, lam, n_v):
    """Eq. 4 at every monitoring position of every pixel: lambda sqrt(log+(u/n_v))
    with u the 1-based position of the observation among the pixel's used ones
    (u = t for a complete series, n_v = n).  NaN where MO is not defined."""
    fin = np.isfinite(mosum)
    u = n_v[None, :] + np.cumsum(fin, axis=0)
    x = u / n_v[None, :]
    b = lam * np.sqrt(np.where(x <= np.e, 1.0, np.log(np.maximum(x, 1.0))))
    return np.where(fin, b, np.nan)


def margins(mosum, brk_a, brk_b, *, bnd=None, lam=None, n_v=None):
    """Smallest relative distance ||MO| - b| / b over the monitoring positions up
    to the later of the two break indices (every position if neither breaks).

    The boundary is ``bnd`` (one value per monitoring time, complete series) or
    Eq. 4 at compacted positions from ``lam`` and the used history counts
    ``n_v`` (one per pixel)."""
    M, P = mosum.shape
    if bnd is not None:
        b = np.broadcast_to(np.asarray(bnd, np.float64)[:, None], (M, P))
    else:
        b = boundary_at(mosum, lam, np.asarray(n_v, np.float64))
    with np.errstate(invalid="ignore"):
        rel = np.abs(np.abs(mosum) - b) / b
    last = np.maximum(brk_a, brk_b)
    last = np.where(last < 0, M - 1, last)
    idx = np.arange(M)[:, None]
    rel = np.where((idx <= last[None, :]) & np.isfinite(rel), rel, np.inf)
    return rel.min(axis=0)


def compare(g: dict, o: dict, *, bnd=None, lam=None, n_v=None, rtol=RTOL, eps=EPS_MARGIN,
            beta_rtol=1e-7):
    """Assert parity of GPU results ``g`` with oracle results ``o`` (numpy dicts).

    Returns a report dict.  When break indices differ, the oracle's MOSUM
    (``o["mosum"]``) and a boundary (``bnd``, or ``lam`` with the used history
    counts ``n_v`` of every pixel, as for missing-value runs) decide whether
    each such pixel is marginal; a non-marginal one fails.
    """
    rep = {}
    st_g, st_o = g["status"], o["status"]
    np.testing.assert_array_equal(st_g, st_o)
    ok = st_o == 0
    rep["pixels"] = int(st_o.size)
    rep["not_ok"] = int((~ok).sum())
    for k in ("sigma", "mag"):
        if k in g:
            a, b = g[k][ok], o[k][ok]
            err = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
            rep[f"max_rel_{k}"] = float(err.max()) if err.size else 0.0
            rep[f"p999_rel_{k}"] = float(np.quantile(err, 0.999)) if err.size else 0.0
            assert rep[f"max_rel_{k}"] <= rtol, (k, rep)
    for k in ("resid", "mosum"):
        if k in g:
            a, b = g[k][:, ok], o[k][:, ok]
            np.testing.assert_array_equal(np.isnan(a), np.isnan(b))
            err = _rel_norm(a, b)
            rep[f"max_rel_{k}"] = float(err.max()) if err.size else 0.0
            rep[f"p999_rel_{k}"] = float(np.quantile(err, 0.999)) if err.size else 0.0
            assert rep[f"max_rel_{k}"] <= rtol, (k, rep)
    if "beta" in g:
        a, b = g["beta"][:, ok], o["beta"][:, ok]
        err = _rel_norm(a, b)
        rep["max_rel_beta"] = float(err.max()) if err.size else 0.0
        assert rep["max_rel_beta"] <= beta_rtol, rep
    diff = g["brk"] != o["brk"]
    rep["brk_mismatch"] = int(diff.sum())
    rep["brk_agree"] = float(1.0 - diff.mean()) if diff.size else 1.0
    rep["marginal"] = 0
    if diff.any():
        assert "mosum" in o, "break indices differ and the oracle run has no MOSUM to judge margins"
        assert bnd is not None or lam is not None, "break indices differ and no boundary was given"
        nv = None
        if bnd is None:
            assert n_v is not None, "lam given without the used history counts n_v"
            nv = np.asarray(n_v)[diff]
        m = margins(o["mosum"][:, diff], g["brk"][diff], o["brk"][diff], bnd=bnd, lam=lam, n_v=nv)
        rep["marginal"] = int((m < eps).sum())
        rep["max_margin_of_mismatch"] = float(m.max())
        assert (m < eps).all(), ("break index differs on a non-marginal pixel", rep, m)
    return rep


def used_history(Y, n, valid=None):
    """Used observations of each pixel's history (numpy (N, P) series, optional
    validity flags): finite values among the first n rows, and flagged ones under
    an explicit mask."""
    h = np.asarray(Y[:n])
    ok = np.isfinite(h) if valid is None else (np.asarray(valid[:n]) != 0)
    return ok.sum(0)


def to_numpy(d: dict) -> dict:
    return {k: v.detach().cpu().numpy() for k, v in d.items()}
