"""Parity rules between the GPU library and the FP64 oracle (test helper).

Bars (FP64 arithmetic on both sides):
  - residuals and MOSUM: per-pixel normwise relative error
    ||gpu - orc||_inf / ||orc||_inf <= 1e-9;
  - sigma and the magnitude: elementwise relative error <= 1e-9;
  - status: identical;
  - break index: identical, except on "marginal" pixels whose MOSUM comes within
    a relative margin EPS_MARGIN of the boundary at a time up to the later of the
    two break indices (there rounding may legitimately decide the crossing);
    marginal pixels are counted and reported.
"""
import numpy as np

RTOL = 1e-9
EPS_MARGIN = 1e-8


def _rel_norm(a, b):
    den = np.nanmax(np.abs(b), axis=0)
    num = np.nanmax(np.abs(a - b), axis=0)
    den = np.where(den > 0, den, 1.0)
    return num / den


def margins(mosum, bnd, brk_a, brk_b):
    """Smallest relative distance of |MO| to the boundary up to the later break."""
    M, P = mosum.shape
    rel = np.abs(np.abs(mosum) - bnd[:, None]) / bnd[:, None]
    last = np.maximum(brk_a, brk_b)
    last = np.where(last < 0, M - 1, last)
    idx = np.arange(M)[:, None]
    rel = np.where((idx <= last[None, :]) & np.isfinite(rel), rel, np.inf)
    return rel.min(axis=0)


def compare(g: dict, o: dict, *, bnd=None, rtol=RTOL, eps=EPS_MARGIN):
    """Assert parity of GPU results ``g`` with oracle results ``o`` (numpy dicts).

    Returns a report dict.  ``bnd`` (the boundary per monitoring time) is needed
    to classify marginal pixels when break indices differ.
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
        assert rep["max_rel_beta"] <= 1e-7, rep
    diff = g["brk"] != o["brk"]
    rep["brk_mismatch"] = int(diff.sum())
    rep["marginal"] = 0
    if diff.any():
        assert bnd is not None and "mosum" in o, "break indices differ and no MOSUM to judge margins"
        m = margins(o["mosum"][:, diff], np.asarray(bnd), g["brk"][diff], o["brk"][diff])
        rep["marginal"] = int((m < eps).sum())
        assert (m < eps).all(), ("break index differs on a non-marginal pixel", rep, m)
    return rep


def to_numpy(d: dict) -> dict:
    return {k: v.detach().cpu().numpy() for k, v in d.items()}
