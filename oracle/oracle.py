"""Python front end of the FP64 CPU oracle (``bfm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark call this module; the GPU library never does.  It shares no
code with the GPU library: it marshals numpy arrays into the C oracle through
ctypes and nothing else.

The oracle follows the paper's Algorithm 1 (Section 2.1) pixel by pixel in FP64;
``bfm_oracle.c`` lists every equation it implements and every reading taken where
the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfm_oracle.c")
_LIB = os.path.join(_HERE, "libbfm_oracle.so")

MASK_NONE, MASK_NAN, MASK_EXPLICIT, MASK_FILL = 0, 1, 2, 3
OK, NONFINITE, INSUFFICIENT, RANK_DEFICIENT, DEGENERATE_SIGMA, NO_MONITOR = range(6)


class _Params(ctypes.Structure):
    _fields_ = [
        ("n_obs", ctypes.c_int32),
        ("n_hist", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("freq", ctypes.c_double),
        ("h_frac", ctypes.c_double),
        ("h_window", ctypes.c_int32),
        ("lambda_", ctypes.c_double),
        ("mask_mode", ctypes.c_int32),
        ("times", ctypes.c_void_p),
    ]


def build(force: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
             "-D_GNU_SOURCE", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


class Oracle:
    """The oracle library at ``lib_path`` (the built ``bfm_oracle.c`` by default)."""

    MASK_NONE, MASK_NAN, MASK_EXPLICIT, MASK_FILL = MASK_NONE, MASK_NAN, MASK_EXPLICIT, MASK_FILL
    OK, NONFINITE, INSUFFICIENT = OK, NONFINITE, INSUFFICIENT
    RANK_DEFICIENT, DEGENERATE_SIGMA, NO_MONITOR = RANK_DEFICIENT, DEGENERATE_SIGMA, NO_MONITOR

    def __init__(self, lib_path: str):
        lib = ctypes.CDLL(lib_path)
        d, i64 = ctypes.c_double, ctypes.c_int64
        vp = ctypes.c_void_p
        lib.bfo_fit_monitor.argtypes = [ctypes.POINTER(_Params), vp, i64, i64, vp, i64,
                                        vp, vp, vp, vp, vp, vp, vp, ctypes.c_int]
        lib.bfo_fit_monitor.restype = ctypes.c_int
        lib.bfo_fit_monitor_f64.argtypes = lib.bfo_fit_monitor.argtypes
        lib.bfo_fit_monitor_f64.restype = ctypes.c_int
        lib.bfo_design_row.argtypes = [d, ctypes.c_int, d, vp]
        lib.bfo_boundary.argtypes = [d, d]
        lib.bfo_boundary.restype = d
        lib.bfo_threads.argtypes = [ctypes.c_int]
        lib.bfo_threads.restype = ctypes.c_int
        self.lib = lib

    def design_row(self, t: float, order: int, freq: float) -> np.ndarray:
        """Eq. 2: x_t at time t (the 1-based index, or an observation's time)."""
        x = np.empty(2 + 2 * order, np.float64)
        self.lib.bfo_design_row(float(t), int(order), float(freq), _ptr(x))
        return x

    def boundary(self, lam: float, ratio: float) -> float:
        """Eq. 4: lambda * sqrt(log+(ratio))."""
        return self.lib.bfo_boundary(float(lam), float(ratio))

    def threads(self, nthreads: int = 0) -> int:
        return self.lib.bfo_threads(int(nthreads))

    def fit_monitor(self, Y, *, n: int, order: int = 3, freq: float = 23.0, h: float = 0.25,
                    h_window: int = 0, lam: float = 2.5, mask_mode: int = MASK_NONE,
                    valid=None, times=None, threads: int = 1, extras: bool = True) -> dict:
        """Run the oracle on a time-major series block ``Y`` of shape (N, P).

        ``Y`` is used as float32 (the library's input type) unless it is a float64
        array, in which case the FP64 entry point is used.  ``times`` (N values,
        strictly increasing) replaces the index t in the design rows of Eq. 2.

        Returns a dict of numpy arrays: ``brk`` (int32, P), ``mag``, ``sigma``
        (float64, P), ``status`` (uint8, P) and, when ``extras``, ``beta`` (p x P),
        ``resid`` (N x P) and ``mosum`` ((N-n) x P), NaN where undefined.
        """
        f64 = isinstance(Y, np.ndarray) and Y.dtype == np.float64
        Y = np.ascontiguousarray(Y, dtype=np.float64 if f64 else np.float32)
        N, P = Y.shape
        p = 2 + 2 * order
        tv = None
        if times is not None:
            tv = np.ascontiguousarray(times, dtype=np.float64)
            assert tv.shape == (N,)
        prm = _Params(N, n, order, float(freq), float(h), int(h_window), float(lam),
                      int(mask_mode), _ptr(tv))
        out = {
            "brk": np.empty(P, np.int32),
            "mag": np.empty(P, np.float64),
            "sigma": np.empty(P, np.float64),
            "status": np.empty(P, np.uint8),
        }
        if extras:
            out["beta"] = np.empty((p, P), np.float64)
            out["resid"] = np.empty((N, P), np.float64)
            out["mosum"] = np.empty((N - n, P), np.float64)
        v = None
        if valid is not None:
            v = np.ascontiguousarray(valid, dtype=np.uint8)
            assert v.shape == (N, P)
        fn = self.lib.bfo_fit_monitor_f64 if f64 else self.lib.bfo_fit_monitor
        rc = fn(ctypes.byref(prm), _ptr(Y), P, P, _ptr(v), P,
                _ptr(out["brk"]), _ptr(out["mag"]), _ptr(out["sigma"]), _ptr(out["status"]),
                _ptr(out.get("beta")), _ptr(out.get("resid")), _ptr(out.get("mosum")),
                int(threads))
        if rc != 0:
            raise ValueError("oracle rejected the parameters")
        return out


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


_default = None


def _oracle() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def design_row(t: float, order: int, freq: float) -> np.ndarray:
    """Eq. 2: x_t at time t (the 1-based index, or an observation's time)."""
    return _oracle().design_row(t, order, freq)


def boundary(lam: float, ratio: float) -> float:
    """Eq. 4: lambda * sqrt(log+(ratio))."""
    return _oracle().boundary(lam, ratio)


def threads(nthreads: int = 0) -> int:
    return _oracle().threads(nthreads)


def fit_monitor(Y, **kw) -> dict:
    """Module-level form of Oracle.fit_monitor on the built oracle."""
    return _oracle().fit_monitor(Y, **kw)
