"""Python binding of libbfm (include/bfm.h): argument marshalling only.

Every step of BFAST Monitor runs in the HIP kernels of ``libbfm.so``; this
module passes torch tensors' device pointers and the current HIP stream through
ctypes.  PyTorch provides device memory and streams, nothing else.  If the
shared library is missing the import of the functions below fails loudly: there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbfm.so")

# include/bfm.h constants
SUCCESS = 0
E_INVAL, E_LAYOUT, E_NOMEM, E_NODEVICE, E_HIP, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6
MASK_NONE, MASK_NAN, MASK_EXPLICIT, MASK_FILL = 0, 1, 2, 3
NOALLOC_MAX_PATHS = 4194304  # BFM_NOALLOC_MAX_PATHS
PREC_FP64, PREC_FP32 = 0, 1
_PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32}
Y_F32, Y_BF16, Y_F16 = 0, 1, 2
_Y_DTYPES = {torch.float32: Y_F32, torch.bfloat16: Y_BF16, torch.float16: Y_F16}
OUT_F32, OUT_F64 = 0, 1
ST_OK, ST_NONFINITE, ST_INSUFFICIENT, ST_RANK_DEFICIENT, ST_DEGENERATE_SIGMA, ST_NO_MONITOR = range(6)

_ERRNAMES = {E_INVAL: "BFM_E_INVAL", E_LAYOUT: "BFM_E_LAYOUT", E_NOMEM: "BFM_E_NOMEM",
             E_NODEVICE: "BFM_E_NODEVICE", E_HIP: "BFM_E_HIP", E_UNSUPPORTED: "BFM_E_UNSUPPORTED"}

# Every symbol include/bfm.h declares.
EXPORTS = ("bfm_version", "bfm_last_error", "bfm_check_params", "bfm_create", "bfm_destroy",
           "bfm_fit_monitor", "bfm_fit_monitor_typed", "bfm_host_operators", "bfm_request_bytes",
           "bfm_server_create", "bfm_server_submit", "bfm_server_wait", "bfm_server_release",
           "bfm_server_take", "bfm_autotune", "bfm_tune_set", "bfm_mosum_null_sup",
           "bfm_critical_value", "bfm_critical_value_noalloc", "bfm_workspace_bytes",
           "bfm_server_get_stats", "bfm_server_destroy", "bfm_operator_budget", "bfm_cache_get_stats",
           "bfm_server_operator_budget")
WANT = {"mag": 1, "sigma": 2, "status": 4, "beta": 8, "resid": 16, "mosum": 32}


class BfmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("n_obs", ctypes.c_int32),
        ("n_hist", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("h_window", ctypes.c_int32),
        ("freq", ctypes.c_double),
        ("h_frac", ctypes.c_double),
        ("lambda_", ctypes.c_double),
        ("mask_mode", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("times", ctypes.c_void_p),
    ]


class Outputs(ctypes.Structure):
    _fields_ = [
        ("brk", ctypes.c_void_p),
        ("mag", ctypes.c_void_p),
        ("sigma", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("beta", ctypes.c_void_p),
        ("resid", ctypes.c_void_p),
        ("mosum", ctypes.c_void_p),
        ("out_dtype", ctypes.c_int32),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("prm", Params),
        ("Y", ctypes.c_void_p),
        ("y_dtype", ctypes.c_int32),
        ("P", ctypes.c_int64),
        ("ld", ctypes.c_int64),
        ("valid", ctypes.c_void_p),
        ("ldv", ctypes.c_int64),
        ("outputs", ctypes.c_uint32),
        ("out_dtype", ctypes.c_int32),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("rc", ctypes.c_int32),
        ("out", Outputs),
        ("queued_us", ctypes.c_double),
        ("latency_us", ctypes.c_double),
        ("device_us", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("queued", "running", "completed", "pool_in_use",
                                             "max_running", "operator_entries", "operator_bytes",
                                             "operator_evictions", "operator_waits")]


class CacheStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("entries", "bytes", "budget", "evictions")]


_lib = None
_lock = threading.Lock()
_ctx = {}


def load():
    """Load libbfm.so (built by ``python -m paper_1807_01751_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1807_01751_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    P_ = ctypes.POINTER(Params)
    lib.bfm_version.restype = ctypes.c_int
    lib.bfm_last_error.restype = ctypes.c_char_p
    lib.bfm_check_params.argtypes = [P_, i64, i64]
    lib.bfm_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.bfm_destroy.argtypes = [vp]
    lib.bfm_fit_monitor.argtypes = [vp, P_, vp, i64, i64, vp, i64, ctypes.POINTER(Outputs), vp]
    lib.bfm_fit_monitor_typed.argtypes = [vp, P_, vp, ctypes.c_int32, i64, i64, vp, i64,
                                          ctypes.POINTER(Outputs), vp]
    lib.bfm_host_operators.argtypes = [P_, vp, vp, vp, vp]
    lib.bfm_autotune.argtypes = [vp, P_, vp, ctypes.c_int32, i64, i64, vp, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_double)]
    lib.bfm_tune_set.argtypes = [vp, P_, ctypes.c_int32, i64, ctypes.c_int32]
    lib.bfm_mosum_null_sup.argtypes = [vp, P_, ctypes.c_uint64, i64, i64, vp, vp]
    lib.bfm_workspace_bytes.argtypes = [P_, i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.bfm_critical_value.argtypes = [vp, P_, ctypes.c_double, i64, ctypes.c_uint64,
                                       ctypes.POINTER(ctypes.c_double), vp]
    lib.bfm_critical_value_noalloc.argtypes = lib.bfm_critical_value.argtypes
    R_ = ctypes.POINTER(Request)
    lib.bfm_request_bytes.argtypes = [R_, ctypes.POINTER(ctypes.c_size_t)]
    lib.bfm_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_size_t]
    lib.bfm_server_submit.argtypes = [vp, R_, ctypes.POINTER(ctypes.c_uint64)]
    lib.bfm_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(Result)]
    lib.bfm_server_release.argtypes = [vp, ctypes.c_uint64]
    lib.bfm_server_take.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(Outputs), vp]
    lib.bfm_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.bfm_server_destroy.argtypes = [vp]
    lib.bfm_operator_budget.argtypes = [vp, ctypes.c_size_t]
    lib.bfm_cache_get_stats.argtypes = [vp, ctypes.POINTER(CacheStats)]
    lib.bfm_server_operator_budget.argtypes = [vp, ctypes.c_size_t]
    _lib = lib
    return lib


def _raise(rc):
    if rc != SUCCESS:
        raise BfmError(rc, load().bfm_last_error().decode())


def version() -> int:
    return load().bfm_version()


def cache_stats(device: int = 0) -> dict:
    """bfm_cache_get_stats of the device's context: cached operator blocks,
    their bytes, the budget and the evictions so far."""
    st = CacheStats()
    _raise(load().bfm_cache_get_stats(context(device), ctypes.byref(st)))
    return {k: getattr(st, k) for k, _ in CacheStats._fields_}


def make_params(N: int, n: int, order: int = 3, freq: float = 23.0, h: float = 0.25,
                h_window: int = 0, lam: float = 2.5, mask_mode: int = MASK_NONE,
                times=None, precision="fp64") -> Params:
    """bfm_params.  ``times`` (N observation times, host) is copied into a
    float64 array that the returned struct keeps alive."""
    keep = None
    if times is not None:
        keep = np.ascontiguousarray(np.asarray(times, dtype=np.float64))
        if keep.shape != (int(N),):
            raise ValueError(f"times must hold N = {N} values")
    prm = Params(int(N), int(n), int(order), int(h_window), float(freq), float(h), float(lam),
                 int(mask_mode), _PRECISIONS.get(precision, precision),
                 None if keep is None else keep.ctypes.data_as(ctypes.c_void_p))
    prm._times = keep
    return prm


def check_params(prm: Params, P: int, ld: int) -> None:
    """bfm_check_params: validation only, no device."""
    _raise(load().bfm_check_params(ctypes.byref(prm), int(P), int(ld)))


def workspace_bytes(prm: Params, P: int) -> int:
    """bfm_workspace_bytes: device bytes the library caches for these parameters."""
    out = ctypes.c_size_t()
    _raise(load().bfm_workspace_bytes(ctypes.byref(prm), int(P), ctypes.byref(out)))
    return out.value


def host_operators(prm: Params):
    """bfm_host_operators: the shared operators as float64 tensors (host only)."""
    N, n, p = prm.n_obs, prm.n_hist, 2 + 2 * prm.order
    q = torch.empty(N, p, dtype=torch.float64)
    w = torch.empty(N - n, p, dtype=torch.float64)
    bnd = torch.empty(N - n, dtype=torch.float64)
    bmap = torch.empty(p, p, dtype=torch.float64)
    rc = load().bfm_host_operators(ctypes.byref(prm), q.data_ptr(), w.data_ptr(), bnd.data_ptr(),
                                   bmap.data_ptr())
    _raise(rc)
    return q, w, bnd, bmap


def create(device: int) -> int:
    """bfm_create: returns an opaque context handle."""
    h = ctypes.c_void_p()
    _raise(load().bfm_create(ctypes.byref(h), int(device)))
    return h.value


def destroy(ctx: int) -> None:
    _raise(load().bfm_destroy(ctx))


def context(device: int) -> int:
    """A per-process context for ``device``, created on first use."""
    with _lock:
        if device not in _ctx:
            _ctx[device] = create(device)
        return _ctx[device]


def _series_layout(Y: torch.Tensor):
    """Accept Y as (N, P) time-major contiguous, or its (P, N) transpose view."""
    if Y.dim() != 2:
        raise ValueError("Y must be 2-D")
    if Y.stride(1) == 1 and Y.stride(0) >= Y.shape[1]:
        return Y, Y.shape[0], Y.shape[1], Y.stride(0)  # (N, P) with row stride ld
    if Y.stride(0) == 1 and Y.stride(1) >= Y.shape[0]:
        return Y, Y.shape[1], Y.shape[0], Y.stride(1)  # (P, N) view of a time-major block
    raise ValueError("Y must be time-major: an (N, P) tensor with unit pixel stride, or its "
                     "transpose; make a time-major copy with Y.t().contiguous()")


def fit_monitor(Y: torch.Tensor, *, n: int, order: int = 3, freq: float = 23.0, h: float = 0.25,
                h_window: int = 0, lam: float = 2.5, mask_mode: int = MASK_NONE,
                valid: torch.Tensor | None = None, times=None, outputs=("brk", "mag"),
                out_dtype: torch.dtype = torch.float64, out: dict | None = None,
                stream: torch.cuda.Stream | None = None, precision="fp64") -> dict:
    """bfm_fit_monitor on a device-resident series block (float32, bfloat16 or
    float16, through bfm_fit_monitor_typed).

    ``Y`` is time-major: shape (N, P) with unit stride along pixels (or the
    (P, N) transpose view of such a block).  ``outputs`` names the arrays to
    produce among brk, mag, sigma, status, beta, resid, mosum; ``out`` may supply
    preallocated tensors for them.  ``times`` (N observation times, host) replaces
    the index t in the design rows.  ``precision`` "fp32" asks for the FP32
    MOSUM of the period-blocked missing-value path (BFM_PREC_FP32); other
    paths compute in FP64 either way.  Work is enqueued on ``stream``
    (default: the current stream) and the call returns without synchronising.
    """
    if Y.dtype not in _Y_DTYPES or Y.device.type != "cuda":
        raise ValueError("Y must be a float32, bfloat16 or float16 tensor on a HIP device")
    Y, N, P, ld = _series_layout(Y)
    dev = Y.device.index if Y.device.index is not None else torch.cuda.current_device()
    prm = make_params(N, n, order, freq, h, h_window, lam, mask_mode, times, precision)
    p = 2 + 2 * order
    shapes = {"brk": ((P,), torch.int32), "mag": ((P,), out_dtype), "sigma": ((P,), out_dtype),
              "status": ((P,), torch.uint8), "beta": ((p, P), out_dtype),
              "resid": ((N, P), out_dtype), "mosum": ((N - n, P), out_dtype)}
    if out_dtype not in (torch.float32, torch.float64):
        raise ValueError("out_dtype must be float32 or float64")
    res = dict(out or {})
    for name in set(outputs) | {"brk"}:
        if name not in shapes:
            raise ValueError(f"unknown output {name}")
        shp, dt = shapes[name]
        t = res.get(name)
        if t is None:
            res[name] = torch.empty(shp, dtype=dt, device=Y.device)
        elif tuple(t.shape) != shp or t.dtype != dt or not t.is_contiguous() or t.device != Y.device:
            raise ValueError(f"out[{name!r}] must be a contiguous {dt} tensor of shape {shp}")
    o = Outputs(*(res[k].data_ptr() if k in res else None
                  for k in ("brk", "mag", "sigma", "status", "beta", "resid", "mosum")),
                OUT_F64 if out_dtype == torch.float64 else OUT_F32)
    vptr, ldv = None, 0
    if mask_mode == MASK_EXPLICIT:
        if valid is None:
            raise ValueError("valid is required with MASK_EXPLICIT")
        valid, Nv, Pv, ldv = _series_layout(valid)
        if (Nv, Pv) != (N, P) or valid.dtype != torch.uint8 or valid.device != Y.device:
            raise ValueError("valid must be a uint8 tensor laid out like Y")
        vptr = valid.data_ptr()
    s = stream if stream is not None else torch.cuda.current_stream(Y.device)
    y_dtype = _Y_DTYPES[Y.dtype]
    rc = load().bfm_fit_monitor_typed(context(dev), ctypes.byref(prm), Y.data_ptr(), y_dtype, P, ld,
                                      vptr, ldv, ctypes.byref(o), s.cuda_stream)
    _raise(rc)
    return res


def mosum_null_sup(*, n: int, N: int, h: float = 0.25, h_window: int = 0, seed: int = 0,
                   path0: int = 0, paths: int = 100000, device: int = 0,
                   stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """bfm_mosum_null_sup: the sup statistic of simulated no-change MOSUM paths
    path0 .. path0+paths-1 (float64 tensor on the device)."""
    prm = make_params(N, n, 0, 23.0, h, h_window, 1.0, MASK_NONE)
    sup = torch.empty(int(paths), dtype=torch.float64, device=f"cuda:{device}")
    s = stream if stream is not None else torch.cuda.current_stream(sup.device)
    _raise(load().bfm_mosum_null_sup(context(device), ctypes.byref(prm), ctypes.c_uint64(seed),
                                     int(path0), int(paths), sup.data_ptr(), s.cuda_stream))
    return sup


def critical_value(alpha: float, *, n: int, N: int, h: float = 0.25, h_window: int = 0,
                   paths: int = 100000, seed: int = 0, device: int = 0,
                   stream: torch.cuda.Stream | None = None) -> float:
    """bfm_critical_value: lambda of Eq. 4 for (alpha, window, N/n) by simulation."""
    prm = make_params(N, n, 0, 23.0, h, h_window, 1.0, MASK_NONE)
    out = ctypes.c_double()
    s = stream if stream is not None else torch.cuda.current_stream(torch.device(f"cuda:{device}"))
    _raise(load().bfm_critical_value(context(device), ctypes.byref(prm), ctypes.c_double(alpha),
                                     int(paths), ctypes.c_uint64(seed), ctypes.byref(out),
                                     s.cuda_stream))
    return out.value


def critical_value_noalloc(alpha: float, *, n: int, N: int, h: float = 0.25, h_window: int = 0,
                           paths: int = 100000, seed: int = 0, device: int = 0,
                           stream: torch.cuda.Stream | None = None) -> float:
    """bfm_critical_value_noalloc: the same value as critical_value, computed in
    the library's fixed scratch array (no device allocation; paths <=
    NOALLOC_MAX_PATHS; calls that overlap on one GPU race)."""
    prm = make_params(N, n, 0, 23.0, h, h_window, 1.0, MASK_NONE)
    out = ctypes.c_double()
    s = stream if stream is not None else torch.cuda.current_stream(torch.device(f"cuda:{device}"))
    _raise(load().bfm_critical_value_noalloc(context(device), ctypes.byref(prm), ctypes.c_double(alpha),
                                             int(paths), ctypes.c_uint64(seed), ctypes.byref(out),
                                             s.cuda_stream))
    return out.value


def autotune(Y: torch.Tensor, *, n: int, order: int = 3, freq: float = 23.0, h: float = 0.25,
             h_window: int = 0, lam: float = 2.5, mask_mode: int = MASK_NONE, stream=None):
    """bfm_autotune: time the row splits on Y (the plain path, or with
    ``mask_mode=MASK_NAN`` the history split of the missing-value path) and keep
    the fastest for this tile shape.  Returns (split, {split: median us})."""
    Y, N, P, ld = _series_layout(Y)
    dev = Y.device.index if Y.device.index is not None else torch.cuda.current_device()
    prm = make_params(N, n, order, freq, h, h_window, lam, mask_mode)
    s = stream if stream is not None else torch.cuda.current_stream(Y.device)
    split = ctypes.c_int32()
    times = (ctypes.c_double * 4)()
    _raise(load().bfm_autotune(context(dev), ctypes.byref(prm), Y.data_ptr(), _Y_DTYPES[Y.dtype], P, ld,
                               s.cuda_stream, ctypes.byref(split), times))
    return split.value, {k: times[i] for i, k in enumerate((1, 2, 4, 8)) if times[i] > 0}


def tune_set(Y: torch.Tensor, split: int, *, n: int, order: int = 3, freq: float = 23.0,
             h: float = 0.25, h_window: int = 0, lam: float = 2.5, mask_mode: int = MASK_NONE):
    """bfm_tune_set: pin the row split for Y's tile shape (the plain path, or
    the missing-value path's history split with MASK_NAN / MASK_EXPLICIT)."""
    Y, N, P, ld = _series_layout(Y)
    dev = Y.device.index if Y.device.index is not None else torch.cuda.current_device()
    prm = make_params(N, n, order, freq, h, h_window, lam, mask_mode)
    _raise(load().bfm_tune_set(context(dev), ctypes.byref(prm), _Y_DTYPES[Y.dtype], P, int(split)))


class Server:
    """bfm_server_*: requests of different shapes and parameters, run as they
    arrive on ``slots`` streams of one device, admitted by free stream, by room
    for their outputs in a device pool of ``pool_bytes`` (allocated once) and by
    room for a new parameter set's operators in ``operator_budget`` bytes
    (default 64 MiB).

    ``submit`` takes the same arguments as ``fit_monitor`` (without ``out``) and
    returns a ticket at once; ``result`` waits for it and returns its outputs as
    new tensors (bfm_server_take copies them out of the pool and releases it)
    with its timings.
    The caller keeps ``Y`` (and ``valid``) alive and unchanged until then.
    """

    def __init__(self, device: int = 0, slots: int = 4, pool_bytes: int = 1 << 30,
                 operator_budget: int | None = None):
        h = ctypes.c_void_p()
        _raise(load().bfm_server_create(ctypes.byref(h), int(device), int(slots), int(pool_bytes)))
        self.handle = h.value
        self.device = torch.device("cuda", device)
        self._pending = {}
        if operator_budget is not None:
            _raise(load().bfm_server_operator_budget(self.handle, int(operator_budget)))

    def close(self):
        if self.handle:
            load().bfm_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def request(self, Y, *, n, order=3, freq=23.0, h=0.25, h_window=0, lam=2.5,
                mask_mode=MASK_NONE, valid=None, times=None, outputs=("brk", "mag"),
                out_dtype=torch.float64, precision="fp64"):
        """The bfm_request for these arguments (no device work).  The request
        keeps its observation times alive."""
        if Y.dtype not in _Y_DTYPES or Y.device.type != "cuda":
            raise ValueError("Y must be a float32, bfloat16 or float16 tensor on a HIP device")
        Y, N, P, ld = _series_layout(Y)
        prm = make_params(N, n, order, freq, h, h_window, lam, mask_mode, times, precision)
        want = 0
        for name in outputs:
            if name != "brk":
                want |= WANT[name]
        vptr, ldv = None, 0
        if mask_mode == MASK_EXPLICIT:
            if valid is None:
                raise ValueError("valid is required with MASK_EXPLICIT")
            valid, _, _, ldv = _series_layout(valid)
            vptr = valid.data_ptr()
        req = Request(prm, Y.data_ptr(), _Y_DTYPES[Y.dtype], P, ld, vptr, ldv, want,
                      OUT_F64 if out_dtype == torch.float64 else OUT_F32)
        req._times = prm._times
        return req

    def submit(self, Y, **kw) -> int:
        req = self.request(Y, **kw)
        t = ctypes.c_uint64()
        _raise(load().bfm_server_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        self._pending[t.value] = (req, kw.get("outputs", ("brk", "mag")),
                                  kw.get("out_dtype", torch.float64))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> Result:
        res = Result()
        _raise(load().bfm_server_wait(self.handle, int(ticket), int(timeout_ms), ctypes.byref(res)))
        return res

    def result(self, ticket: int, timeout_ms: int = -1) -> dict:
        """Wait for a request, copy its outputs into new tensors, release it.
        Returns the outputs plus ``rc`` and the timings in microseconds."""
        req, outputs, out_dtype = self._pending.pop(ticket)
        res = self.wait(ticket, timeout_ms)
        P, N, n, p = req.P, req.prm.n_obs, req.prm.n_hist, 2 + 2 * req.prm.order
        shapes = {"brk": ((P,), torch.int32), "mag": ((P,), out_dtype), "sigma": ((P,), out_dtype),
                  "status": ((P,), torch.uint8), "beta": ((p, P), out_dtype),
                  "resid": ((N, P), out_dtype), "mosum": ((N - n, P), out_dtype)}
        out = {"rc": res.rc, "queued_us": res.queued_us, "latency_us": res.latency_us,
               "device_us": res.device_us}
        if res.rc != SUCCESS:
            _raise(load().bfm_server_release(self.handle, int(ticket)))
            return out
        for name in set(outputs) | {"brk"}:
            shp, dt = shapes[name]
            out[name] = torch.empty(shp, dtype=dt, device=self.device)
        dst = Outputs(*(out[k].data_ptr() if k in out else None
                        for k in ("brk", "mag", "sigma", "status", "beta", "resid", "mosum")),
                      req.out_dtype)
        s = torch.cuda.current_stream(self.device)
        _raise(load().bfm_server_take(self.handle, int(ticket), ctypes.byref(dst), s.cuda_stream))
        return out

    def stats(self) -> dict:
        st = ServerStats()
        _raise(load().bfm_server_get_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}
