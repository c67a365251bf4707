"""The no-allocation critical value against the allocating one (GPU).

bfm_critical_value_noalloc runs the same kernels as bfm_critical_value in the
library's fixed scratch array; both are called through the C ABI on the same
seeds and must return the same order statistic (the selection is exact, so the
values are equal bit for bit), on two calls in a row with the second smaller
(the scratch keeps the first call's statistics and counters), and a path count
past the array's capacity is refused.
"""
import ctypes
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def bfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_01751_amd import bfm as b
    b.load()
    return b


def _call(bfm, fn, prm, alpha, paths, seed):
    lib = bfm.load()
    out = ctypes.c_double()
    s = torch.cuda.current_stream()
    rc = getattr(lib, fn)(bfm.context(0), ctypes.byref(prm), ctypes.c_double(alpha), int(paths),
                          ctypes.c_uint64(seed), ctypes.byref(out), s.cuda_stream)
    return rc, out.value


@pytest.mark.parametrize("first,second", [(1 << 20, 50000), (300000, 4097)])
def test_noalloc_equals_allocating_entry_point(bfm, first, second):
    for paths, (n, N, hw, alpha, seed) in ((first, (200, 400, 50, 0.05, 7)),
                                           (second, (114, 228, 28, 0.01, 8))):
        say(f"case noalloc paths={paths} n={n} N={N} H={hw} alpha={alpha} seed={seed}")
        prm = bfm.make_params(N, n, 0, h_window=hw)
        rc_a, lam_a = _call(bfm, "bfm_critical_value", prm, alpha, paths, seed)
        rc_b, lam_b = _call(bfm, "bfm_critical_value_noalloc", prm, alpha, paths, seed)
        assert rc_a == 0 and rc_b == 0, bfm.load().bfm_last_error()
        assert lam_a == lam_b and 0.5 < lam_b < 6.0, (paths, lam_a, lam_b)


def test_noalloc_refuses_more_paths_than_its_array_holds(bfm):
    prm = bfm.make_params(400, 200, 0, h_window=50)
    say("case noalloc paths over capacity")
    rc, _ = _call(bfm, "bfm_critical_value_noalloc", prm, 0.05, bfm.NOALLOC_MAX_PATHS + 1, 1)
    assert rc == bfm.E_INVAL
    assert "paths must be in" in bfm.load().bfm_last_error().decode()
