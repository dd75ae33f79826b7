"""qnsch_residual_noalloc (the entry point for callers that cannot allocate)
against qnsch_residual of a context holding the same iterate and time-n data:
two calls in a row, the second on a smaller grid, through the C ABI.  Both
run the same residual and reduction kernels over the same tiles, so the norms
agree to rounding (1e-13 relative asked; the same sums in the same order)."""
import sys

import numpy as np
import pytest

from paper_1703_06606_amd import qnsch as Q
from paper_1703_06606_amd import workloads as W

pytestmark = pytest.mark.gpu
FIELDS = ("c", "mu", "p", "u", "v")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _hip():
    """the HIP runtime the library runs on (the test's own device buffers
    come from it, so that one runtime serves the process)"""
    import ctypes as C
    Q.lib()
    h = C.CDLL("libamdhip64.so.7")
    h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    h.hipFree.argtypes = [C.c_void_p]
    return h


def _device(h, a, keep):
    import ctypes as C
    a = np.ascontiguousarray(a, dtype=np.float64)
    p = C.c_void_p()
    assert h.hipMalloc(C.byref(p), a.nbytes) == 0
    keep.append(p)
    assert h.hipMemcpy(p, a.ctypes.data_as(C.c_void_p), a.nbytes, 1) == 0  # host to device
    return p.value


def _case(cfg, seed_w, seed_n, dt):
    grid, params = cfg["grid"], cfg["params"]
    w, wn = W.random_state(grid, seed_w), W.random_state(grid, seed_n)
    g = Q.Solver(grid, params, W.default_opts())
    g.set_time_n_and_iterate(wn, w, dt)
    _, ref = g.residual()
    h, keep = _hip(), []
    try:
        dw = {k: _device(h, w[k], keep) for k in FIELDS}
        dn = {k: _device(h, wn[k], keep) for k in ("c", "u", "v")}
        got = Q.residual_noalloc(grid, params, dt, dw, dn)
    finally:
        for p in keep:
            h.hipFree(p)
    say(cfg["name"], "context", ref, "no-alloc", got)
    assert np.allclose(got, ref, rtol=1e-13, atol=0), (got, ref)
    return got


def test_residual_noalloc_matches_context_residual():
    say("no-alloc residual: 40x24 walls, then 16x32 periodic x")
    big = W.rising_drop(40, 24, eps=0.05, radius=0.2)
    small = W.capillary(16, 32, eps=0.08, levels=3)
    a = _case(big, 51, 52, 0.3)
    b = _case(small, 53, 54, 0.2)
    assert not np.array_equal(a, b)
    # sizes beyond the static array are rejected on the host
    huge = dict(big["grid"], m1=4096, m2=2048, Lx=1.0, Ly=0.5)
    with pytest.raises(Q.QnschError):
        Q.residual_noalloc(huge, big["params"], 0.1, {k: 1 for k in FIELDS}, {k: 1 for k in ("c", "u", "v")})
