"""Oracle: plain, slow FP64 sum-product decoders on the CPU (flooding and
layered schedules).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the decoder library and
its Python binding never do.  It shares no code with the GPU path.

``decode`` follows Section II of arxiv 1812.06545 (Tanner graph of H, two-phase
message passing, Algorithm 1's loop order) with the sum-product check rule of
Section I; see spa_oracle.c for the exact definition and readings.  With
``schedule="layered"`` it runs the serial check-node schedule of the paper's
layered algorithm (Algorithm 2, Section II) instead; see layered_oracle.c.
With ``rule="minsum"`` the check rule is min-sum (the rule Algorithm 1 is
named after), with optional scale and offset of the magnitude; see
minsum_oracle.c.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB, LIB_LD, compile_long_double, compile_oracle

R_MAX = 20.0  # clamp on check-to-variable messages (a reading: the paper gives none)

_lib = None


def _load(path: str = LIB):
    global _lib
    if _lib is None or path != LIB:
        if not os.path.exists(path):
            compile_oracle(out=path) if path == LIB else None
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        for name in ("oracle_spa_decode", "oracle_spa_layered_decode"):
            if not hasattr(lib, name):  # a test build may hold only one of the two
                continue
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int,
                          ctypes.c_double, P, P, P, P, P, ctypes.c_int]
            f.restype = ctypes.c_int
        if hasattr(lib, "oracle_minsum_decode"):
            f = lib.oracle_minsum_decode
            f.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P, P, P, P, ctypes.c_int]
            f.restype = ctypes.c_int
        if path != LIB:
            return lib
        _lib = lib
    return _lib


_lib_ld = None


def long_double_lib():
    """The flooding sum-product oracle with its check node evaluated in 80-bit
    long double (each message rounded to double): the same definition at
    higher precision, for bounding the double oracle's own rounding and for
    tight FP64 comparisons.  Pass it as ``decode(..., lib=...)``."""
    global _lib_ld
    if _lib_ld is None:
        if not os.path.exists(LIB_LD):
            compile_long_double()
        _lib_ld = _load(LIB_LD)
    return _lib_ld


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def decode(code, llr, max_iter: int, early_stop: bool, r_max: float = R_MAX, nthreads: int = 1,
           want_trace: bool = True, lib=None, schedule: str = "flooding", rule: str = "spa",
           ms_scale: float = 1.0, ms_offset: float = 0.0):
    """Decode frames ``llr`` (F, n) -> dict(bits, iters, posterior, cond, min_abs).

    ``schedule`` is "flooding" (all checks, then all variables, per iteration)
    or "layered" (check rows one at a time in ascending order, each updating
    its variables at once; one iteration = one pass over the rows).  ``rule``
    is "spa" (sum-product) or "minsum" (|r| = max(ms_scale * min - ms_offset,
    0), then the clamp).

    float32 input is upcast to float64 unchanged, so both sides see the same
    values.  ``lib`` lets the tests point at a deliberately broken build.
    """
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float64)
    F, n = llr.shape
    assert n == code.n
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    bits = np.zeros((F, n), dtype=np.uint8)
    iters = np.zeros(F, dtype=np.int32)
    post = np.zeros((F, n), dtype=np.float64)
    cond = np.zeros((F, n), dtype=np.float64)
    mabs = np.zeros((F, max_iter + 1), dtype=np.float64) if want_trace else None
    L = lib if lib is not None else _load()
    if schedule not in ("flooding", "layered"):
        raise ValueError(f"unknown schedule {schedule!r}")
    if rule == "minsum":
        st = L.oracle_minsum_decode(code.m, n, _ptr(rp), _ptr(ci), F, _ptr(llr), int(max_iter), int(bool(early_stop)),
                                    int(schedule == "layered"), float(ms_scale), float(ms_offset), float(r_max),
                                    _ptr(bits), _ptr(iters), _ptr(post), _ptr(cond), _ptr(mabs), int(nthreads))
    elif rule == "spa":
        fn = L.oracle_spa_decode if schedule == "flooding" else L.oracle_spa_layered_decode
        st = fn(code.m, n, _ptr(rp), _ptr(ci), F, _ptr(llr), int(max_iter), int(bool(early_stop)), float(r_max),
                _ptr(bits), _ptr(iters), _ptr(post), _ptr(cond), _ptr(mabs), int(nthreads))
    else:
        raise ValueError(f"unknown rule {rule!r}")
    if st != 0:
        raise ValueError(f"oracle ({schedule}, {rule}) failed with status {st}")
    return {"bits": bits, "iters": iters, "posterior": post, "cond": cond, "min_abs": mabs}
