"""How accurate is the FP64 oracle itself?  (CPU only.)

The oracle evaluates the check rule exactly as defined, 2 atanh(prod tanh(q/2)),
in double precision.  Near the clamp the product is within a few 1e-9 of 1
and 2 atanh loses digits, so the oracle's posterior carries a small error of
its own.  This test builds the copy whose check node runs in 80-bit long
double (ORACLE_CHECK_LD: a precision variant, not a different method) and
bounds the FP64 oracle's deviation on the Gallager workload; that bound is
what the FP64 parity tolerance rests on.
"""
import platform

import numpy as np
import pytest

import oracle
from oracle.build import SRC, compile_oracle
from workloads import configs


@pytest.mark.skipif(platform.machine() not in ("x86_64", "AMD64"), reason="needs x87 long double")
def test_fp64_oracle_error_bound(tmp_path):
    lib = oracle._load(compile_oracle(SRC, str(tmp_path / "libld.so"), extra=("-DORACLE_CHECK_LD",)))
    b = configs.gallager504(frames=400)
    a = oracle.decode(b.code, b.llr, 20, True, nthreads=4)
    h = oracle.decode(b.code, b.llr, 20, True, nthreads=4, lib=lib)
    same = a["iters"] == h["iters"]
    assert same.mean() > 0.99
    err = np.abs(a["posterior"] - h["posterior"]) / np.maximum(np.abs(h["posterior"]), h["cond"])
    worst = err[same].max()
    assert worst < 1e-6, worst
    assert worst > 1e-12  # the effect is real: the FP64 definition is not exact here
