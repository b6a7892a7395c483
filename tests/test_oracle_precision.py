"""How accurate is the FP64 oracle itself?  (CPU only.)

The oracle evaluates the check rule exactly as defined, 2 atanh(prod tanh(q/2)),
in double precision.  Near the clamp the product is within a few 1e-9 of 1
and 2 atanh loses digits, so the oracle's posterior carries a small error of
its own.  This test builds a copy whose check node runs in 80-bit long double
(a precision variant, not a different method) and bounds the FP64 oracle's
deviation on the Gallager workload; that bound is what the FP64 parity
tolerance rests on.
"""
import platform

import numpy as np
import pytest

import oracle
from oracle.build import SRC, compile_oracle
from workloads import configs

EDITS = [
    ("th[e] = tanh(q[e] / 2.0);", "th[e] = (double)tanhl((long double)q[e] / 2.0L);"),
    ("""                    double p = 1.0;
                    for (int32_t o = e0; o < e1; ++o)
                        if (o != e)
                            p *= th[o];
                    double v = 2.0 * atanh(p);""",
     """                    long double p = 1.0L;
                    for (int32_t o = e0; o < e1; ++o)
                        if (o != e)
                            p *= tanhl((long double)q[o] / 2.0L);
                    double v = (double)(2.0L * atanhl(p));"""),
]


@pytest.mark.skipif(platform.machine() not in ("x86_64", "AMD64"), reason="needs x87 long double")
def test_fp64_oracle_error_bound(tmp_path):
    src = open(SRC).read()
    for old, new in EDITS:
        assert old in src
        src = src.replace(old, new)
    p = tmp_path / "oracle_ld.c"
    p.write_text(src)
    lib = oracle._load(compile_oracle(str(p), str(tmp_path / "libld.so"), extra=("-Wno-error",)))
    b = configs.gallager504(frames=400)
    a = oracle.decode(b.code, b.llr, 20, True, nthreads=4)
    h = oracle.decode(b.code, b.llr, 20, True, nthreads=4, lib=lib)
    same = a["iters"] == h["iters"]
    assert same.mean() > 0.99
    err = np.abs(a["posterior"] - h["posterior"]) / np.maximum(np.abs(h["posterior"]), h["cond"])
    worst = err[same].max()
    assert worst < 1e-6, worst
    assert worst > 1e-12  # the effect is real: the FP64 definition is not exact here
