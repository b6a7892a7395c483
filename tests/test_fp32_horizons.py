"""The FP32 horizons of the sum-product parity tests (CPU only).

An FP32 decoder rounds every message, posterior and extrinsic value to 24
bits.  On a frame that converges this changes nothing visible; on a frame
that never converges the rounding differences grow from iteration to
iteration, and past some horizon no FP32 implementation can stay within the
1e-4 bar of the FP64 oracle.  This test measures that growth without any GPU
code: it builds copies of the FP64 oracles (flooding and layered) that add
relative noise of 6e-8 (one FP32 rounding) to every q, r and L they form, and
takes the largest spread of their posteriors from the clean oracle
(relative to max(|L|, A_n), frames with equal iteration counts) over a few
noise seeds.  It pins:
  - at the horizons the GPU tests compare in full (10 flooding iterations,
    5 layered passes: HORIZON_F32), the spread of every parity input stays
    below half the 1e-4 bar;
  - past them, on the chaotic input qc_d16, the spread exceeds the bar
    (20 flooding iterations) or is of order 1e-1 (20 layered passes), so
    comparing there in full would test rounding, not the decoder.
"""
import ctypes

import numpy as np
import pytest

import oracle
import degree_cases as degrees
from oracle.build import SRC, SRC_LAYERED, compile_oracle
from parity_util import HORIZON_F32
from workloads import channel, configs

NOISE = """#define ORACLE_ENOMEM (-2)
static unsigned long long g_state = 1;
void noise_seed(unsigned long long s) { g_state = s; }
static double noise(double v)
{
    g_state = g_state * 6364136223846793005ULL + 1442695040888963407ULL;
    const double u = (double)(g_state >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    return v * (1.0 + u * 6e-8);
}"""

EDITS = {
    "flooding": (SRC, [("r[e] = v;", "r[e] = noise(v);"), ("L[j] = s;", "L[j] = noise(s);"),
                       ("q[g->col_edge[k]] = s - r[g->col_edge[k]];",
                        "q[g->col_edge[k]] = noise(s - r[g->col_edge[k]]);")]),
    "layered": (SRC_LAYERED, [("q[e - e0] = L[col_idx[e]] - r[e];", "q[e - e0] = noise(L[col_idx[e]] - r[e]);"),
                              ("        r[e] = v;\n    }", "        r[e] = noise(v);\n    }"),
                              ("L[col_idx[e]] = q[e - e0] + r[e];", "L[col_idx[e]] = noise(q[e - e0] + r[e]);")]),
}


@pytest.fixture(scope="module")
def noisy(tmp_path_factory):
    d = tmp_path_factory.mktemp("noisy")
    libs = {}
    for sched, (src_path, edits) in EDITS.items():
        src = open(src_path).read().replace("#define ORACLE_ENOMEM (-2)", NOISE)
        for old, new in edits:
            assert src.count(old) == 1, old
            src = src.replace(old, new)
        path = d / f"noisy_{sched}.c"
        path.write_text(src)
        lib = oracle._load(compile_oracle(str(path), str(d / f"libnoisy_{sched}.so"), extra=("-Wno-error",)))
        lib.noise_seed.argtypes = [ctypes.c_ulonglong]
        libs[sched] = lib
    return libs


def spread(lib, code, llr, T, es, sched, seeds=(1, 2, 3)):
    base = oracle.decode(code, llr, T, es, nthreads=4, schedule=sched)
    scale = np.maximum(np.abs(base["posterior"]), base["cond"])
    worst = 0.0
    for seed in seeds:
        lib.noise_seed(seed)
        o = oracle.decode(code, llr, T, es, nthreads=1, schedule=sched, lib=lib)
        same = o["iters"] == base["iters"]
        worst = max(worst, float((np.abs(o["posterior"] - base["posterior"]) / scale)[same].max()))
    return worst


@pytest.mark.parametrize("name", degrees.NAMES)
def test_degree_inputs_within_horizon(noisy, name):
    code, llr = degrees.workload(name, "f32")
    for sched in ("flooding", "layered"):
        T = HORIZON_F32[sched]
        assert spread(noisy[sched], code, llr, T, False, sched) < 0.5e-4, (name, sched)


def test_qc1944_within_horizon(noisy):
    """The headline inputs at the benchmark horizon, and the layered parity input at 5 passes."""
    for snr in configs.QC1944_SNRS:
        b = configs.qc1944(snr, frames=64)
        assert spread(noisy["flooding"], b.code, b.llr, 10, False, "flooding") < 0.5e-4, snr
    b = configs.qc1944(2.0, frames=64)
    llr = channel.bpsk_awgn_llr(b.codewords, 3.5, 0.5, 911, dtype=np.float32)
    assert spread(noisy["layered"], b.code, llr, 5, False, "layered") < 0.5e-4


def test_beyond_horizon_spreads(noisy):
    code, llr = degrees.workload("qc_d16", "f32")
    assert spread(noisy["flooding"], code, llr, 20, True, "flooding", seeds=(1, 2, 3, 4)) > 1e-4
    assert spread(noisy["layered"], code, llr, 20, True, "layered") > 1e-2
