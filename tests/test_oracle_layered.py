"""The layered-schedule oracle against its pins, and planted mistakes in it
caught by those pins (CPU only).

Each mutant is a copy of layered_oracle.c with one plausible slip (a dropped
term, a wrong sign, order or index, a wrong comparison); it is compiled to a
temporary library and run through every pin, and at least one pin must fail.
"""
import ctypes

import numpy as np
import pytest

import oracle
import pins_layered
from oracle.build import SRC_LAYERED, compile_oracle
from parity_util import TOL_LAYERED
from workloads import channel, configs


def _dec(lib=None):
    return lambda code, llr, T, es: oracle.decode(code, llr, T, es, schedule="layered", lib=lib)


@pytest.mark.parametrize("check", pins_layered.ALL, ids=lambda f: f.__name__)
def test_layered_pin(check, oracle_mod):
    check(_dec())


MUTANTS = {
    "self_in_product": ("if (o != e)", "if (1)"),
    "no_half_in_tanh": ("tanh(q[e - e0] / 2.0)", "tanh(q[e - e0])"),
    "no_factor_two": ("double v = 2.0 * atanh(p);", "double v = atanh(p);"),
    "sign_flip": ("double v = 2.0 * atanh(p);", "double v = -2.0 * atanh(p);"),
    "no_extrinsic": ("q[e - e0] = L[col_idx[e]] - r[e];", "q[e - e0] = L[col_idx[e]];"),
    "new_message_dropped": ("L[col_idx[e]] = q[e - e0] + r[e];", "L[col_idx[e]] = q[e - e0];"),
    "old_message_kept": ("L[col_idx[e]] = q[e - e0] + r[e];", "L[col_idx[e]] += r[e];"),
    "rows_descending": ("for (int i = 0; i < m; ++i)\n                visit_row",
                        "for (int i = m - 1; i >= 0; --i)\n                visit_row"),
    "decision_le": ("x[j] = (uint8_t)(L[j] < 0.0);\n            if (min_abs)",
                    "x[j] = (uint8_t)(L[j] <= 0.0);\n            if (min_abs)"),
    "no_clamp": ("if (v > r_max)\n            v = r_max;", ""),
    "iters_off_by_one": ("t_done = t;", "t_done = t - 1;"),
    "no_initial_stop": ("if (early_stop && layered_syndrome_is_zero(m, row_ptr, col_idx, x)) {\n        t_done = 0;",
                        "if (0) {\n        t_done = 0;"),
    "cond_message_signed": ("cond[col_idx[e]] += fabs(r[e]);", "cond[col_idx[e]] += r[e];"),
    "cond_channel_signed": ("cond[j] = fabs(llr[j]);", "cond[j] = llr[j];"),
    "min_abs_signed": ("if (fabs(L[j]) < v)\n            v = fabs(L[j]);", "if (L[j] < v)\n            v = L[j];"),
    "min_abs_shifted": ("min_abs[t] = layered_min_abs(n, L);", "min_abs[t - 1] = layered_min_abs(n, L);"),
    "messages_not_reset": ("        r[e] = 0.0;\n    if (min_abs)", "        r[e] = r[e];\n    if (min_abs)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_layered_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC_LAYERED).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mpath = tmp_path / f"mut_{name}.c"
    mpath.write_text(src.replace(old, new, 1))
    lib = oracle._load(compile_oracle(str(mpath), str(tmp_path / f"libmut_{name}.so"), extra=("-Wno-error",)))
    failed = []
    for check in pins_layered.ALL:
        try:
            check(_dec(lib))
        except (AssertionError, ValueError, FloatingPointError):
            failed.append(check.__name__)
    assert failed, f"mutant {name} passed every pin"


def test_fp32_rounding_spread(tmp_path):
    """Justifies the FP32 bar of the layered parity tests: the FP64 layered
    oracle with relative noise of 6e-8 (one FP32 rounding) injected into every
    q, r and L update, on the 3.5 dB qc1944 input of the GPU parity test, 10
    passes.  The spread of the posteriors (relative to max(|L|, A_n)) exceeds
    the flooding bar of 1e-4, so no FP32 implementation can be held to it,
    and stays below half of the layered bar."""
    src = open(SRC_LAYERED).read()
    src = src.replace("#define ORACLE_ENOMEM (-2)", """#define ORACLE_ENOMEM (-2)
static unsigned long long g_state = 1;
void noise_seed(unsigned long long s) { g_state = s; }
static double noise(double v)
{
    g_state = g_state * 6364136223846793005ULL + 1442695040888963407ULL;
    const double u = (double)(g_state >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    return v * (1.0 + u * 6e-8);
}""")
    edits = [("q[e - e0] = L[col_idx[e]] - r[e];", "q[e - e0] = noise(L[col_idx[e]] - r[e]);"),
             ("        r[e] = v;\n    }", "        r[e] = noise(v);\n    }"),
             ("L[col_idx[e]] = q[e - e0] + r[e];", "L[col_idx[e]] = noise(q[e - e0] + r[e]);")]
    for old, new in edits:
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    path = tmp_path / "noisy.c"
    path.write_text(src)
    lib = oracle._load(compile_oracle(str(path), str(tmp_path / "libnoisy.so"), extra=("-Wno-error",)))
    lib.noise_seed.argtypes = [ctypes.c_ulonglong]
    b = configs.qc1944(2.0, frames=130)
    llr = channel.bpsk_awgn_llr(b.codewords, 3.5, 0.5, 911, dtype=np.float32)
    base = oracle.decode(b.code, llr, 10, False, nthreads=4, schedule="layered")
    scale = np.maximum(np.abs(base["posterior"]), base["cond"])
    spread = 0.0
    for seed in (1, 2, 3, 4):
        lib.noise_seed(seed)
        noisy = oracle.decode(b.code, llr, 10, False, nthreads=1, schedule="layered", lib=lib)
        spread = max(spread, float((np.abs(noisy["posterior"] - base["posterior"]) / scale).max()))
    assert 1e-4 < spread < 0.5 * TOL_LAYERED[np.float32], spread
