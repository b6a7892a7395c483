"""Planted mistakes in the oracle are caught by the pins (CPU only).

Each mutant is a copy of spa_oracle.c with one plausible slip (a dropped term,
a wrong sign or index, a wrong comparison).  It is compiled to a temporary
library and run through every pin; the test asserts that at least one pin
fails, so a mistake of that kind in the real oracle could not pass unnoticed.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle
import pins
from oracle.build import SRC, compile_oracle

MUTANTS = {
    "self_in_product": ("if (o != e)", "if (1)"),
    "no_half_in_tanh": ("th[e] = CHK_TANH((chk_real)q[e] / 2);", "th[e] = CHK_TANH((chk_real)q[e]);"),
    "no_factor_two": ("double v = (double)(2 * CHK_ATANH(p));", "double v = (double)CHK_ATANH(p);"),
    "sign_flip": ("double v = (double)(2 * CHK_ATANH(p));", "double v = (double)(-2 * CHK_ATANH(p));"),
    "drop_channel_term": ("double s = llr[j];", "double s = 0.0;"),
    "no_extrinsic": ("q[g->col_edge[k]] = s - r[g->col_edge[k]];", "q[g->col_edge[k]] = s;"),
    "decision_le": ("x[j] = (uint8_t)(L[j] < 0.0);", "x[j] = (uint8_t)(L[j] <= 0.0);"),
    "no_clamp": ("if (v > r_max)\n                        v = r_max;", ""),
    "iters_off_by_one": ("t_done = t;", "t_done = t - 1;"),
    "no_initial_stop": ("if (early_stop && syndrome_is_zero(m, g->row_ptr, g->col_idx, x)) {\n        t_done = 0;",
                        "if (0) {\n        t_done = 0;"),
    "stale_decision": ("x[j] = (uint8_t)(L[j] < 0.0);\n            if (min_abs)",
                       "x[j] = (uint8_t)(q[g->col_ptr[j]] < 0.0);\n            if (min_abs)"),
    "cond_message_unsigned_dropped": ("a += fabs(r[g->col_edge[k]]);", "a += r[g->col_edge[k]];"),
    "cond_channel_dropped": ("double a = fabs(llr[j]);", "double a = 0.0;"),
    "cond_wrong_column": ("for (int32_t k = g->col_ptr[j]; k < g->col_ptr[j + 1]; ++k)\n                a += fabs",
                          "for (int32_t k = g->col_ptr[(j + 1) % n]; k < g->col_ptr[(j + 1) % n + 1]; ++k)\n"
                          "                a += fabs"),
    "min_abs_signed": ("if (fabs(L[j]) < v)\n            v = fabs(L[j]);", "if (L[j] < v)\n            v = L[j];"),
    "min_abs_shifted": ("min_abs[t] = min_abs_of(n, L);", "min_abs[t - 1] = min_abs_of(n, L);"),
    "first_edge_dropped_in_sum": ("for (int32_t k = g->col_ptr[j]; k < g->col_ptr[j + 1]; ++k)\n                    s += r",
                                  "for (int32_t k = g->col_ptr[j] + 1; k < g->col_ptr[j + 1]; ++k)\n                    s += r"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new, 1)
    mpath = tmp_path / f"mut_{name}.c"
    mpath.write_text(mutated)
    lib_path = str(tmp_path / f"libmut_{name}.so")
    compile_oracle(str(mpath), lib_path, extra=("-Wno-error",))
    lib = oracle._load(lib_path)
    dec = lambda code, llr, T, es: oracle.decode(code, llr, T, es, lib=lib)
    failed = []
    for check in pins.ALL:
        try:
            check(dec)
        except (AssertionError, ValueError, FloatingPointError):
            failed.append(check.__name__)
    assert failed, f"mutant {name} passed every pin"
