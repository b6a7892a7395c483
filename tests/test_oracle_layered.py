"""The layered-schedule oracle against its pins, and planted mistakes in it
caught by those pins (CPU only).

Each mutant is a copy of layered_oracle.c with one plausible slip (a dropped
term, a wrong sign, order or index, a wrong comparison); it is compiled to a
temporary library and run through every pin, and at least one pin must fail.
"""
import pytest

import oracle
import pins_layered
from oracle.build import SRC_LAYERED, compile_oracle


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
