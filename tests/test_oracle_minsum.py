"""The min-sum oracle against its pins, and planted mistakes in it caught by
those pins (CPU only).  Each mutant is a copy of minsum_oracle.c with one
plausible slip, compiled to a temporary library and run through every pin;
at least one pin must fail.  (Taking sgn(0) = -1 is no mutant: an exactly
zero incoming message makes every other message of its row zero in
magnitude, so its sign can only turn +0 into -0, which no output shows.)"""
import pytest

import oracle
import pins_minsum
from oracle.build import SRC_MINSUM, compile_oracle


def _dec(lib=None):
    def dec(code, llr, T, es, scale=1.0, offset=0.0, schedule="flooding"):
        return oracle.decode(code, llr, T, es, rule="minsum", ms_scale=scale, ms_offset=offset,
                             schedule=schedule, lib=lib)
    return dec


@pytest.mark.parametrize("check", pins_minsum.ALL, ids=lambda f: f.__name__)
def test_minsum_pin(check, oracle_mod):
    check(_dec())


MUTANTS = {
    "self_in_min": ("        if (o == e)\n            continue;\n", ""),
    "sign_dropped": ("    return negative ? -mag : mag;", "    return mag;"),
    "scale_ignored": ("    double mag = scale * mn - offset;", "    double mag = mn - offset;"),
    "offset_added": ("    double mag = scale * mn - offset;", "    double mag = scale * mn + offset;"),
    "offset_not_floored": ("    if (mag < 0.0)\n        mag = 0.0;\n", ""),
    "no_clamp": ("    if (mag > r_max)\n        mag = r_max;\n", ""),
    "flooding_no_extrinsic": ("                        q[g->col_edge[k]] = s - r[g->col_edge[k]];",
                              "                        q[g->col_edge[k]] = s;"),
    "layered_no_extrinsic": ("                        q[e] = L[g->col_idx[e]] - r[e];", "                        q[e] = L[g->col_idx[e]];"),
    "layered_message_dropped": ("                        L[g->col_idx[e]] = q[e] + r[e];",
                                "                        L[g->col_idx[e]] = q[e];"),
    "channel_dropped": ("                    double s = llr[j];", "                    double s = 0.0;"),
    "iters_off_by_one": ("                t_done = t;", "                t_done = t - 1;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_minsum_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC_MINSUM).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mpath = tmp_path / f"mut_{name}.c"
    mpath.write_text(src.replace(old, new, 1))
    lib = oracle._load(compile_oracle(str(mpath), str(tmp_path / f"libmut_{name}.so"), extra=("-Wno-error",)))
    failed = []
    for check in pins_minsum.ALL:
        try:
            check(_dec(lib))
        except (AssertionError, ValueError, FloatingPointError):
            failed.append(check.__name__)
    assert failed, f"mutant {name} passed every pin"
