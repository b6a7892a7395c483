"""Comparison of GPU decoder outputs with the oracle.

Gate (per frame): the oracle's final posterior has min_n |L_n| > GATE.
  - gated frames: identical bits and identical iteration counts;
  - every frame: iteration counts equal, unless the oracle's trace shows some
    |L| <= GATE at a decision point up to the smaller count (a near-tie in a
    hard decision may legitimately flip the stop test); such excusals are
    counted and returned;
  - frames with equal counts: bits identical wherever |L_ref| > GATE, and
    |L_gpu - L_ref| <= tol * max(|L_ref|, A_n) for every bit, where
    A_n = |Lch_n| + sum_m |r_mn| is the scale of the sum forming L_n.
Tolerances: FP32 1e-4 (the bar set for the FP32 posterior).  FP64 1e-6,
derived from the oracle's own conditioning: near the clamp, 2 atanh(p) with
p = prod tanh(q/2) close to 1 loses digits in double precision (1 - p is
formed from values rounded near 1), and over 20 iterations of the Gallager
workload the FP64 oracle deviates from an 80-bit evaluation of the same
definition by up to about 1e-7 (test_oracle_precision pins this at < 1e-6).
"""
from __future__ import annotations

import numpy as np

GATE = 1e-3
TOL = {np.float32: 1e-4, np.float64: 1e-6}
# Layered schedule: every row sees the rows before it within a pass, which
# amplifies rounding differences faster than flooding does.  Injecting
# relative noise of 6e-8 (FP32 rounding) into every q, r and L update of the
# FP64 layered oracle moves posteriors of the 3.5 dB qc1944 parity input by
# about 2e-4 after 10 passes (test_oracle_layered pins this spread between
# 1e-4 and half the bar), so the FP32 bar is 1e-3 there; at five passes or
# fewer the flooding bar of 1e-4 still holds and is tested.
TOL_LAYERED = {np.float32: 1e-3, np.float64: 1e-6}
# FP32 horizons at which the bars above hold on every frame: FP32-sized
# rounding noise injected into the FP64 oracle spreads the posteriors of
# frames that never converge by at most 1e-5 after 10 flooding iterations and
# 2.3e-5 after 5 layered passes on the parity inputs, but by 2e-4 after 20
# flooding iterations and up to 0.13 after 20 layered passes on the chaotic
# ones (test_fp32_horizons pins these).  Beyond its horizon an FP32 run is
# compared in full on the frames either side stops within the horizon, and
# checked for validity on the rest (compare_horizon).
HORIZON_F32 = {"flooding": 10, "layered": 5}
# FP32 min-sum at its benchmark horizon (10 flooding iterations, qc1944 at
# 2 dB): the same noise spreads posteriors by up to 2.1e-3 (plain rule),
# so the bar there is 1e-2, with bits compared wherever |L_ref| exceeds it
# relative to A_n (test_oracle_minsum pins the spread below half of it).
TOL_MS_FLOOD10 = 1e-2


def compare(ref, bits, iters, post, dtype, where="", tol=None, rel_gate=False):
    """rel_gate: gate bits (and frames) on |L_ref| > max(GATE, tol * A_n)
    instead of |L_ref| > GATE, for bars wider than the FP32 one, where a bit
    within tol * A_n of zero may legitimately decide either way."""
    if tol is None:
        tol = TOL[np.dtype(dtype).type]
    bits = np.asarray(bits)
    iters = np.asarray(iters)
    Lr = ref["posterior"]
    A = ref["cond"]
    thr = np.maximum(GATE, tol * A) if rel_gate else GATE
    gated = (np.abs(Lr) > thr).all(axis=1)
    same_it = iters == ref["iters"]
    excused = 0
    for f in np.flatnonzero(~same_it):
        upto = int(min(iters[f], ref["iters"][f]))
        tr = ref["min_abs"][f, : upto + 1]
        assert not gated[f], f"{where}: gated frame {f} iters {iters[f]} vs oracle {ref['iters'][f]}"
        assert np.nanmin(tr) <= GATE, f"{where}: frame {f} iters {iters[f]} vs oracle {ref['iters'][f]} unexcused"
        excused += 1
    sel = same_it
    assert (bits[gated] == ref["bits"][gated]).all(), f"{where}: bit mismatch on a gated frame"
    conf = (np.abs(Lr) > thr) & sel[:, None]
    nbad = int((bits != ref["bits"])[conf].sum())
    assert nbad == 0, f"{where}: {nbad} confident bits differ"
    stats = {"frames": int(len(iters)), "gated": int(gated.sum()), "excused": excused}
    if post is not None:
        post = np.asarray(post, dtype=np.float64)
        err = np.abs(post - Lr) / np.maximum(np.maximum(np.abs(Lr), A), 1e-300)
        err = err[sel]
        worst = float(err.max()) if err.size else 0.0
        assert worst <= tol, f"{where}: posterior error {worst:.3g} > {tol}"
        stats["max_err"] = worst
    return stats


def compare_horizon(ref, bits, iters, post, dtype, where, code, max_iter, horizon, tol=None):
    """An early-stop run past the FP32 horizon: frames that either side
    stopped within `horizon` iterations are compared in full (compare);
    on the others both sides ran past the horizon, where FP32 and FP64
    trajectories of an unconverged frame may part, so only validity is
    checked: a frame that stopped before max_iter decided a codeword
    (independent dense syndrome), one that did not ran max_iter."""
    from mapref import dense_syndrome

    bits = np.asarray(bits)
    iters = np.asarray(iters)
    near = np.minimum(iters, ref["iters"]) <= horizon
    sub = {k: (v[near] if v is not None else None) for k, v in ref.items()}
    stats = compare(sub, bits[near], iters[near], None if post is None else np.asarray(post)[near], dtype, where, tol)
    far = ~near
    stopped = far & (iters < max_iter)
    assert (dense_syndrome(code, bits[stopped]) == 0).all(), f"{where}: a frame stopped on a non-codeword"
    assert (iters[far & ~stopped] == max_iter).all()
    stats.update(beyond_horizon=int(far.sum()), beyond_stopped=int(stopped.sum()))
    return stats
