"""Pins for the min-sum oracle (both schedules): checks against what
mathematics fixes, independent of the oracle's own code.  Each check takes a
decoder callable ``dec(code, llr, max_iter, early_stop, scale=1.0,
offset=0.0, schedule="flooding") -> dict``.

Min-sum-specific pins (each names what it fixes):
  spc_closed_form   one parity check, one iteration, several scales and
                    offsets: L_n = Lch_n + s_n * clamp(max(scale * m_n - offset,
                    0)), m_n the smallest |Lch_j| over j != n and s_n the sign
                    product of the others, computed here directly; pins the
                    exclusive minimum, the sign rule, scale, offset and clamp.
  tree_maxlog       random cycle-free Tanner graphs, plain min-sum: the
                    posterior equals the max-log MAP value by enumeration,
                    max_{c: c_n=0} M(c) - max_{c: c_n=1} M(c) with
                    M(c) = sum_j (1 - 2 c_j) Lch_j / 2, after ceil(D/2)
                    iterations (flooding, and not one iteration earlier) or
                    passes (layered); min-sum is max-product on a tree.
  chain_sums        degree-2 checks pass their input through exactly, so the
                    path code gives the repetition sums: flooding after n-1
                    iterations, layered with the window sum_{j <= v+t}.
  homogeneous       plain min-sum is positively homogeneous: decoding 2 Lch
                    gives exactly twice the posterior (no term like phi may
                    sneak in); with an offset it is not.
The schedule-independent pins of ``pins`` that hold for any check rule
(clamp, noiseless, zero iterations, zero posterior, symmetry, zero syndrome,
prefix, fixed iterations, stop iteration) run too, for both schedules.
"""
from __future__ import annotations

import math

import numpy as np

import pins
from mapref import all_codewords
from workloads import codes


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def maxlog_llr(code, llr):
    """Max-log MAP value of every bit by enumeration of the codewords."""
    cws = all_codewords(code).astype(np.float64)
    out = np.zeros_like(llr, dtype=np.float64)
    for f in range(llr.shape[0]):
        metric = ((1.0 - 2.0 * cws) * llr[f]).sum(axis=1) / 2.0
        for j in range(code.n):
            out[f, j] = metric[cws[:, j] == 0].max() - metric[cws[:, j] == 1].max()
    return out


def spc_closed_form(dec):
    for n, seed in ((2, 51), (3, 52), (6, 53), (11, 54)):
        code = codes.single_parity_check(n)
        llr = _rng(seed).normal(0.0, 3.0, size=(5, n))
        llr[0, 0] = 25.0  # a message that reaches the clamp
        for scale, offset in ((1.0, 0.0), (0.75, 0.0), (1.0, 0.5), (0.8125, 0.25)):
            want = np.empty_like(llr)
            for f in range(llr.shape[0]):
                for k in range(n):
                    others = np.delete(llr[f], k)
                    if others.size == 0:
                        mag, neg = 20.0, False
                    else:
                        mag = min(max(scale * np.abs(others).min() - offset, 0.0), 20.0)
                        neg = bool((others < 0).sum() % 2)
                    want[f, k] = llr[f, k] + (-mag if neg else mag)
            for sched in ("flooding", "layered"):
                out = dec(code, llr, 1, False, scale=scale, offset=offset, schedule=sched)
                np.testing.assert_allclose(out["posterior"], want, rtol=0, atol=1e-12,
                                           err_msg=f"SPC n={n} scale={scale} offset={offset} {sched}")
                # A_n = |Lch_n| + |r_n|, the message being the posterior minus the channel term
                np.testing.assert_allclose(out["cond"], np.abs(llr) + np.abs(want - llr), rtol=0, atol=1e-12,
                                           err_msg=f"A_n on SPC n={n} scale={scale} offset={offset} {sched}")


def tree_maxlog(dec):
    for nv, seed in ((6, 21), (9, 23), (12, 25), (14, 26)):
        code = codes.random_tree_code(nv, seed)
        t_exact = math.ceil(codes.tanner_vn_diameter(code) / 2)
        llr = _rng(seed + 200).uniform(-1.5, 1.5, size=(3, nv))
        ref = maxlog_llr(code, llr)
        for sched in ("flooding", "layered"):
            for t in (t_exact, t_exact + 2):
                out = dec(code, llr, t, False, schedule=sched)
                np.testing.assert_allclose(out["posterior"], ref, rtol=0, atol=1e-12,
                                           err_msg=f"tree nv={nv} {sched} t={t}")
        if t_exact >= 2:
            early = dec(code, llr, t_exact - 1, False, schedule="flooding")
            assert np.abs(early["posterior"] - ref).max() > 1e-6, f"tree nv={nv} max-log exact too early"


def chain_sums(dec):
    for n, seed in ((5, 55), (8, 56)):
        code = codes.repetition_chain(n)
        llr = _rng(seed).uniform(-2.0, 2.0, size=(3, n))
        total = llr.sum(axis=1, keepdims=True) * np.ones((1, n))
        out = dec(code, llr, n - 1, False, schedule="flooding")
        np.testing.assert_allclose(out["posterior"], total, rtol=0, atol=1e-12, err_msg=f"chain n={n} flooding")
        cs = np.cumsum(llr, axis=1)
        for t in (1, 2, n - 1):
            want = np.stack([cs[:, min(n - 1, v + t)] for v in range(n)], axis=1)
            out = dec(code, llr, t, False, schedule="layered")
            np.testing.assert_allclose(out["posterior"], want, rtol=0, atol=1e-12,
                                       err_msg=f"chain n={n} layered t={t}")


def homogeneous(dec):
    code = codes.qc_code(4, 8, 5, seed=57)
    llr = _rng(58).normal(0.5, 1.0, size=(6, code.n))
    for sched in ("flooding", "layered"):
        a = dec(code, llr, 5, False, schedule=sched)
        b = dec(code, 2.0 * llr, 5, False, schedule=sched)
        assert np.array_equal(b["posterior"], 2.0 * a["posterior"]), f"min-sum not homogeneous ({sched})"
        assert np.array_equal(a["bits"], b["bits"])
        c = dec(code, llr, 5, False, offset=0.5, schedule=sched)
        d = dec(code, 2.0 * llr, 5, False, offset=0.5, schedule=sched)
        assert not np.allclose(d["posterior"], 2.0 * c["posterior"]), f"offset had no effect ({sched})"


def _both(check, scale=1.0):
    """A schedule-independent pin of ``pins`` run for both schedules.  Pins
    that need frames to converge within a few iterations at their fixed
    inputs use the normalised rule (scale 0.75): plain min-sum converges
    more slowly than sum-product at the same Eb/N0."""
    def run(dec):
        for sched in ("flooding", "layered"):
            check(lambda code, llr, T, es: dec(code, llr, T, es, scale=scale, schedule=sched))
    run.__name__ = check.__name__ + ("" if scale == 1.0 else f"_scale{scale}")
    return run


MINSUM = [spc_closed_form, tree_maxlog, chain_sums, homogeneous]
SHARED = ([_both(c) for c in (pins.clamp, pins.noiseless, pins.zero_iter, pins.zero_posterior, pins.symmetry,
                              pins.zero_syndrome, pins.fixed_iters, pins.stop_iteration)]
          + [_both(c, 0.75) for c in (pins.zero_syndrome, pins.prefix, pins.stop_iteration, pins.min_abs_trace)]
          + [_both(c) for c in (pins.cond_chain, pins.cond_bound)])
ALL = MINSUM + SHARED
