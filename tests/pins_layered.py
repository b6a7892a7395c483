"""Pins for the layered-schedule oracle: checks against what mathematics fixes,
independent of the oracle's own code.  Each check takes a decoder callable
``dec(code, llr, max_iter, early_stop) -> dict`` running the layered schedule
(check rows one at a time in ascending order, each updating its variables at
once; arxiv 1812.06545, Section II, Algorithm 2).

Layered-specific pins (each names what it fixes):
  chain_forward     path of degree-2 checks, rows in path order: after t passes
                    L_v = sum_{j <= min(n-1, v+t)} Lch_j exactly (everything to
                    the left arrives within the first pass, one more variable
                    from the right per pass).  Flooding would give the window
                    |j - v| <= t, so this pins the immediate update, the
                    extrinsic subtraction and the ascending row order.
  chain_backward    the same path with its rows listed in reverse: the mirror
                    image, L_v = sum_{j >= max(0, v-t)} Lch_j.
  tree_map          random cycle-free Tanner graphs: posterior = exact MAP
                    (brute force) after ceil(D/2) passes and later.
  row_order         rows that share no variable commute: permuting the rows
                    inside each block-row of a QC code leaves every output
                    bit-identical; swapping two block-rows that share columns
                    changes the posteriors.
  faster_than_flooding  on the (3,6) Gallager code at 2 dB with early stop the
                    mean number of passes is at most 3/4 of flooding's
                    iterations (layered decoding's faster convergence, which
                    the paper cites as its reason for the schedule).
The schedule-independent pins of ``pins`` (SPC MAP after one pass, clamp,
noiseless, zero iterations, zero posterior, symmetry, zero syndrome, prefix,
fixed iterations, stop iteration, and the conditioning output A_n and the
min |L| trace: single parity check, settled chain, bounds, truncated runs) also
hold for the layered schedule and are run against it too.
"""
from __future__ import annotations

import math

import numpy as np

import oracle
import pins
from mapref import map_llr
from workloads import codes, configs


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def permute_rows(code, order):
    """The same code with its check rows listed in `order`."""
    return codes.Code.from_dense(code.to_dense()[np.asarray(order)], name=code.name + "-perm")


def chain_forward(dec):
    for n, seed in ((4, 41), (6, 42), (9, 43)):
        code = codes.repetition_chain(n)
        llr = _rng(seed).uniform(-2.0, 2.0, size=(3, n))
        cs = np.cumsum(llr, axis=1)
        for t in range(1, n):
            want = np.stack([cs[:, min(n - 1, v + t)] for v in range(n)], axis=1)
            out = dec(code, llr, t, False)
            np.testing.assert_allclose(out["posterior"], want, rtol=1e-9, atol=1e-9,
                                       err_msg=f"chain n={n} after {t} passes")


def chain_backward(dec):
    for n, seed in ((5, 44), (8, 45)):
        code = permute_rows(codes.repetition_chain(n), np.arange(n - 2, -1, -1))
        llr = _rng(seed).uniform(-2.0, 2.0, size=(3, n))
        rs = np.cumsum(llr[:, ::-1], axis=1)[:, ::-1]  # rs[:, v] = sum_{j >= v}
        for t in range(1, n):
            want = np.stack([rs[:, max(0, v - t)] for v in range(n)], axis=1)
            out = dec(code, llr, t, False)
            np.testing.assert_allclose(out["posterior"], want, rtol=1e-9, atol=1e-9,
                                       err_msg=f"reversed chain n={n} after {t} passes")


def tree_map(dec):
    for nv, seed in ((6, 21), (9, 23), (12, 25), (14, 26), (16, 27)):
        code = codes.random_tree_code(nv, seed)
        t_exact = math.ceil(codes.tanner_vn_diameter(code) / 2)
        llr = _rng(seed + 100).uniform(-1.2, 1.2, size=(3, nv))
        ref = map_llr(code, llr)
        for t in (t_exact, t_exact + 3):
            out = dec(code, llr, t, False)
            np.testing.assert_allclose(out["posterior"], ref, rtol=1e-9, atol=1e-9,
                                       err_msg=f"tree nv={nv} after {t} passes")


def row_order(dec):
    Z, mb = 7, 4
    code = codes.qc_code(mb, 8, Z, seed=46)
    llr = _rng(47).normal(1.0, 1.2, size=(6, code.n))
    rng = _rng(48)
    inside = np.concatenate([b * Z + rng.permutation(Z) for b in range(mb)])
    base = dec(code, llr, 6, False)
    same = dec(permute_rows(code, inside), llr, 6, False)
    for key in ("bits", "iters", "posterior"):
        assert np.array_equal(base[key], same[key]), f"row permutation inside block-rows changed {key}"
    swapped = np.concatenate([np.arange(Z, 2 * Z), np.arange(0, Z), np.arange(2 * Z, mb * Z)])
    H = code.to_dense()
    assert (H[:Z].sum(axis=0) * H[Z:2 * Z].sum(axis=0)).any(), "block-rows 0 and 1 share no column"
    other = dec(permute_rows(code, swapped), llr, 6, False)
    assert np.abs(other["posterior"] - base["posterior"]).max() > 1e-6, "swapping block-rows changed nothing"


def faster_than_flooding(dec):
    b = configs.gallager504(frames=160)
    lay = dec(b.code, b.llr, 40, True)
    flood = oracle.decode(b.code, b.llr, 40, True, nthreads=4, want_trace=False)
    assert lay["iters"].mean() <= 0.75 * flood["iters"].mean(), (lay["iters"].mean(), flood["iters"].mean())


LAYERED = [chain_forward, chain_backward, tree_map, row_order, faster_than_flooding]
SHARED = [pins.spc_map, pins.clamp, pins.noiseless, pins.zero_iter, pins.zero_posterior, pins.symmetry,
          pins.zero_syndrome, pins.prefix, pins.fixed_iters, pins.stop_iteration, pins.cond_spc, pins.cond_chain,
          pins.cond_bound, pins.min_abs_trace]
ALL = LAYERED + SHARED
