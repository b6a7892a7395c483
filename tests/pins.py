"""Pins for the oracle: checks against what mathematics fixes, independent of
the oracle's own code.  Each check takes a decoder callable
``dec(code, llr, max_iter, early_stop) -> dict`` so that the same checks run
against the real oracle and against deliberately broken copies of it.

Pins (each names what it fixes):
  spc_map           single parity check, 1 iteration: posterior = exact bitwise
                    MAP (brute force), which pins the check rule (tanh product
                    over the *other* edges, factor 1/2 and 2, sign) and the
                    variable rule's channel term.
  repetition_sum    path of degree-2 checks: after n-1 iterations every
                    posterior equals the sum of all channel LLRs (the exact MAP
                    of a repetition code), and not yet after n-2 iterations;
                    pins extrinsic subtraction and the flooding schedule depth.
  tree_map          random cycle-free Tanner graphs: posterior = exact MAP once
                    t >= ceil(D/2) (D = variable-to-variable diameter), and not
                    at t = ceil(D/2) - 1.
  clamp             two-bit parity check with |L| = 30: r = 2 atanh(tanh(15)) = 30
                    is clamped to R_MAX = 20, so the posterior is 30 + 20.
  noiseless         L = A(1-2c) for a codeword c: iters 0, bits c, posterior = L.
  zero_iter         max_iter = 0: bits = [L < 0] (+0 and -0 give 0), posterior = L.
  zero_posterior    a three-bit parity check with two zero LLRs: every message
                    into those two bits is 2 atanh(0) = 0 exactly, so their
                    posteriors are exactly +0 or -0 after any iteration and the
                    decision [L < 0] gives 0 (the tie reading).
  symmetry          decoding L*(1-2c) gives bits xor c, the same iters and the
                    same |posterior| (tanh/atanh odd, signs exact).
  zero_syndrome     early stop: every frame that stopped before max_iter has
                    H bits = 0 by an independent dense product.
  prefix            a run with a larger max_iter that stopped at iters <= T
                    equals the run with max_iter T.
  fixed_iters       early stop off: iters = max_iter for every frame.
  stop_iteration    with early stop, iters is the first t whose hard decision
                    (taken from the early-stop-off run truncated at t) has a
                    zero syndrome by an independent dense product, else T.
  cond_spc          the conditioning output A_n = |Lch_n| + sum_m |r_mn| on a
                    single parity check, whose one message is the exact MAP
                    value minus the channel term (brute force), clamp included.
  cond_chain        A_n on a repetition chain once every message has settled:
                    the two messages into variable j are the sums of the
                    channel LLRs on either side of it, so
                    A_j = |Lch_j| + |sum_{i<j} Lch_i| + |sum_{i>j} Lch_i|
                    (mixed signs, so a dropped absolute value or a wrong
                    column shows).
  cond_bound        on noisy frames: |Lch| <= A, |posterior| <= A (triangle
                    inequality) and A - |Lch| <= degree * R_MAX.
  min_abs_trace     the trace min_n |L_n| at decision point t equals that of
                    the early-stop-off run truncated at t, for t <= iters;
                    NaN after the frame stopped; t = 0 is min |Lch|.
  hamming_first_iteration  Hamming(7,4) (a graph with 4-cycles): after one
                    iteration the posterior of every bit equals exact MAP on
                    its depth-1 computation tree (brute force), for all 112
                    single-error patterns at |L| = 1.5, 2, 3 and random LLRs.
  hamming_regression  Hamming(7,4), all 112 single-error patterns, 20
                    iterations with early stop, against exact MAP of the code:
                    |L| = 2: every pattern is corrected within 2 iterations;
                    |L| = 3 and 4: an error on the weight-3 column is turned,
                    in iteration 1, into the weight-3 codeword that the
                    depth-1 tree MAP decisions predict (MAP corrects it), the
                    other patterns are corrected; |L| = 1.5: errors on weight-1
                    and weight-2 columns never clear the syndrome (20
                    iterations), while an error on the weight-3 column is
                    corrected in iteration 1.  Beyond iteration 1 these are
                    regression values of the decoding dynamics on a graph
                    with cycles (no closed form).
"""
from __future__ import annotations

import math

import numpy as np

from workloads import channel, codes, configs
from mapref import all_codewords, dense_syndrome, depth1_tree, map_llr

R_MAX = 20.0


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def spc_map(dec):
    for n, seed in ((2, 1), (3, 2), (5, 3), (8, 4), (12, 5)):
        code = codes.single_parity_check(n)
        llr = _rng(seed).normal(0.0, 1.5, size=(6, n))
        ref = map_llr(code, llr)
        for T in (1, 3):
            out = dec(code, llr, T, False)
            np.testing.assert_allclose(out["posterior"], ref, rtol=1e-12, atol=1e-12,
                                       err_msg=f"SPC n={n} T={T}")


def repetition_sum(dec):
    for n, seed in ((4, 11), (6, 12), (9, 13)):
        code = codes.repetition_chain(n)
        llr = _rng(seed).uniform(-2.0, 2.0, size=(4, n))
        total = llr.sum(axis=1, keepdims=True) * np.ones((1, n))
        np.testing.assert_allclose(map_llr(code, llr), total, rtol=1e-12, atol=1e-12)
        out = dec(code, llr, n - 1, False)
        np.testing.assert_allclose(out["posterior"], total, rtol=1e-9, atol=1e-9,
                                   err_msg=f"repetition n={n} after n-1 iterations")
        early = dec(code, llr, n - 2, False)
        assert np.abs(early["posterior"] - total).max() > 1e-3, "repetition exact too early"


def tree_map(dec):
    checked = 0
    for nv, seed in ((6, 21), (8, 22), (9, 23), (11, 24), (12, 25), (14, 26)):
        code = codes.random_tree_code(nv, seed)
        D = codes.tanner_vn_diameter(code)
        t_exact = math.ceil(D / 2)
        llr = _rng(seed + 100).uniform(-1.2, 1.2, size=(3, nv))
        ref = map_llr(code, llr)
        out = dec(code, llr, t_exact, False)
        np.testing.assert_allclose(out["posterior"], ref, rtol=1e-9, atol=1e-9,
                                   err_msg=f"tree nv={nv} D={D} at t={t_exact}")
        later = dec(code, llr, t_exact + 3, False)
        np.testing.assert_allclose(later["posterior"], ref, rtol=1e-9, atol=1e-9)
        if t_exact >= 2:
            before = dec(code, llr, t_exact - 1, False)
            assert np.abs(before["posterior"] - ref).max() > 1e-6, f"tree nv={nv} exact too early"
            checked += 1
    assert checked >= 3


def clamp(dec):
    code = codes.single_parity_check(2)
    llr = np.array([[30.0, 30.0], [-30.0, 30.0], [3.0, 30.0]])
    out = dec(code, llr, 1, False)
    want = np.array([[50.0, 50.0], [-30.0 + 20.0, 30.0 - 20.0], [3.0 + 20.0, 30.0 + 3.0]])
    np.testing.assert_allclose(out["posterior"], want, rtol=1e-9, atol=1e-9)


def _gallager_noisy(frames, seed, ebn0=2.0):
    code = configs.gallager504(frames=frames).code
    cw = configs.gallager504(frames=frames).codewords
    llr = channel.bpsk_awgn_llr(cw, ebn0, 0.5, seed, dtype=np.float64)
    return code, cw, llr


def noiseless(dec):
    code, cw, _ = _gallager_noisy(8, 31)
    for A in (0.5, 3.0):
        llr = channel.noiseless_llr(cw, A)
        out = dec(code, llr, 20, True)
        assert (out["iters"] == 0).all()
        assert (out["bits"] == cw).all()
        assert (out["posterior"] == llr).all()


def zero_iter(dec):
    code, cw, llr = _gallager_noisy(4, 32)
    llr = llr.copy()
    llr[0, :4] = [0.0, -0.0, -1e-300, 1e-300]
    for es in (False, True):
        out = dec(code, llr, 0, es)
        assert (out["iters"] == 0).all()
        assert (out["bits"] == (llr < 0)).all()
        assert (out["posterior"] == llr).all()
    assert list(out["bits"][0, :4]) == [0, 0, 1, 0]


def zero_posterior(dec):
    code = codes.single_parity_check(3)
    llr = np.array([[1.5, 0.0, 0.0], [-1.5, -0.0, -0.0], [0.7, 0.0, -0.0]])
    for T in (1, 2):
        out = dec(code, llr, T, False)
        assert (out["posterior"][:, 1:] == 0.0).all(), out["posterior"]
        assert (out["bits"][:, 1:] == 0).all(), f"a zero posterior decided as 1 after {T} iterations"


def symmetry(dec):
    code, cw, llr = _gallager_noisy(12, 33, ebn0=1.5)
    base = dec(code, llr, 20, True)
    cw2 = configs.gallager504(frames=24).codewords[12:24]
    flipped = llr * (1.0 - 2.0 * cw2)
    out = dec(code, flipped, 20, True)
    assert (out["bits"] == (base["bits"] ^ cw2)).all()
    assert (out["iters"] == base["iters"]).all()
    assert (np.abs(out["posterior"]) == np.abs(base["posterior"])).all()


def zero_syndrome(dec):
    code, cw, llr = _gallager_noisy(40, 34)
    out = dec(code, llr, 20, True)
    stopped = out["iters"] < 20
    assert stopped.sum() >= 20
    assert (dense_syndrome(code, out["bits"][stopped]) == 0).all()


def prefix(dec):
    code, cw, llr = _gallager_noisy(30, 35, ebn0=1.5)
    a = dec(code, llr, 8, True)
    b = dec(code, llr, 25, True)
    sel = b["iters"] <= 8
    assert sel.sum() >= 5
    assert (a["iters"][sel] == b["iters"][sel]).all()
    assert (a["bits"][sel] == b["bits"][sel]).all()
    assert (a["posterior"][sel] == b["posterior"][sel]).all()


def fixed_iters(dec):
    code, cw, llr = _gallager_noisy(10, 36)
    out = dec(code, llr, 7, False)
    assert (out["iters"] == 7).all()


def stop_iteration(dec):
    code, cw, llr = _gallager_noisy(24, 37, ebn0=1.8)
    T = 12
    es = dec(code, llr, T, True)
    first = np.full(llr.shape[0], T)
    for t in range(T, -1, -1):
        bits_t = dec(code, llr, t, False)["bits"]
        ok = (dense_syndrome(code, bits_t) == 0).all(axis=1)
        first[ok] = t
    assert len(set(first.tolist())) >= 3
    assert (es["iters"] == first).all()


def cond_spc(dec):
    for n, seed in ((3, 63), (6, 64)):
        code = codes.single_parity_check(n)
        llr = _rng(seed).normal(0.0, 2.0, size=(5, n))
        r = map_llr(code, llr) - llr  # the check's message (Gallager's lemma)
        for T in (1, 2):
            out = dec(code, llr, T, False)
            np.testing.assert_allclose(out["cond"], np.abs(llr) + np.abs(r), rtol=1e-9, atol=1e-9,
                                       err_msg=f"A_n on SPC n={n} T={T}")
    out = dec(codes.single_parity_check(2), np.array([[30.0, 30.0], [-30.0, 30.0]]), 1, False)
    np.testing.assert_allclose(out["cond"], np.full((2, 2), 50.0), rtol=1e-12, atol=1e-12)


def cond_chain(dec):
    for n, seed in ((5, 61), (8, 62)):
        code = codes.repetition_chain(n)
        llr = _rng(seed).uniform(-2.0, 2.0, size=(4, n))
        cs = np.cumsum(llr, axis=1)
        left = cs - llr                      # sum_{i<j}
        right = cs[:, -1:] - cs              # sum_{i>j}
        want = np.abs(llr) + np.abs(left) + np.abs(right)
        assert (np.abs(left + llr + right) < want - 1e-3).any(), "inputs of one sign test nothing"
        out = dec(code, llr, n + 2, False)
        np.testing.assert_allclose(out["cond"], want, rtol=1e-9, atol=1e-9, err_msg=f"A_n on chain n={n}")


def cond_bound(dec):
    code, cw, llr = _gallager_noisy(12, 38, ebn0=1.5)
    out = dec(code, llr, 7, False)
    A = out["cond"]
    assert (A >= np.abs(llr)).all()
    assert (np.abs(out["posterior"]) <= A * (1 + 1e-12)).all()
    assert (A - np.abs(llr) <= code.col_degrees() * R_MAX * (1 + 1e-12)).all()
    assert (A > np.abs(out["posterior"]) * (1 + 1e-6)).any(), "no cancellation anywhere: the bound tests nothing"


def min_abs_trace(dec):
    code, cw, llr = _gallager_noisy(16, 39, ebn0=1.8)
    T = 10
    es = dec(code, llr, T, True)
    tr = es["min_abs"]
    assert tr.shape == (llr.shape[0], T + 1)
    assert (es["iters"] < T).sum() >= 3 and (es["iters"] >= 2).sum() >= 3
    np.testing.assert_array_equal(tr[:, 0], np.abs(llr).min(axis=1))
    for t in range(1, T + 1):
        want = np.abs(dec(code, llr, t, False)["posterior"]).min(axis=1)
        ran = es["iters"] >= t
        np.testing.assert_array_equal(tr[ran, t], want[ran], err_msg=f"min |L| trace at t={t}")
        assert np.isnan(tr[~ran, t]).all(), f"trace entry after the stop at t={t}"
    fixed = dec(code, llr, T, False)
    np.testing.assert_array_equal(fixed["min_abs"][:, T], np.abs(fixed["posterior"]).min(axis=1))


def _hamming_single_errors(A):
    """Every codeword of Hamming(7,4) at reliability A with one bit's sign
    flipped: (codewords, flipped positions, LLRs), 112 frames."""
    code = codes.hamming74()
    cw = all_codewords(code)
    C = np.repeat(cw, 7, axis=0)
    P = np.tile(np.arange(7), len(cw))
    llr = A * (1.0 - 2.0 * C.astype(np.float64))
    llr[np.arange(len(P)), P] *= -1.0
    return code, C, P, llr


def hamming_first_iteration(dec):
    trees = [depth1_tree(codes.hamming74(), j) for j in range(7)]
    inputs = [_hamming_single_errors(A)[3] for A in (1.5, 2.0, 3.0)]
    inputs.append(_rng(65).normal(0.5, 1.5, size=(20, 7)))
    for llr in inputs:
        out = dec(codes.hamming74(), llr, 1, False)
        for j, (tree, src) in enumerate(trees):
            want = map_llr(tree, llr[:, src])[:, 0]
            np.testing.assert_allclose(out["posterior"][:, j], want, rtol=1e-9, atol=1e-9,
                                       err_msg=f"Hamming(7,4) bit {j} after one iteration")


def hamming_regression(dec):
    weight = codes.hamming74().to_dense().sum(axis=0)
    for A in (1.5, 2.0, 3.0, 4.0):
        code, C, P, llr = _hamming_single_errors(A)
        map_bits = (map_llr(code, llr) < 0).astype(np.uint8)
        assert (map_bits == C).all(), "MAP corrects every single error"
        out = dec(code, llr, 20, True)
        ok = (out["bits"] == C).all(axis=1)
        w = weight[P]
        if A == 2.0:
            assert ok.all() and (out["iters"] <= 2).all(), f"|L|=2: {out['iters']}"
        elif A >= 3.0:
            assert ok[w < 3].all() and (out["iters"][w < 3] <= 2).all()
            sel = np.flatnonzero(w == 3)
            # iteration 1 by the depth-1 tree MAP of every bit, then the decision
            trees = [depth1_tree(code, j) for j in range(7)]
            post1 = np.stack([map_llr(t, llr[sel][:, s])[:, 0] for t, s in trees], axis=1)
            pred = (post1 < 0).astype(np.uint8)
            assert (dense_syndrome(code, pred) == 0).all()
            assert ((pred ^ C[sel]).sum(axis=1) == 3).all(), "the predicted word is a weight-3 neighbour"
            assert (out["iters"][sel] == 1).all() and (out["bits"][sel] == pred).all(), f"|L|={A} weight-3 column"
        else:
            assert (~ok[w < 3]).all() and (out["iters"][w < 3] == 20).all(), f"|L|=1.5: {out['iters']}"
            assert ok[w == 3].all() and (out["iters"][w == 3] == 1).all()


ALL = [spc_map, repetition_sum, tree_map, clamp, noiseless, zero_iter, zero_posterior, symmetry, zero_syndrome,
       prefix, fixed_iters, stop_iteration, cond_spc, cond_chain, cond_bound, min_abs_trace, hamming_first_iteration,
       hamming_regression]
