"""GPU parity of the layered schedule (ldpc_decode with LDPC_LAYERED) against
the layered-schedule oracle.

The oracle visits the check rows one at a time in ascending order; the GPU
runs each layer (a maximal run of consecutive rows sharing no variable) as one
launch.  Sizes span several 64-frame chunks and a ragged tail; the full
headline batch is checked on a sample of frames (frames decode independently,
so the oracle on a sample is an exact reference for those frames).
"""
import sys

import numpy as np
import pytest

import oracle
from parity_util import TOL_LAYERED, compare
from workloads import channel, codes, configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_06545_amd as lib
    return lib


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_layered(L, handle, llr, T, es):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    bits, iters, post = L.decode(handle, t, T, early_stop=es, layered=True)
    torch.cuda.synchronize()
    return bits.cpu().numpy(), iters.cpu().numpy(), post.cpu().numpy()


def check(L, code, llr, T, es, where, sample=None, handle=None, tol=None):
    _log(f"[gpu] layered {where}: n={code.n} frames={llr.shape[0]} T={T} es={es} dtype={llr.dtype}")
    h = handle or L.Code.from_workload(code)
    bits, iters, post = gpu_layered(L, h, llr, T, es)
    idx = np.arange(llr.shape[0]) if sample is None else np.asarray(sample)
    ref = oracle.decode(code, llr[idx], T, es, nthreads=8, schedule="layered")
    if tol is None:
        tol = TOL_LAYERED[np.dtype(llr.dtype).type]
    stats = compare(ref, bits[idx], iters[idx], post[idx], llr.dtype, f"layered {where}", tol=tol)
    _log(f"[gpu] layered {where}: {stats}")
    return bits, iters, post


def test_layer_tables(L):
    q = L.Code.from_workload(configs.qc1944(2.0, frames=8).code)
    assert L.ldpc_code_layers(q) == (12, 81, 81)  # one layer per block-row
    g = L.Code.from_workload(configs.gallager504(frames=8).code)
    nl, lo, hi = L.ldpc_code_layers(g)
    assert nl > 1 and lo >= 1 and hi <= 252
    chain = L.Code.from_workload(codes.repetition_chain(7))
    assert L.ldpc_code_layers(chain) == (6, 1, 1)  # consecutive chain checks share a variable


@pytest.mark.parametrize("snr", configs.QC1944_SNRS)
def test_qc1944_small(L, snr):
    b = configs.qc1944(snr, frames=100)  # two chunks, ragged tail of 36
    check(L, b.code, b.llr, 10, False, f"qc1944 {snr}dB x100")


def test_qc1944_early_stop(L):
    b = configs.qc1944(2.0, frames=130)
    llr = channel.bpsk_awgn_llr(b.codewords, 3.5, 0.5, 911, dtype=np.float32)
    _, iters, _ = check(L, b.code, llr, 10, True, "qc1944 3.5dB early stop")
    assert iters.min() < 10


def test_qc1944_few_passes_flooding_bar(L):
    """Up to five passes the layered FP32 path meets the flooding bar (1e-4)."""
    b = configs.qc1944(2.0, frames=130)
    llr = channel.bpsk_awgn_llr(b.codewords, 3.5, 0.5, 911, dtype=np.float32)
    for T in (1, 3, 5):
        check(L, b.code, llr, T, False, f"qc1944 3.5dB {T} passes", tol=1e-4)


def test_qc1944_full_sampled(L):
    b = configs.qc1944(1.5)
    sample = np.random.default_rng(7).choice(b.llr.shape[0], 192, replace=False)
    check(L, b.code, b.llr, 10, False, "qc1944 1.5dB 4096 frames (sampled)", sample=sample)


def test_gallager504_f64(L):
    b = configs.gallager504()
    _, iters, _ = check(L, b.code, b.llr, 20, True, "gallager504 FP64")
    flood = oracle.decode(b.code, b.llr, 20, True, nthreads=8, want_trace=False)
    _log(f"[gpu] gallager504 mean iterations: layered {iters.mean():.2f}, flooding {flood['iters'].mean():.2f}")
    assert iters.mean() < 0.8 * flood["iters"].mean()


def test_gallager504_f32(L):
    b = configs.gallager504(frames=200)
    check(L, b.code, b.llr.astype(np.float32), 10, True, "gallager504 FP32")


@pytest.mark.parametrize("idx", [0, 5, 11])
def test_qc_mix_codes(L, idx):
    b = configs.qc_mix(total=1200)[idx]
    check(L, b.code, b.llr, 10, True, f"qc_mix code {idx} ({b.code.name})")


def test_small_codes_and_degenerate(L):
    rng = np.random.default_rng(3)
    for code in (codes.single_parity_check(8), codes.repetition_chain(9), codes.hamming74(),
                 codes.random_tree_code(12, 5)):
        llr = rng.normal(0.5, 1.5, size=(70, code.n)).astype(np.float32)
        for T, es in ((1, False), (6, True)):
            check(L, code, llr, T, es, f"{code.name or 'code'} m={code.m} T={T}")
    # a variable in no check and a check on one variable
    code = codes.Code.from_row_lists(3, 6, [[0, 1, 2], [3], [2, 4]])
    llr = rng.normal(0.0, 2.0, size=(65, 6)).astype(np.float32)
    check(L, code, llr, 4, False, "degree-0 column, degree-1 row")


def test_zero_iterations_and_noiseless(L):
    b = configs.qc1944(2.0, frames=70)
    bits, iters, post = gpu_layered(L, L.Code.from_workload(b.code), b.llr, 0, True)
    assert (iters == 0).all() and (bits == (b.llr < 0)).all() and np.array_equal(post, b.llr)
    llr = channel.noiseless_llr(b.codewords, 2.0).astype(np.float32)
    bits, iters, post = gpu_layered(L, L.Code.from_workload(b.code), llr, 10, True)
    assert (iters == 0).all() and (bits == b.codewords).all() and np.array_equal(post, llr)


def test_prefix_bitwise(L):
    """A run that stopped at t <= 8 gives the same outputs with max_iter 8 or 25."""
    b = configs.gallager504(frames=300)
    h = L.Code.from_workload(b.code)
    a = gpu_layered(L, h, b.llr, 8, True)
    c = gpu_layered(L, h, b.llr, 25, True)
    sel = c[1] <= 8
    assert sel.sum() > 50
    for x, y in zip(a, c):
        assert np.array_equal(x[sel], y[sel])


def _batch_vs_plain(L, items, dtype_name):
    """items: (handle, llr ndarray, T, es, layered).  One ldpc_decode_batch
    call (fused frame-resident kernel) must equal ldpc_decode of each job
    alone, bit for bit."""
    import torch
    jobs = [L.Job(h, torch.from_numpy(x).cuda(), T, early_stop=es, layered=lay) for h, x, T, es, lay in items]
    L.decode_batch(jobs)
    torch.cuda.synchronize()
    for (h, x, T, es, lay), j in zip(items, jobs):
        bits, iters, post = L.decode(h, torch.from_numpy(x).cuda(), T, early_stop=es, layered=lay)
        torch.cuda.synchronize()
        where = f"{dtype_name} layered={lay} n={x.shape[1]} frames={x.shape[0]}"
        assert np.array_equal(j.bits.cpu().numpy(), bits.cpu().numpy()), where
        assert np.array_equal(j.iters.cpu().numpy(), iters.cpu().numpy()), where
        assert np.array_equal(j.posterior.cpu().numpy(), post.cpu().numpy()), where
    return jobs


def test_batch_layered_matches_plain(L):
    """Layered and flooding jobs of several codes in one fused launch equal the
    plain path's results for each job alone."""
    mix = configs.qc_mix(total=900)
    sel = [1, 6, 10, 11]
    items = [(L.Code.from_workload(mix[i].code), mix[i].llr, 10, True, lay)
             for i, lay in zip(sel, (True, False, True, True))]
    b = configs.qc1944(2.5, frames=70)
    items.append((L.Code.from_workload(b.code), b.llr, 10, False, True))
    jobs = _batch_vs_plain(L, items, "FP32")
    # the fused layered results against the oracle too
    for (h, x, T, es, lay), j, idx in zip(items, jobs, sel + [None]):
        if not lay:
            continue
        code = mix[idx].code if idx is not None else b.code
        ref = oracle.decode(code, x, T, es, nthreads=8, schedule="layered")
        compare(ref, j.bits.cpu().numpy(), j.iters.cpu().numpy(), j.posterior.cpu().numpy(), np.float32,
                f"fused layered {code.name}", tol=TOL_LAYERED[np.float32])


def test_batch_layered_f64_csr(L):
    """FP64 layered in the fused kernel on a code without circulant structure
    (the code's layer table drives the layers)."""
    g = configs.gallager504(frames=300)
    h = L.Code.from_workload(g.code)
    jobs = _batch_vs_plain(L, [(h, g.llr, 20, True, True)], "FP64")
    ref = oracle.decode(g.code, g.llr, 20, True, nthreads=8, schedule="layered")
    compare(ref, jobs[0].bits.cpu().numpy(), jobs[0].iters.cpu().numpy(), jobs[0].posterior.cpu().numpy(),
            np.float64, "fused layered gallager504 FP64", tol=TOL_LAYERED[np.float64])


def test_batch_layered_small_codes(L):
    """Degenerate shapes through the fused layered kernel: one check, a chain
    (one row per layer), cycles, a tree, a variable in no check and a check on
    one variable; 0 and 1 iterations; all equal to the plain path."""
    rng = np.random.default_rng(5)
    items = []
    for code in (codes.single_parity_check(8), codes.repetition_chain(9), codes.hamming74(),
                 codes.random_tree_code(12, 5), codes.Code.from_row_lists(3, 6, [[0, 1, 2], [3], [2, 4]])):
        h = L.Code.from_workload(code)
        llr = rng.normal(0.4, 1.5, size=(67, code.n)).astype(np.float32)
        for T, es in ((0, False), (1, False), (7, True)):
            items.append((h, llr, T, es, True))
    _batch_vs_plain(L, items, "FP32 small codes")


def test_server_refuses_layered(L):
    pool = configs.ServePool(per_code=8)
    handles = [L.Code.from_workload(c) for c in pool.codes[:1]]
    srv = L.ldpc_server_create(handles, 1 << 22, max_inflight=1, max_group_frames=8)
    try:
        llr = np.ascontiguousarray(pool.llr_pool(0)[:1])
        bits, iters = np.zeros((1, pool.codes[0].n), np.uint8), np.zeros(1, np.int32)
        st, _ = L.ldpc_server_submit(srv, 0, 1, 10, L.LDPC_LAYERED, llr, bits, iters)
        assert st == L.LDPC_EINVAL
    finally:
        L.ldpc_server_destroy(srv)
