"""GPU parity of the plain per-iteration path (ldpc_decode) against the oracle.

Every test calls the HIP kernels through the C ABI (via the thin binding)
and compares with the oracle on the same seeded inputs; sizes span several
64-frame chunks and a ragged tail, and the full workloads are checked on
sampled frames (the oracle decodes frames independently, so a sample of
frames is an exact reference for those frames).
"""
import sys

import numpy as np
import pytest

import oracle
from parity_util import compare
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


def gpu_decode(L, code_handle, llr, T, es, want_post=True):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    bits, iters, post = L.decode(code_handle, t, T, early_stop=es, want_posterior=want_post)
    torch.cuda.synchronize()
    return bits.cpu().numpy(), iters.cpu().numpy(), (post.cpu().numpy() if post is not None else None)


def run_and_compare(L, code, llr, T, es, where, sample=None, handle=None):
    _log(f"[gpu] {where}: n={code.n} frames={llr.shape[0]} T={T} es={es} dtype={llr.dtype}")
    h = handle or L.Code.from_workload(code)
    bits, iters, post = gpu_decode(L, h, llr, T, es)
    idx = np.arange(llr.shape[0]) if sample is None else np.asarray(sample)
    ref = oracle.decode(code, llr[idx], T, es, nthreads=8)
    stats = compare(ref, bits[idx], iters[idx], post[idx], llr.dtype, where)
    _log(f"[gpu] {where}: {stats}")
    return bits, iters, post, stats


@pytest.mark.parametrize("snr", configs.QC1944_SNRS)
def test_qc1944_small(L, snr):
    b = configs.qc1944(snr, frames=100)  # two chunks, ragged tail of 36
    run_and_compare(L, b.code, b.llr, 10, False, f"qc1944 {snr}dB x100")


def test_qc1944_small_early_stop(L):
    b = configs.qc1944(2.0, frames=130)
    llr = channel.bpsk_awgn_llr(b.codewords, 4.0, 0.5, 901, dtype=np.float32)
    _, iters, _, _ = run_and_compare(L, b.code, llr, 10, True, "qc1944 4dB early stop")
    assert iters.min() < 10


def test_qc1944_csr_layout_same_as_qc(L):
    """The same matrix given as CSR or as circulant shifts decodes identically."""
    b = configs.qc1944(1.5, frames=64)
    hq = L.Code.from_workload(b.code)
    hc = L.Code.from_csr(b.code.m, b.code.n, b.code.row_ptr, b.code.col_idx)
    a = gpu_decode(L, hq, b.llr, 10, False)
    c = gpu_decode(L, hc, b.llr, 10, False)
    for x, y in zip(a, c):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("snr", configs.QC1944_SNRS)
def test_qc1944_full_sampled(L, snr):
    b = configs.qc1944(snr)
    rng = np.random.default_rng(7)
    sample = np.unique(np.concatenate([[0, 63, 64, 4095], rng.choice(4096, 20, replace=False)]))
    run_and_compare(L, b.code, b.llr, 10, False, f"qc1944 {snr}dB full", sample=sample)


def test_gallager504_f64(L):
    b = configs.gallager504()
    _, iters, _, stats = run_and_compare(L, b.code, b.llr, b.max_iter, True, "gallager504 f64")
    assert stats["excused"] <= 5
    assert 5 < iters.mean() < 15


def test_gallager504_f32(L):
    b = configs.gallager504(frames=300)
    run_and_compare(L, b.code, b.llr.astype(np.float32), 20, True, "gallager504 f32")


def test_stair64800_sampled(L):
    b = configs.stair64800()
    sample = [0, 77, 128, 255]
    _, iters, _, _ = run_and_compare(L, b.code, b.llr, b.max_iter, True, "stair64800", sample=sample)
    assert iters.max() <= 50


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_small_codes(L, dtype):
    rng = np.random.default_rng(11)
    paper = np.loadtxt(__file__.replace("test_gpu_stream.py", "golden/paper_eq1_H.txt"), dtype=np.uint8)
    cases = [codes.single_parity_check(5), codes.repetition_chain(7), codes.hamming74(),
             codes.random_tree_code(12, 3), codes.Code.from_dense(paper)]
    for code in cases:
        llr = rng.normal(1.0, 1.5, size=(70, code.n)).astype(dtype)
        for es in (False, True):
            run_and_compare(L, code, llr, 8, es, f"{code.name or 'eq1'} es={es}")


def test_degenerate_graph(L):
    """Empty row, empty column, a degree-1 check and a degree-24 check."""
    rows = [[], [0], [1, 2, 3], list(range(4, 28)), [2, 5, 9]]
    code = codes.Code.from_row_lists(len(rows), 30, rows, "degenerate")
    rng = np.random.default_rng(5)
    llr = rng.normal(0.5, 2.0, size=(65, 30)).astype(np.float32)
    for es in (False, True):
        for T in (0, 1, 6):
            run_and_compare(L, code, llr, T, es, f"degenerate T={T} es={es}")


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_noiseless_and_zero_iterations(L, dtype):
    b = configs.qc1944(2.0, frames=70)
    h = L.Code.from_workload(b.code)
    llr = channel.noiseless_llr(b.codewords, 2.5, dtype)
    bits, iters, post = gpu_decode(L, h, llr, 10, True)
    assert (iters == 0).all() and (bits == b.codewords).all() and np.array_equal(post, llr)
    noisy = b.llr.astype(dtype)
    for es in (False, True):
        bits, iters, post = gpu_decode(L, h, noisy, 0, es)
        assert (iters == 0).all() and (bits == (noisy < 0)).all() and np.array_equal(post, noisy)


def test_codeword_symmetry(L):
    b = configs.qc1944(1.5, frames=96)
    h = L.Code.from_workload(b.code)
    cw2 = configs.qc1944(1.5, frames=192).codewords[96:]
    flipped = (b.llr * (1.0 - 2.0 * cw2)).astype(np.float32)
    bits0, it0, p0 = gpu_decode(L, h, b.llr, 10, False)
    bits1, it1, p1 = gpu_decode(L, h, flipped, 10, False)
    assert np.array_equal(bits1, bits0 ^ cw2)
    assert np.array_equal(it0, it1)
    assert np.array_equal(np.abs(p0), np.abs(p1))


def test_deterministic(L):
    b = configs.qc1944(1.0, frames=200)
    h = L.Code.from_workload(b.code)
    a = gpu_decode(L, h, b.llr, 10, True)
    c = gpu_decode(L, h, b.llr, 10, True)
    for x, y in zip(a, c):
        assert np.array_equal(x, y)


def test_frames_zero_and_errors(L):
    import torch
    b = configs.qc1944(2.0, frames=64)
    h = L.Code.from_workload(b.code)
    llr = torch.from_numpy(b.llr).cuda()
    bits = torch.full((64, b.code.n), 7, dtype=torch.uint8, device="cuda")
    iters = torch.full((64,), -7, dtype=torch.int32, device="cuda")
    need = L.ldpc_workspace_bytes(h.handle, torch.float32, 64, 10)
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    assert L.ldpc_decode(h.handle, torch.float32, 0, 10, 0, llr, bits, iters, None, ws, need) == L.LDPC_OK
    assert L.ldpc_decode(h.handle, torch.float32, 64, 10, 0, llr, bits, iters, None, ws, need - 1) == L.LDPC_EINVAL
    assert L.ldpc_decode(h.handle, torch.float32, 64, 10, 8, llr, bits, iters, None, ws, need) == L.LDPC_EINVAL
    assert L.ldpc_decode(h.handle, torch.float32, 64, -1, 0, llr, bits, iters, None, ws, need) == L.LDPC_EINVAL
    assert L.ldpc_decode(h.handle, torch.float32, 64, 10, 0, None, bits, iters, None, ws, need) == L.LDPC_EINVAL
    misaligned = ws.data_ptr() + 16
    assert L.ldpc_decode(h.handle, torch.float32, 64, 10, 0, llr, bits, iters, None, misaligned,
                         need) == L.LDPC_EINVAL
    torch.cuda.synchronize()
    assert (bits == 7).all() and (iters == -7).all()


def test_batch_matches_single(L):
    import torch
    mix = configs.qc_mix(total=600)
    jobs, singles = [], []
    for bt in mix:
        h = L.Code.from_workload(bt.code)
        llr = torch.from_numpy(bt.llr).cuda()
        jobs.append(L.Job(h, llr, 10, early_stop=True))
        singles.append(gpu_decode(L, h, bt.llr, 10, True))
    L.decode_batch(jobs)
    torch.cuda.synchronize()
    for j, s in zip(jobs, singles):
        assert np.array_equal(j.bits.cpu().numpy(), s[0])
        assert np.array_equal(j.iters.cpu().numpy(), s[1])
        assert np.array_equal(j.posterior.cpu().numpy(), s[2])
