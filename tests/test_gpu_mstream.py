"""GPU test of the multi-stream baseline (the paper's W workers x F frames
structure, Section III-C): every batch's outputs match the oracle (bits and
iteration counts under the parity rule; the path returns no posteriors) and
equal ldpc_decode of the same frames, bit for bit, whatever worker decoded
it; argument errors are refused before anything runs."""
import sys

import numpy as np
import pytest

import oracle
from parity_util import compare
from workloads import configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_06545_amd as lib
    return lib


@pytest.mark.parametrize("workers,frames,batches,layered", [(3, 100, 7, False), (1, 64, 2, True), (4, 33, 9, False)])
def test_mstream_matches_single_decode(L, workers, frames, batches, layered):
    import torch
    b = configs.qc1944(2.5, frames=frames * batches)
    h = L.Code.from_workload(b.code)
    llr = np.ascontiguousarray(b.llr)
    bits = np.zeros((frames * batches, b.code.n), np.uint8)
    iters = np.full(frames * batches, -1, np.int32)
    flags = L.LDPC_EARLY_STOP | (L.LDPC_LAYERED if layered else 0)
    ref = oracle.decode(b.code, llr, 10, True, nthreads=8, schedule="layered" if layered else "flooding")
    for blocking in (1, 0):
        rc, stats = L.ldpc_mstream_run(h, workers, frames, batches, 10, flags, blocking, llr, bits, iters)
        print(f"[gpu] mstream W={workers} F={frames} B={batches} blocking={blocking}: rc={rc} {stats}", flush=True)
        sys.stdout.flush()
        assert rc == 0
        assert stats["wall_ms"] > 0 and stats["cpu_ms"] >= 0
        print(f"[gpu]   oracle: {compare(ref, bits, iters, None, np.float32, 'mstream')}", flush=True)
        for k in range(batches):
            sl = slice(k * frames, (k + 1) * frames)
            rb, ri, _ = L.decode(h, torch.from_numpy(llr[sl]).cuda(), 10, early_stop=True, layered=layered,
                                 want_posterior=False)
            torch.cuda.synchronize()
            assert np.array_equal(bits[sl], rb.cpu().numpy()), f"batch {k}"
            assert np.array_equal(iters[sl], ri.cpu().numpy()), f"batch {k}"


def test_mstream_argument_errors(L):
    b = configs.qc1944(2.5, frames=8)
    h = L.Code.from_workload(b.code)
    llr = np.ascontiguousarray(b.llr)
    bits = np.zeros((8, b.code.n), np.uint8)
    iters = np.zeros(8, np.int32)
    for args in ((0, 8, 1), (65, 8, 1), (1, 0, 1), (1, 8, -1)):
        rc, _ = L.ldpc_mstream_run(h, *args, 10, 0, 1, llr, bits, iters)
        assert rc == L.LDPC_EINVAL, args
    rc, _ = L.ldpc_mstream_run(h, 1, 8, 1, 10, 8, 1, llr, bits, iters)  # unknown flag
    assert rc == L.LDPC_EINVAL
    rc, stats = L.ldpc_mstream_run(h, 2, 8, 0, 10, 0, 1, None, None, None)  # no batches: nothing to do
    assert rc == 0
