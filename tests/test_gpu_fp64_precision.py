"""How close is the FP64 GPU path to the exact messages?  (GPU.)

The FP64 kernels evaluate the check rule in the phi domain,
|r| = phi(sum phi(|q|)) with phi(x) = -ln tanh(x / 2) from log1p / expm1 forms,
so each message carries a few units in the last place.  The FP64 oracle
itself loses digits near the clamp (2 atanh(p), p close to 1), which is why
the FP64 parity bar against it is 1e-6.  Here the reference is the oracle
built with its check node in 80-bit long double (the same definition, each
message rounded to double), and the FP64 GPU posteriors are held to
TOL_LD relative to max(|L|, A_n) on every frame whose iteration count
matches, with identical bits and counts on gated frames.
"""
import sys

import numpy as np
import pytest

import oracle
from parity_util import compare
from workloads import configs

pytestmark = pytest.mark.gpu

TOL_LD = 1e-9


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_06545_amd as lib
    return lib


def _run(L, code, llr, T, es, where):
    import torch
    h = L.Code.from_workload(code)
    bits, iters, post = L.decode(h, torch.from_numpy(np.ascontiguousarray(llr)).cuda(), T, early_stop=es)
    torch.cuda.synchronize()
    ld = oracle.decode(code, llr, T, es, nthreads=8, lib=oracle.long_double_lib())
    dbl = oracle.decode(code, llr, T, es, nthreads=8)
    got = (bits.cpu().numpy(), iters.cpu().numpy(), post.cpu().numpy())
    both = (ld["iters"] == dbl["iters"]) & (ld["iters"] == got[1])
    scale = np.maximum(np.abs(ld["posterior"]), ld["cond"])
    e_gpu = (np.abs(got[2] - ld["posterior"]) / scale)[both].max()
    e_dbl = (np.abs(dbl["posterior"] - ld["posterior"]) / scale)[both].max()
    print(f"[gpu] {where}: GPU FP64 vs 80-bit oracle {e_gpu:.3g}; FP64 oracle vs 80-bit oracle {e_dbl:.3g}",
          flush=True)
    sys.stdout.flush()
    stats = compare(ld, *got, np.float64, where, tol=TOL_LD)
    return e_gpu, e_dbl, stats


def test_gallager504(L):
    b = configs.gallager504(frames=600)
    _run(L, b.code, b.llr, 20, True, "gallager504 FP64 20 it")


def test_qc1944(L):
    b = configs.qc1944(2.0, frames=200)
    _run(L, b.code, b.llr.astype(np.float64), 10, False, "qc1944 FP64 10 it")
