"""GPU parity against the oracle for every kernel body the library
instantiates, on codes chosen for their row and column degrees.

The kernels are compiled per degree bucket: exact straight-line check-row
bodies for FP32 rows of degree 1..32 (buckets 8/16/24/32), a guarded body for
rows of degree 33..64, FP64 buckets 8/16/32/64, min-sum buckets 8/16/32/64,
the same for the layered schedule, and the fused frame-resident kernel's FP32
buckets 8/16/24/32 and FP64 buckets 8/16/32 (rows of degree <= 32; wider
codes are routed to the plain path).  Column bodies are exact up to degree 16
and a loop beyond.  The codes here reach every one of these:

  qc_d16      QC, block-row degrees 16 14 12 10 9 9, Z = 27 (FP64 bucket 16)
  qc_d24      QC, block-row degrees 24 22 20 18 17, Z = 27 (FP32 bucket 24)
  qc_d32      QC with a dense block-row: degrees 32 30 28 26 25 20, Z = 27
  qc_d64      QC, block-row degrees 64 57 48 40 33, Z = 11 (degree 33..64)
  csr_d25_32  CSR rows of degree 25..32 and one column in every row (degree 40)
  csr_d33_64  CSR rows of degree 33..63 and one column of degree 24
  spc30/40/64 single parity checks of 30, 40 and 64 bits

Inputs are random codewords (GF(2) encoder of H) through BPSK/AWGN at an
Eb/N0 where some frames converge within the horizon and some do not; 200
frames (three 64-frame chunks and a ragged tail of 8).

Bars (tests/parity_util.py): flooding FP32 1e-4 and FP64 1e-6; layered FP32
1e-4 and FP64 1e-6; min-sum FP64 bit for bit, FP32 1e-4 up to 4 iterations
(flooding) or 1 pass (layered); the fused kernel equal to the plain path bit
for bit.  FP32 runs are compared in full up to the FP32 horizon (10 flooding
iterations, 5 layered passes; test_fp32_horizons pins the rounding spread of
these inputs there), and 20-iteration early-stop runs in full on the frames
that stop within it, with validity checked on the rest (compare_horizon).
"""
import sys

import numpy as np
import pytest

import oracle
from degree_cases import FRAMES, FUSED_FITS, NAMES, workload
from parity_util import HORIZON_F32, compare, compare_horizon
from workloads import configs

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_06545_amd as lib
    return lib


@pytest.fixture(scope="module")
def handles(L):
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = L.Code.from_workload(workload(name, "f64")[0])
        return cache[name]
    return get


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _np(*ts):
    return tuple(None if t is None else t.cpu().numpy() for t in ts)


def gpu_plain(L, h, llr, T, es, layered=False, rule="spa", scale=1.0):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    out = L.decode(h, x, T, early_stop=es, layered=layered, rule=rule, ms_scale=scale)
    torch.cuda.synchronize()
    return _np(*out)


def test_codes_reach_every_bucket(L, handles):
    """The degree profile each case is meant to have."""
    import torch
    want_max = {"qc_d16": 16, "qc_d24": 24, "qc_d32": 32, "qc_d64": 64, "spc30": 30, "spc40": 40, "spc64": 64}
    for name in NAMES:
        code, _ = workload(name, "f64")
        m, n, e = L.ldpc_code_info(handles(name))
        assert (m, n, e) == (code.m, code.n, code.edges)
        dmax = int(code.row_degrees().max())
        if name in want_max:
            assert dmax == want_max[name], name
        fits32, _ = L.ldpc_batch_fits_fused(handles(name), torch.float32)
        fits64, _ = L.ldpc_batch_fits_fused(handles(name), torch.float64)
        assert fits32 == fits64 == (name in FUSED_FITS), name
    assert workload("csr_d25_32", "f64")[0].col_degrees().max() == 40  # column loop beyond 16


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("name", NAMES)
def test_flooding(L, handles, name, dtype):
    code, llr = workload(name, dtype)
    for T, es in ((20, True), (10, False)):
        _log(f"[gpu] flooding {name} {dtype} T={T} es={es}")
        bits, iters, post = gpu_plain(L, handles(name), llr, T, es)
        ref = oracle.decode(code, llr, T, es, nthreads=8)
        where = f"flooding {name} {dtype} T={T}"
        if dtype == "f32" and T > HORIZON_F32["flooding"]:
            stats = compare_horizon(ref, bits, iters, post, llr.dtype, where, code, T, HORIZON_F32["flooding"])
        else:
            stats = compare(ref, bits, iters, post, llr.dtype, where)
        _log(f"[gpu]   {stats}, mean iters {iters.mean():.2f}")
        if es:
            assert 0 < (iters < T).sum() < FRAMES or name.startswith("spc"), "inputs should mix stops and non-stops"


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("name", NAMES)
def test_layered(L, handles, name, dtype):
    code, llr = workload(name, dtype)
    for T, es in ((5, False), (20, True)):
        _log(f"[gpu] layered {name} {dtype} T={T} es={es}")
        bits, iters, post = gpu_plain(L, handles(name), llr, T, es, layered=True)
        ref = oracle.decode(code, llr, T, es, nthreads=8, schedule="layered")
        where = f"layered {name} {dtype} T={T}"
        if dtype == "f32" and T > HORIZON_F32["layered"]:
            stats = compare_horizon(ref, bits, iters, post, llr.dtype, where, code, T, HORIZON_F32["layered"])
        else:
            stats = compare(ref, bits, iters, post, llr.dtype, where)
        _log(f"[gpu]   {stats}, mean passes {iters.mean():.2f}")


@pytest.mark.parametrize("layered", [False, True])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("name", NAMES)
def test_minsum(L, handles, name, dtype, layered):
    code, llr = workload(name, dtype)
    sched = "layered" if layered else "flooding"
    if dtype == "f64":
        T, es = 20, True
    else:
        T, es = (1 if layered else 4), False
    _log(f"[gpu] min-sum {name} {dtype} {sched} T={T}")
    bits, iters, post = gpu_plain(L, handles(name), llr, T, es, layered=layered, rule="minsum", scale=0.75)
    ref = oracle.decode(code, llr, T, es, nthreads=8, schedule=sched, rule="minsum", ms_scale=0.75)
    if dtype == "f64":
        assert np.array_equal(iters, ref["iters"]) and np.array_equal(bits, ref["bits"])
        assert np.array_equal(post, ref["posterior"]), "FP64 min-sum posteriors differ from the oracle"
    else:
        _log(f"[gpu]   {compare(ref, bits, iters, post, llr.dtype, f'min-sum {name} {sched}')}")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("name", NAMES)
def test_batch(L, handles, name, dtype):
    """One ldpc_decode_batch call holding a flooding, a layered and a min-sum
    job of this code (fused kernel where the code fits it, else the plain
    route): each equals ldpc_decode of the same job bit for bit, and the
    flooding job matches the oracle."""
    import torch
    code, llr = workload(name, dtype)
    h = handles(name)
    x = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    specs = [dict(layered=False, rule="spa"), dict(layered=True, rule="spa"),
             dict(layered=False, rule="minsum", ms_scale=0.75)]
    jobs = [L.Job(h, x, 20, early_stop=True, **s) for s in specs]
    _log(f"[gpu] batch {name} {dtype} fused={name in FUSED_FITS}")
    L.decode_batch(jobs)
    torch.cuda.synchronize()
    for s, j in zip(specs, jobs):
        want = gpu_plain(L, h, llr, 20, True, layered=s["layered"], rule=s["rule"], scale=s.get("ms_scale", 1.0))
        got = _np(j.bits, j.iters, j.posterior)
        for a, b, what in zip(got, want, ("bits", "iters", "posterior")):
            assert np.array_equal(a, b), f"batch {name} {dtype} {s}: {what} differ from the plain path"
    ref = oracle.decode(code, llr, 20, True, nthreads=8)
    got = _np(jobs[0].bits, jobs[0].iters, jobs[0].posterior)
    if dtype == "f32":
        stats = compare_horizon(ref, *got, llr.dtype, f"batch {name}", code, 20, HORIZON_F32["flooding"])
    else:
        stats = compare(ref, *got, llr.dtype, f"batch {name}")
    _log(f"[gpu]   {stats}")


@pytest.mark.parametrize("layered", [False, True])
def test_qc1944_fp64(L, layered):
    """FP64 sum-product on the headline code (rows of degree 13..21, FP64
    bucket 32): plain path and fused kernel, against the oracle."""
    import torch
    b = configs.qc1944(2.0, frames=FRAMES)
    llr = b.llr.astype(np.float64)
    h = L.Code.from_workload(b.code)
    sched = "layered" if layered else "flooding"
    _log(f"[gpu] qc1944 FP64 {sched}")
    got = gpu_plain(L, h, llr, 10, False, layered=layered)
    ref = oracle.decode(b.code, llr, 10, False, nthreads=8, schedule=sched)
    _log(f"[gpu]   {compare(ref, *got, np.float64, f'qc1944 FP64 {sched}')}")
    job = L.Job(h, torch.from_numpy(llr).cuda(), 10, early_stop=False, layered=layered)
    L.decode_batch([job])
    torch.cuda.synchronize()
    for a, c in zip(_np(job.bits, job.iters, job.posterior), got):
        assert np.array_equal(a, c), "fused FP64 differs from the plain path"
