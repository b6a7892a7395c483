"""GPU tests of ldpc_decode_batch: the fused frame-resident persistent kernel
(and the plain-path route for codes that do not fit it).

Bars: every job's outputs equal the oracle's within the parity rule, and
equal the plain per-iteration path bit for bit (both paths evaluate each
message with the same operations in the same order); a job decoded inside a
mixed batch equals the same job decoded alone, bit for bit.
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


def _batch(L, items, es=True, T=10):
    """items: list of (code handle, llr ndarray) -> list of Job (decoded)."""
    import torch
    jobs = [L.Job(h, torch.from_numpy(np.ascontiguousarray(llr)).cuda(), T, early_stop=es) for h, llr in items]
    L.decode_batch(jobs)
    torch.cuda.synchronize()
    return jobs


def _plain(L, h, llr, T, es):
    import torch
    b, i, p = L.decode(h, torch.from_numpy(np.ascontiguousarray(llr)).cuda(), T, early_stop=es)
    torch.cuda.synchronize()
    return b.cpu().numpy(), i.cpu().numpy(), p.cpu().numpy()


def _np(job):
    return job.bits.cpu().numpy(), job.iters.cpu().numpy(), job.posterior.cpu().numpy()


def test_fused_fit_reporting(L):
    import torch
    qc = L.Code.from_workload(configs.qc1944(2.0, frames=1).code)
    ok, lds = L.ldpc_batch_fits_fused(qc, torch.float32)
    _log(f"[gpu] qc1944 fused fit={ok} lds={lds}")
    assert ok and 60000 < lds < 100000
    props = torch.cuda.get_device_properties(0)
    _log(f"[gpu] device {props.name} CUs={props.multi_processor_count}")
    stair = L.Code.from_workload(configs.stair64800(frames=1).code)
    assert L.ldpc_batch_fits_fused(stair, torch.float32)[0] is False


@pytest.mark.parametrize("snr", [1.0, 2.5])
def test_fused_qc1944_vs_oracle_and_plain(L, snr):
    b = configs.qc1944(snr, frames=130)
    h = L.Code.from_workload(b.code)
    _log(f"[gpu] fused qc1944 {snr} dB x130")
    job = _batch(L, [(h, b.llr)], es=False)[0]
    bits, iters, post = _np(job)
    ref = oracle.decode(b.code, b.llr, 10, False, nthreads=8)
    _log(f"[gpu]   {compare(ref, bits, iters, post, np.float32, 'fused qc1944')}")
    pb, pi, pp = _plain(L, h, b.llr, 10, False)
    assert np.array_equal(bits, pb) and np.array_equal(iters, pi) and np.array_equal(post, pp)


def test_fused_early_stop_high_snr(L):
    b = configs.qc1944(2.0, frames=100)
    llr = channel.bpsk_awgn_llr(b.codewords, 4.0, 0.5, 905, dtype=np.float32)
    h = L.Code.from_workload(b.code)
    _log("[gpu] fused qc1944 4 dB early stop")
    job = _batch(L, [(h, llr)], es=True)[0]
    bits, iters, post = _np(job)
    ref = oracle.decode(b.code, llr, 10, True, nthreads=8)
    compare(ref, bits, iters, post, np.float32, "fused es")
    assert iters.min() < 10
    pb, pi, pp = _plain(L, h, llr, 10, True)
    assert np.array_equal(bits, pb) and np.array_equal(iters, pi) and np.array_equal(post, pp)


def test_fused_mix_isolation_and_oracle(L):
    """The 12-code QC mix in one batch: each job equals the oracle (sampled
    frames), the plain path and the same job decoded alone, bit for bit."""
    mix = configs.qc_mix(total=1200)
    handles = [L.Code.from_workload(m.code) for m in mix]
    _log(f"[gpu] fused mix: {[m.llr.shape[0] for m in mix]}")
    jobs = _batch(L, list(zip(handles, [m.llr for m in mix])), es=True)
    for k, (m, h, j) in enumerate(zip(mix, handles, jobs)):
        bits, iters, post = _np(j)
        alone = _np(_batch(L, [(h, m.llr)], es=True)[0])
        for x, y in zip((bits, iters, post), alone):
            assert np.array_equal(x, y), f"job {k} differs alone vs in the mix"
        pb, pi, pp = _plain(L, h, m.llr, 10, True)
        assert np.array_equal(bits, pb) and np.array_equal(iters, pi) and np.array_equal(post, pp)
        idx = np.unique(np.r_[0, m.llr.shape[0] - 1, np.arange(0, m.llr.shape[0], 17)])
        ref = oracle.decode(m.code, m.llr[idx], 10, True, nthreads=8)
        compare(ref, bits[idx], iters[idx], post[idx], np.float32, f"mix job {k}")


@pytest.mark.parametrize("mode", ["flooding", "layered", "min-sum"])
def test_schedule_instance_matches_general_instance(L, mode):
    """A batch whose jobs are all FP32 on codes with a circulant view and all
    take one of sum-product flooding, sum-product layered or min-sum flooding
    runs a kernel instance compiled with those rows alone (no other rule or
    schedule, no CSR rows).  Adding a job of another kind, or a job on a code
    without a circulant view, makes the same jobs run the general instance:
    their outputs stay the same, bit for bit."""
    import torch
    kinds = {"flooding": {}, "layered": {"layered": True}, "min-sum": {"rule": "minsum", "ms_scale": 0.75}}
    kw = kinds[mode]
    mix = configs.qc_mix(total=720)[::3]
    hs = [L.Code.from_workload(m.code) for m in mix]
    g = configs.gallager504(frames=64)
    hg = L.Code.from_workload(g.code)
    for es in (True, False):
        def jobs_of():
            return [L.Job(h, torch.from_numpy(np.ascontiguousarray(m.llr)).cuda(), 10, early_stop=es, **kw)
                    for h, m in zip(hs, mix)]
        first = jobs_of()
        L.decode_batch(first)
        torch.cuda.synchronize()
        base = [_np(j) for j in first]
        x0 = torch.from_numpy(np.ascontiguousarray(mix[0].llr)).cuda()
        extras = {other: L.Job(hs[0], x0, 10, early_stop=es, **kinds[other]) for other in kinds if other != mode}
        extras["csr code"] = L.Job(hg, torch.from_numpy(g.llr.astype(np.float32)).cuda(), 10, early_stop=es, **kw)
        for name, extra in extras.items():
            _log(f"[gpu] {mode} instance vs general (+{name}, early stop {es})")
            jobs = jobs_of()
            L.decode_batch(jobs + [extra])
            torch.cuda.synchronize()
            for k, (j, ref) in enumerate(zip(jobs, base)):
                for x, y in zip(_np(j), ref):
                    assert np.array_equal(x, y), f"job {k} differs with a {name} job in the batch"


def test_fused_f64_gallager(L):
    b = configs.gallager504(frames=300)
    h = L.Code.from_workload(b.code)
    _log("[gpu] fused gallager504 f64")
    job = _batch(L, [(h, b.llr)], es=True, T=20)[0]
    bits, iters, post = _np(job)
    ref = oracle.decode(b.code, b.llr, 20, True, nthreads=8)
    compare(ref, bits, iters, post, np.float64, "fused f64")
    pb, pi, pp = _plain(L, h, b.llr, 20, True)
    assert np.array_equal(bits, pb) and np.array_equal(iters, pi) and np.array_equal(post, pp)


def test_batch_routes_large_code_through_plain(L):
    """A batch holding a code too large for LDS next to fused jobs."""
    stair = configs.stair64800(frames=8)
    qc = configs.qc1944(1.5, frames=70)
    hs, hq = L.Code.from_workload(stair.code), L.Code.from_workload(qc.code)
    _log("[gpu] batch with stair64800 + qc1944")
    jobs = _batch(L, [(hq, qc.llr), (hs, stair.llr)], es=True, T=50)
    for (bt, h), j in zip(((qc, hq), (stair, hs)), jobs):
        bits, iters, post = _np(j)
        pb, pi, pp = _plain(L, h, bt.llr, 50, True)
        assert np.array_equal(bits, pb) and np.array_equal(iters, pi) and np.array_equal(post, pp)
    ref = oracle.decode(stair.code, stair.llr[:2], 50, True)
    bits, iters, post = _np(jobs[1])
    compare(ref, bits[:2], iters[:2], post[:2], np.float32, "stair in batch")


def test_fused_small_and_degenerate_codes(L):
    rng = np.random.default_rng(3)
    rows = [[], [0], [1, 2, 3], list(range(4, 28)), [2, 5, 9]]
    degenerate = codes.Code.from_row_lists(len(rows), 30, rows, "degenerate")
    cases = [codes.single_parity_check(5), codes.hamming74(), codes.random_tree_code(12, 3), degenerate]
    for code in cases:
        h = L.Code.from_csr(code.m, code.n, code.row_ptr, code.col_idx)
        llr = rng.normal(0.5, 2.0, size=(67, code.n)).astype(np.float32)
        for es in (False, True):
            for T in (0, 1, 7):
                _log(f"[gpu] fused {code.name} T={T} es={es}")
                bits, iters, post = _np(_batch(L, [(h, llr)], es=es, T=T)[0])
                ref = oracle.decode(code, llr, T, es)
                compare(ref, bits, iters, post, np.float32, f"fused {code.name}")
                pb, pi, pp = _plain(L, h, llr, T, es)
                assert np.array_equal(bits, pb) and np.array_equal(iters, pi) and np.array_equal(post, pp)


def test_fused_qc_with_empty_base_rows_and_columns(L):
    """Circulant codes whose base matrix has empty block-columns (first,
    middle, last) and an empty block-row: the fused kernel's column phase
    reads a spare table word for empty columns and its row phase skips empty
    rows; results equal the oracle and the plain path bit for bit."""
    rng = np.random.default_rng(17)
    Z = 27
    shifts = rng.integers(0, Z, size=(4, 10)).astype(np.int32)
    shifts[:, [0, 4, 9]] = -1          # empty block-columns, the last one included
    shifts[2, :] = -1                  # an empty block-row
    shifts[0, 1] = shifts[1, 3] = -1   # some ordinary holes
    code = codes.qc_expand(shifts, Z, "qc with empty base rows and columns")
    h = L.Code.from_workload(code)
    fits, _ = L.ldpc_batch_fits_fused(h, L.LDPC_F32)
    assert fits
    llr = rng.normal(0.8, 2.0, size=(131, code.n)).astype(np.float32)
    for es in (False, True):
        for T in (1, 6):
            _log(f"[gpu] fused {code.name} T={T} es={es}")
            bits, iters, post = _np(_batch(L, [(h, llr)], es=es, T=T)[0])
            ref = oracle.decode(code, llr, T, es)
            compare(ref, bits, iters, post, np.float32, f"fused {code.name}")
            pb, pi, pp = _plain(L, h, llr, T, es)
            assert np.array_equal(bits, pb) and np.array_equal(iters, pi) and np.array_equal(post, pp)


def test_fused_noiseless_zero_iterations(L):
    b = configs.qc1944(2.0, frames=40)
    h = L.Code.from_workload(b.code)
    llr = channel.noiseless_llr(b.codewords, 3.0, np.float32)
    bits, iters, post = _np(_batch(L, [(h, llr)], es=True, T=10)[0])
    assert (iters == 0).all() and (bits == b.codewords).all() and np.array_equal(post, llr)
    bits, iters, post = _np(_batch(L, [(h, b.llr)], es=False, T=0)[0])
    assert (iters == 0).all() and (bits == (b.llr < 0)).all() and np.array_equal(post, b.llr)


@pytest.mark.parametrize("threads", [64, 192, 256, 512])
def test_fused_threads_do_not_change_results(L, threads):
    b = configs.qc_mix(total=200)
    items = [(L.Code.from_workload(m.code), m.llr) for m in b[:4]]
    L.ldpc_tuning_clear()  # no tuned per-code size may override the one set here
    assert L.ldpc_batch_set_threads(threads) == 0
    try:
        got = [_np(j) for j in _batch(L, items)]
    finally:
        L.ldpc_batch_set_threads(512)
    want = [_np(j) for j in _batch(L, items)]
    for g, w in zip(got, want):
        for x, y in zip(g, w):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("threads", [64, 512])
def test_fused_early_stop_many_rows_per_lane(L, threads):
    """Regression: with fewer lanes than rows a lane checks several rows, and
    the frame's stop test must see any unsatisfied one (rows' parities are
    ORed, not XORed: two unsatisfied rows on one lane once cancelled and
    stopped a frame early).  All 12 codes, early stop, against the plain path
    (one row per wavefront) bit for bit, and every stopped frame's bits must
    satisfy H by an independent dense product."""
    from mapref import dense_syndrome
    mix = configs.qc_mix(total=2000)
    items = [(L.Code.from_workload(m.code), m.llr) for m in mix]
    L.ldpc_tuning_clear()
    assert L.ldpc_batch_set_threads(threads) == 0
    try:
        jobs = _batch(L, items)
    finally:
        L.ldpc_batch_set_threads(512)
    for (h, llr), m, j in zip(items, mix, jobs):
        bits, iters, post = _np(j)
        pb, pi, pp = _plain(L, h, llr, 10, True)
        assert np.array_equal(iters, pi) and np.array_equal(bits, pb) and np.array_equal(post, pp), m.code.name
        stopped = iters < 10
        assert (dense_syndrome(m.code, bits[stopped]) == 0).all(), m.code.name


def test_plan_replays_match_eager(L):
    """A captured plan replayed several times, with eager work and
    synchronisations between replays and new LLRs in place, matches the eager
    ldpc_decode_batch on the same inputs every time."""
    import torch
    mix = configs.qc_mix(total=600)
    stair = configs.stair64800(frames=4)
    items = [(L.Code.from_workload(m.code), m.llr) for m in mix[:5]] + [(L.Code.from_workload(stair.code), stair.llr)]
    jobs = [L.Job(h, torch.from_numpy(np.ascontiguousarray(llr)).cuda(), 12, early_stop=True) for h, llr in items]
    plan = L.Plan(jobs)
    rng = np.random.default_rng(9)
    try:
        for rep in range(4):
            if rep:
                for j in jobs:  # new inputs in the same buffers
                    j.llr.copy_(torch.from_numpy((rng.normal(1.5, 2.0, size=tuple(j.llr.shape))).astype(np.float32)))
            _log(f"[gpu] plan replay {rep}")
            plan.launch()
            torch.cuda.synchronize()
            got = [_np(j) for j in jobs]
            _ = torch.ones(1024, device="cuda").sum().item()  # eager work between replays
            eager = [L.Job(j.code, j.llr.clone(), 12, early_stop=True) for j in jobs]
            L.decode_batch(eager)
            torch.cuda.synchronize()
            for g, e in zip(got, eager):
                for x, y in zip(g, _np(e)):
                    assert np.array_equal(x, y), f"replay {rep} differs from eager"
    finally:
        plan.close()


def test_autotune_keeps_results(L):
    import torch
    mix = configs.qc_mix(total=2000)
    items = [(L.Code.from_workload(m.code), m.llr) for m in mix]
    before = [_np(j) for j in _batch(L, items)]
    jobs = [L.Job(h, torch.from_numpy(llr).cuda(), 10, early_stop=True) for h, llr in items]
    try:
        threads, ms = L.autotune_batch(jobs)
        per_job = L.ldpc_batch_job_threads([j.c_struct() for j in jobs], torch.float32)
        _log(f"[gpu] autotune: threads={threads} ms={ms:.3f} per code={per_job}")
        assert threads in (64, 128, 192, 256, 384, 512) and ms > 0
        assert all(t in (64, 128, 192, 256, 384, 512) for t in per_job) and threads == per_job[0]
        # a batch of these codes now runs as one launch per workgroup size, with the same results
        after = [_np(j) for j in _batch(L, items)]
        for b, a in zip(before, after):
            for x, y in zip(b, a):
                assert np.array_equal(x, y)
    finally:
        L.ldpc_tuning_clear()


def test_plan_under_tuned_sizes_matches_eager(L):
    """With per-code workgroup sizes tuned, a batch is several fused launches;
    a plan captured then replays them and matches the eager call bit for bit."""
    import torch
    mix = configs.qc_mix(total=1200)
    items = [(L.Code.from_workload(m.code), m.llr) for m in mix]
    jobs = [L.Job(h, torch.from_numpy(np.ascontiguousarray(llr)).cuda(), 10, early_stop=True) for h, llr in items]
    L.ldpc_tuning_clear()
    try:
        L.autotune_batch(jobs)
        sizes = L.ldpc_batch_job_threads([j.c_struct() for j in jobs], torch.float32)
        _log(f"[gpu] tuned sizes {sizes}")
        plan = L.Plan(jobs)
        try:
            for rep in range(3):
                plan.launch()
                torch.cuda.synchronize()
                got = [_np(j) for j in jobs]
                eager = [L.Job(j.code, j.llr.clone(), 10, early_stop=True) for j in jobs]
                L.decode_batch(eager)
                torch.cuda.synchronize()
                for g, e in zip(got, eager):
                    for x, y in zip(g, _np(e)):
                        assert np.array_equal(x, y), f"replay {rep} differs from eager"
        finally:
            plan.close()
    finally:
        L.ldpc_tuning_clear()
