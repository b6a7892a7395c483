"""Two frames per workgroup in the fused kernel (ldpc_batch_set_frames_per_group)
and the autotuner that chooses it.

Bars: with two frames per workgroup every job's outputs equal those with one
frame per workgroup bit for bit (the same arithmetic on each frame, in its
own LDS region): QC and CSR codes, odd frame counts (a last pair of one
frame), early stop with the two frames of a pair stopping at different
iterations, and batches mixing eligible jobs with layered and min-sum jobs
(which keep one frame per workgroup).  The one-frame path is held to the
oracle by the batch and degree tests.  The autotuner records a choice whose
outputs match every other candidate's; its table survives a save and load.
"""
import sys

import numpy as np
import pytest

from degree_cases import workload
from workloads import channel, configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_06545_amd as lib
    yield lib
    lib.ldpc_batch_set_frames_per_group(1)


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(L, specs, fpw):
    """specs: (handle, llr ndarray, T, early_stop, layered, rule) -> outputs per job."""
    import torch
    assert L.ldpc_batch_set_frames_per_group(fpw) == L.LDPC_OK
    jobs = [L.Job(h, torch.from_numpy(np.ascontiguousarray(x)).cuda(), T, early_stop=es, layered=lay, rule=rule,
                  ms_scale=0.75 if rule == "minsum" else 1.0) for h, x, T, es, lay, rule in specs]
    L.decode_batch(jobs)
    torch.cuda.synchronize()
    L.ldpc_batch_set_frames_per_group(1)
    return [(j.bits.cpu().numpy(), j.iters.cpu().numpy(), j.posterior.cpu().numpy()) for j in jobs]


def _same(L, specs, where):
    a = _run(L, specs, 1)
    b = _run(L, specs, 2)
    for k, (x, y) in enumerate(zip(a, b)):
        for u, v, what in zip(x, y, ("bits", "iters", "posterior")):
            assert np.array_equal(u, v), f"{where}: job {k} {what} differ with two frames per workgroup"
    _log(f"[gpu] {where}: {len(specs)} jobs bit-identical with 1 and 2 frames per workgroup")
    return a


@pytest.mark.parametrize("frames", [1, 3, 64, 127, 300])
def test_pairs_qc1944_fixed_iterations(L, frames):
    b = configs.qc1944(1.5, frames=frames)
    h = L.Code.from_workload(b.code)
    _same(L, [(h, b.llr, 10, False, False, "spa")], f"qc1944 x{frames}")


def test_pairs_early_stop_frames_part(L):
    """4 dB inputs converge at different iterations: the frames of many pairs
    stop apart, and each keeps its own posteriors and count."""
    b = configs.qc1944(2.0, frames=257)
    llr = channel.bpsk_awgn_llr(b.codewords, 3.0, 0.5, 951, dtype=np.float32)
    h = L.Code.from_workload(b.code)
    out = _same(L, [(h, llr, 20, True, False, "spa")], "qc1944 3 dB early stop x257")
    it = out[0][1]
    pairs = it[: 256].reshape(-1, 2)
    assert (pairs[:, 0] != pairs[:, 1]).sum() > 20, "frames of a pair should stop apart"
    assert it.min() < 20


def test_pairs_mix_and_other_modes(L):
    mix = configs.qc_mix(total=2000)
    hs = [L.Code.from_workload(m.code) for m in mix]
    specs = [(hs[i], mix[i].llr, 10, True, False, "spa") for i in range(12)]
    specs += [(hs[3], mix[3].llr, 10, True, True, "spa"), (hs[5], mix[5].llr, 10, True, False, "minsum")]
    _same(L, specs, "qc_mix 12 codes + layered + min-sum jobs")


@pytest.mark.parametrize("name", ["csr_d25_32", "qc_d32", "spc30"])
def test_pairs_degree_cases(L, name):
    code, llr = workload(name, "f32")
    h = L.Code.from_workload(code)
    _same(L, [(h, llr, 20, True, False, "spa"), (h, llr[:77], 10, False, False, "spa")], f"{name}")


def test_pairs_gallager_fp32(L):
    g = configs.gallager504(frames=301)
    h = L.Code.from_workload(g.code)
    _same(L, [(h, g.llr.astype(np.float32), 20, True, False, "spa")], "gallager504 FP32 x301")


def test_autotune_chooses_and_persists(L, tmp_path):
    import torch
    mix = configs.qc_mix(total=1200)[:4]
    hs = [L.Code.from_workload(m.code) for m in mix]
    jobs = [L.Job(h, torch.from_numpy(m.llr).cuda(), 10, early_stop=True) for h, m in zip(hs, mix)]
    cj = [j.c_struct() for j in jobs]
    L.ldpc_tuning_clear()
    try:
        threads, ms = L.autotune_batch(jobs)
        cfg = L.ldpc_batch_launch_config(cj, torch.float32)
        per_job = L.ldpc_batch_job_threads(cj, torch.float32)
        _log(f"[gpu] autotune: {cfg}, per code {per_job}, {ms:.3f} ms")
        assert cfg["tuned"] and cfg["threads"] == threads == per_job[0] and cfg["frames_per_group"] in (1, 2)
        path = tmp_path / "tune.txt"
        assert L.ldpc_tuning_save(str(path)) == L.LDPC_OK
        lines = path.read_text().splitlines()
        assert all(len(line.split()) == 5 for line in lines)
        fpw_fields = [int(line.split()[3]) for line in lines]
        assert fpw_fields.count(0) == 4 and len(fpw_fields) == 5  # one line per code, one for the batch
        L.ldpc_tuning_clear()
        assert not L.ldpc_batch_launch_config(cj, torch.float32)["tuned"]
        assert L.ldpc_batch_job_threads(cj, torch.float32) == [512] * 4
        st, n = L.ldpc_tuning_load(str(path))
        assert st == L.LDPC_OK and n == len(lines)
        assert L.ldpc_batch_launch_config(cj, torch.float32) == cfg
        assert L.ldpc_batch_job_threads(cj, torch.float32) == per_job
        # a later decode of the same shape uses the choice and gives the same outputs
        ref = [(j.bits.clone(), j.iters.clone()) for j in jobs]
        L.decode_batch(jobs)
        torch.cuda.synchronize()
        for (b0, i0), j in zip(ref, jobs):
            assert torch.equal(b0, j.bits) and torch.equal(i0, j.iters)
    finally:
        L.ldpc_tuning_clear()
