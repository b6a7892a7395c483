"""GPU tests of the serving loop (continuous batching).

Each request's result must equal the same frames decoded alone with
ldpc_decode, bit for bit, whatever it was batched with; admission must respect
the memory arena; queued requests can be cancelled; bad requests are refused
before anything is queued.
"""
import sys
import time

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


@pytest.fixture(scope="module")
def pool():
    return configs.ServePool(per_code=128)


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _requests(pool, count, seed, max_frames=64):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        cid = int(rng.integers(12))
        fr = int(rng.integers(1, max_frames + 1))
        req = configs.ServeRequest(0.0, cid, fr, float(rng.uniform(1.0, 3.0)))
        llr, cw = pool.request_llr(i + 1000 * seed, req)
        n = pool.codes[cid].n
        out.append({"code": cid, "frames": fr, "llr": np.ascontiguousarray(llr),
                    "bits": np.full((fr, n), 9, np.uint8), "iters": np.full(fr, -9, np.int32),
                    "post": np.zeros((fr, n), np.float32)})
    return out


def _submit_all(L, srv, reqs, T=10, flags=1):
    tickets = []
    for r in reqs:
        st, t = L.ldpc_server_submit(srv, r["code"], r["frames"], T, flags, r["llr"], r["bits"], r["iters"], r["post"])
        assert st == 0, st
        tickets.append(t)
    return tickets


def test_server_isolation_and_oracle(L, pool):
    import torch
    handles = [L.Code.from_workload(c) for c in pool.codes]
    srv = L.ldpc_server_create(handles, 64 << 20, max_inflight=3, max_group_frames=512)
    try:
        reqs = _requests(pool, 120, seed=1)
        _log(f"[gpu] serve: {len(reqs)} requests, {sum(r['frames'] for r in reqs)} frames")
        tickets = _submit_all(L, srv, reqs)
        for t in tickets:
            assert L.ldpc_server_wait(srv, t, 60000.0) == 0
        stats = L.ldpc_server_stats_get(srv)
        _log(f"[gpu] serve stats: {stats}")
        assert stats["completed"] == len(reqs) and stats["failed"] == 0
        assert stats["launches"] >= 2
        # the slowest request's stages add up to its latency, and none is negative
        parts = [stats["worst_" + k + "_ms"] for k in ("queue", "stage", "device", "copyout")]
        assert min(parts) >= 0.0 and stats["max_step_ms"] > 0.0
        assert abs(sum(parts) + stats["worst_submit_ms"] - stats["max_ms"]) < 1e-3
    finally:
        L.ldpc_server_destroy(srv)
    for k, r in enumerate(reqs):
        bits, iters, post = L.decode(handles[r["code"]], torch.from_numpy(r["llr"]).cuda(), 10, early_stop=True)
        torch.cuda.synchronize()
        assert np.array_equal(r["bits"], bits.cpu().numpy()), f"request {k} bits differ from alone"
        assert np.array_equal(r["iters"], iters.cpu().numpy()), f"request {k} iters differ from alone"
        assert np.array_equal(r["post"], post.cpu().numpy()), f"request {k} posterior differs from alone"
        if k % 15 == 0:
            ref = oracle.decode(pool.codes[r["code"]], r["llr"], 10, True)
            compare(ref, r["bits"], r["iters"], r["post"], np.float32, f"serve request {k}")


def test_server_memory_admission(L, pool):
    """An arena that holds one 64-frame request at a time still completes
    everything, one group at a time, in submission order."""
    handles = [L.Code.from_workload(c) for c in pool.codes]
    one = 64 * max(c.n for c in pool.codes) * 10 + 4096
    srv = L.ldpc_server_create(handles, one, max_inflight=3, max_group_frames=64)
    try:
        reqs = _requests(pool, 12, seed=2)
        tickets = _submit_all(L, srv, reqs)
        for t in tickets:
            assert L.ldpc_server_wait(srv, t, 60000.0) == 0
        stats = L.ldpc_server_stats_get(srv)
        _log(f"[gpu] small arena stats: {stats}")
        assert stats["completed"] == 12
        assert stats["mean_group_frames"] <= 64
    finally:
        L.ldpc_server_destroy(srv)
    assert all((r["iters"] >= 0).all() for r in reqs)


def test_server_cancel_and_errors(L, pool):
    handles = [L.Code.from_workload(c) for c in pool.codes]
    one = 64 * max(c.n for c in pool.codes) * 10 + 4096
    srv = L.ldpc_server_create(handles, one, max_inflight=1, max_group_frames=64, max_queue=40)
    try:
        reqs = _requests(pool, 30, seed=3)
        tickets = _submit_all(L, srv, reqs)
        cancelled = 0
        for t in tickets[::-1][:10]:
            if L.ldpc_server_cancel(srv, t) == 0:
                cancelled += 1
        assert cancelled >= 1
        for t in tickets:
            assert L.ldpc_server_wait(srv, t, 60000.0) == 0
        st = L.ldpc_server_stats_get(srv)
        assert st["completed"] + st["cancelled"] == 30
        r = reqs[0]
        bad = [(12, 1), (-1, 1), (0, 0), (0, 65), (0, 100000)]
        for cid, fr in bad:
            s, _ = L.ldpc_server_submit(srv, cid, fr, 10, 1, r["llr"], r["bits"], r["iters"])
            assert s == L.LDPC_EINVAL, (cid, fr, s)
        s, _ = L.ldpc_server_submit(srv, 0, 1, 10, 8, r["llr"], r["bits"], r["iters"])
        assert s == L.LDPC_EINVAL
        assert L.ldpc_server_wait(srv, 10 ** 9, 1.0) == L.LDPC_EINVAL
    finally:
        L.ldpc_server_destroy(srv)


def test_server_queue_limit(L, pool):
    handles = [L.Code.from_workload(c) for c in pool.codes[:1]]
    srv = L.ldpc_server_create(handles, 1 << 20, max_inflight=1, max_group_frames=8, max_queue=4)
    try:
        reqs = _requests(pool, 1, seed=4, max_frames=1)
        r = reqs[0]
        r["code"] = 0
        llr = np.ascontiguousarray(pool.request_llr(5, configs.ServeRequest(0, 0, 1, 2.0))[0])
        busy = 0
        tickets = []
        outs = [(np.zeros((1, pool.codes[0].n), np.uint8), np.zeros(1, np.int32)) for _ in range(64)]
        for k in range(64):
            s, t = L.ldpc_server_submit(srv, 0, 1, 10, 1, llr, outs[k][0], outs[k][1])
            if s == L.LDPC_EBUSY:
                busy += 1
            else:
                assert s == 0
                tickets.append(t)
        assert busy >= 1
        for t in tickets:
            assert L.ldpc_server_wait(srv, t, 60000.0) == 0
    finally:
        L.ldpc_server_destroy(srv)


def test_server_merges_alike_requests(L, pool):
    """Many small requests of a few codes with mixed iteration limits, flags
    and posterior wishes: the scheduler lays each group out by code and
    merges neighbours decoded alike into one job, so every group (at most
    3 codes x 2 limits x 2 flag sets x 2 posterior wishes = 24 distinct jobs)
    is one fused launch, and every request's result still equals decoding it
    alone with its own settings."""
    import torch
    handles = [L.Code.from_workload(c) for c in pool.codes]
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(160):
        cid = int(rng.choice([0, 5, 11]))
        fr = int(rng.integers(1, 9))
        req = configs.ServeRequest(0.0, cid, fr, float(rng.uniform(1.0, 3.0)))
        llr, _ = pool.request_llr(7000 + i, req)
        n = pool.codes[cid].n
        reqs.append({"code": cid, "frames": fr, "llr": np.ascontiguousarray(llr), "T": int(rng.choice([5, 10])),
                     "flags": int(rng.integers(2)), "bits": np.full((fr, n), 9, np.uint8),
                     "iters": np.full(fr, -9, np.int32),
                     "post": np.zeros((fr, n), np.float32) if rng.integers(2) else None})
    srv = L.ldpc_server_create(handles, 64 << 20, max_inflight=2, max_group_frames=1024)
    try:
        L.ldpc_profile_collect()  # drop the creation warm-up's records
        assert L.ldpc_profile_enable(True) == 0
        L.ldpc_server_stats_get(srv, reset=True)
        tickets = []
        for r in reqs:
            st, t = L.ldpc_server_submit(srv, r["code"], r["frames"], r["T"], r["flags"], r["llr"], r["bits"],
                                         r["iters"], r["post"])
            assert st == 0, st
            tickets.append(t)
        for t in tickets:
            assert L.ldpc_server_wait(srv, t, 60000.0) == 0
        stats = L.ldpc_server_stats_get(srv)
        prof = L.ldpc_profile_collect()
    finally:
        L.ldpc_profile_enable(False)
        L.ldpc_server_destroy(srv)
    _log(f"[gpu] merge: {stats['launches']} groups, mean {stats['mean_group_frames']:.1f} frames, "
         f"fused launches {prof['fused'][1]}")
    assert stats["completed"] == len(reqs) and stats["failed"] == 0
    assert stats["mean_group_frames"] > 16  # groups of several requests were formed
    assert prof["fused"][1] == stats["launches"], "a group took more than one fused launch"
    for k, r in enumerate(reqs):
        bits, iters, post = L.decode(handles[r["code"]], torch.from_numpy(r["llr"]).cuda(), r["T"],
                                     early_stop=bool(r["flags"]))
        torch.cuda.synchronize()
        assert np.array_equal(r["bits"], bits.cpu().numpy()), f"request {k} bits differ from alone"
        assert np.array_equal(r["iters"], iters.cpu().numpy()), f"request {k} iters differ from alone"
        if r["post"] is not None:
            assert np.array_equal(r["post"], post.cpu().numpy()), f"request {k} posterior differs from alone"


def test_server_with_tuned_workgroup_sizes(L, pool):
    """After the autotuner has given the codes different workgroup sizes, a
    server group of mixed codes runs as one fused launch per size; every
    request still equals decoding it alone, bit for bit."""
    import torch
    handles = [L.Code.from_workload(c) for c in pool.codes]
    L.ldpc_tuning_clear()
    try:
        tune = [L.Job(h, torch.from_numpy(np.ascontiguousarray(pool.llr_pool(i)[:64])).cuda(), 10, early_stop=True)
                for i, h in enumerate(handles)]
        L.autotune_batch(tune)
        sizes = L.ldpc_batch_job_threads([j.c_struct() for j in tune], torch.float32)
        _log(f"[gpu] serve after tuning: per-code workgroup sizes {sizes}")
        srv = L.ldpc_server_create(handles, 64 << 20, max_inflight=3, max_group_frames=512)
        try:
            reqs = _requests(pool, 60, seed=7)
            for t in _submit_all(L, srv, reqs):
                assert L.ldpc_server_wait(srv, t, 60000.0) == 0
            stats = L.ldpc_server_stats_get(srv)
            assert stats["completed"] == len(reqs) and stats["failed"] == 0
        finally:
            L.ldpc_server_destroy(srv)
        for k, r in enumerate(reqs):
            bits, iters, post = L.decode(handles[r["code"]], torch.from_numpy(r["llr"]).cuda(), 10, early_stop=True)
            torch.cuda.synchronize()
            assert np.array_equal(r["bits"], bits.cpu().numpy()), f"request {k} bits differ from alone"
            assert np.array_equal(r["iters"], iters.cpu().numpy()), f"request {k} iters differ from alone"
            assert np.array_equal(r["post"], post.cpu().numpy()), f"request {k} posterior differs from alone"
    finally:
        L.ldpc_tuning_clear()
