#!/usr/bin/env python3
"""Decoded Mbit/s of flooding sum-product LDPC decoding on one MI355X.

Workload (one "step" = one batch through the whole decoder: ingest, 10
iterations of check-node / variable-node updates with hard decisions, output):
a seeded quasi-cyclic rate-1/2 code with a 12 x 24 base matrix and Z = 81
(n = 1944), 4096 random codewords per batch, BPSK over AWGN, FP32, exactly 10
iterations (early stop off).  Four batches at Eb/N0 = 1.0, 1.5, 2.0, 2.5 dB
are resident in HBM and the steps cycle through them.

Prints one JSON line: throughput (coded bits per second of device time), the
median and spread of single steps (event pairs around each step, timed
after the headline region), the dominant kernel's roofline position
measured with HIP events inside the timed region, and the CPU oracle timed
on the host on a bounded sample (all host threads, and one thread).
Beside the headline (skipped with --no-extra unless noted) it reports: the
same workload through the fused batch kernel; the other seeded workloads
(gallager504 FP64, the 12-code mix, stair64800); the layered schedule and
the min-sum rule on qc1944; the paper's multi-stream structure over host
buffers; the copy probe (--copy-probe-mb); an open-loop serving run
(--serve-seconds); the CPU oracle (--no-cpu-baseline skips it).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20, help="untimed steps first: the GPU clock ramps up over the first ~10 ms of load")
    ap.add_argument("--path", choices=("plain", "batch", "layered"), default="plain",
                    help="plain: per-iteration kernels (ldpc_decode); batch: ldpc_decode_batch; "
                         "layered: ldpc_decode with the layered schedule (10 passes instead of iterations)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target wall time of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the measured open-loop serving run (0 = skip)")
    ap.add_argument("--serve-warmup", type=float, default=1.0,
                    help="seconds of the same traffic before the measured run (statistics reset after it)")
    ap.add_argument("--serve-rate", type=float, default=20000.0, help="offered requests per second")
    ap.add_argument("--no-extra", action="store_true", help="skip the batch-path and other-workload timings")
    ap.add_argument("--only-workload", choices=("gallager504_f64", "qc_mix_16384", "stair64800"), default=None,
                    help="of the other workloads, time this one alone (for a profile of its kernels)")
    ap.add_argument("--profile-every", type=int, default=PROFILE_EVERY,
                    help="bracket the launches of every N-th timed step with HIP events (kernel durations)")
    ap.add_argument("--copy-probe-mb", type=int, default=512,
                    help="size of the streaming copy that measures achievable HBM bandwidth (0 = skip)")
    return ap.parse_args()


HBM_PEAK_GBS = 8000.0
PROFILE_EVERY = 10  # timed steps per step whose launches are bracketed by HIP events

# HBM bytes per check-kernel launch on this workload, from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE; reads scaled by 2.0 and writes by 1.0,
# the ratios of true bytes to counter readings for the library's copy
# kernel), averaged over one first-iteration and nine later launches.  Valid
# only for the kernel source they were taken on (hash below); otherwise null.
CHECK_TRAFFIC = {
    "bytes_per_launch": 543.1e6,
    "source_sha256": "a3106c90e407f8897c1385d47829ff15770e00aa0a419879e150a4f24eae300e",
    "profile": "profiles/hbm_traffic_check_qc1944.md",
}
CHECK_SOURCES = ("flood_kernels.h", "spa_math.h", "check_f32_d24.hip")

# The check kernel is co-limited by VALU issue.  Wavefront VALU instructions
# per launch on this workload, from the SQ_INSTS_VALU counter run (same
# source hash, same averaging over one first-iteration and nine later
# launches).  Issue peak: 1024 SIMDs x 2.4 GHz / 4 cycles per wave64
# instruction (4 of the instructions per edge and chunk are transcendentals,
# which hold their SIMD longer, so this fraction understates the issue load).
CHECK_VALU = {
    "insts_per_launch": 36.21e6,
    "source_sha256": CHECK_TRAFFIC["source_sha256"],
    "profile": "profiles/check_variable_qc1944_plain.md",
}
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4  # wavefront instructions per second


def check_source_hash():
    import hashlib
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1812_06545_amd", "csrc")
    lines = "".join(f"{hashlib.sha256(open(os.path.join(here, f), 'rb').read()).hexdigest()}  "
                    f"paper_1812_06545_amd/csrc/{f}\n" for f in CHECK_SOURCES)
    return hashlib.sha256(lines.encode()).hexdigest()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE={world}): "
              "frames are independent, so multi-GPU decoding is a frame split with no exchange and is not "
              "measured here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1812_06545_amd as L
    from workloads import configs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    T = 10
    batches = [configs.qc1944(snr) for snr in configs.QC1944_SNRS]
    code = batches[0].code
    F, n, E = batches[0].llr.shape[0], code.n, code.edges
    k_info = batches[0].k
    h = L.Code.from_workload(code)
    llrs = [torch.from_numpy(b.llr).to(dev) for b in batches]
    bits = torch.empty((F, n), dtype=torch.uint8, device=dev)
    iters = torch.empty(F, dtype=torch.int32, device=dev)
    post = torch.empty((F, n), dtype=torch.float32, device=dev)

    if args.path in ("plain", "layered"):
        ws_bytes = L.ldpc_workspace_bytes(h.handle, torch.float32, F, T)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        flags = L.LDPC_LAYERED if args.path == "layered" else 0

        def step(i):
            st = L.ldpc_decode(h.handle, torch.float32, F, T, flags, llrs[i % 4], bits, iters, post, ws, ws_bytes)
            if st != 0:
                raise L.LdpcError(st, "ldpc_decode")
    else:
        jobs = [[L.ldpc_job(h.handle, F, T, 0, llrs[i].data_ptr(), bits.data_ptr(), iters.data_ptr(),
                            post.data_ptr())] for i in range(4)]
        ws_bytes = L.ldpc_batch_workspace_bytes(jobs[0], torch.float32)
        ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=dev)

        def step(i):
            st = L.ldpc_decode_batch(jobs[i % 4], torch.float32, ws, ws_bytes)
            if st != 0:
                raise L.LdpcError(st, "ldpc_decode_batch")

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    L.ldpc_profile_collect()
    torch.cuda.synchronize()
    # Kernel durations come from HIP events the library records around every
    # launch of every PROFILE_EVERY-th step of the timed region; each event pair
    # adds a few microseconds of gap between dependent launches, so the other
    # steps run without them.
    t0 = time.perf_counter()
    for i in range(args.steps):
        # every profile_every-th step counted back from the last one (the
        # first step, which follows a host pause, only when it is the last)
        L.ldpc_profile_enable((args.steps - 1 - i) % args.profile_every == 0)
        step(i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    L.ldpc_profile_enable(False)
    prof = L.ldpc_profile_collect()

    ms_per_step = elapsed * 1e3 / args.steps
    coded_bits = F * n
    value = coded_bits * args.steps / elapsed / 1e6

    # Per-step device times (an event pair around each step), after the timed
    # region and apart from it: median and spread of the same step.
    step_ms = []
    for i in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        step(i)
        e1.record()
        step_ms.append((e0, e1))
    torch.cuda.synchronize()
    step_ms = sorted(a.elapsed_time(b) for a, b in step_ms)
    per_step = {"median_ms": step_ms[len(step_ms) // 2], "min_ms": step_ms[0], "max_ms": step_ms[-1],
                "steps": len(step_ms), "median_mbps": coded_bits / (step_ms[len(step_ms) // 2] * 1e-3) / 1e6}

    # Roofline of the dominant kernel.  Algorithmic bytes of one check-node
    # launch over F frames: read r (4E, not on the first iteration), write r
    # (4E), read the posterior once per variable (4n).
    if args.path == "plain":
        name, (kms, kcount) = "check", prof["check"]
        per_frame_first = 4 * E + 4 * n
        per_frame_later = 8 * E + 4 * n
        bytes_per_launch = F * (per_frame_first + (T - 1) * per_frame_later) / T
    elif args.path == "layered":
        # one launch per layer; per edge and frame a layer reads r and L and
        # writes both (16 bytes; 12 on the first pass, which reads no r);
        # averaged over the launches of one decode
        name, (kms, kcount) = "layer", prof["check"]
        layers = L.ldpc_code_layers(h)[0]
        bytes_per_launch = F * (12 * E + (T - 1) * 16 * E) / (T * layers)
    else:
        name, (kms, kcount) = "fused", prof["fused"]
        # frame-resident kernel: reads the channel LLRs and writes bits and the
        # posterior once per frame; messages live in LDS
        bytes_per_launch = F * (4 * n + n + 4 * n + 4)
    avg_ms = kms / max(kcount, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if kcount else None
    traffic = None
    if args.path == "plain" and check_source_hash() == CHECK_TRAFFIC["source_sha256"]:
        traffic = CHECK_TRAFFIC["bytes_per_launch"]
    roofline = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                "traffic_unit": "bytes per launch", "traffic_profile": CHECK_TRAFFIC["profile"] if traffic else None,
                "launch_ms": avg_ms, "launches": kcount, "bytes_per_launch": bytes_per_launch,
                "timed_launches": f"HIP events on every launch of every {args.profile_every}th timed step"}
    if args.path == "plain" and kcount and check_source_hash() == CHECK_VALU["source_sha256"]:
        insts = CHECK_VALU["insts_per_launch"]
        roofline["valu"] = {"achieved": insts / (avg_ms * 1e-3) / 1e9, "peak": VALU_ISSUE_PEAK / 1e9,
                            "unit": "G wavefront instructions/s", "frac": insts / (avg_ms * 1e-3) / VALU_ISSUE_PEAK,
                            "insts_per_launch": insts, "profile": CHECK_VALU["profile"]}
    # the whole step against its algorithmic floor (every frame runs T iterations)
    roofline["step_floor"] = floor_frac(E, n, 4, F * T, ms_per_step)
    kernels = {k: {"ms_total": v[0], "launches": v[1]} for k, v in prof.items() if v[1]}

    other_path = None
    rest = not args.no_extra and args.only_workload is None
    if args.path == "plain" and rest:
        other_path = batch_path_run(h, llrs, bits, iters, post, F, n, T, args.steps)
    extra = None if args.no_extra else extra_workloads(args.only_workload)
    layered = layered_workloads(args.steps) if rest else None
    minsum = minsum_workloads(args.steps) if rest else None
    mstream = mstream_run() if rest else None

    copy = copy_probe(args.copy_probe_mb) if args.copy_probe_mb > 0 else None
    if copy and achieved:
        roofline["frac_of_copy"] = achieved / copy["gbs"]

    serving = serve_run(args.serve_seconds, args.serve_rate, warmup_s=args.serve_warmup) \
        if args.serve_seconds > 0 else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(batches, T, args.cpu_seconds)

    out = {
        "metric": "decoded Mbit/s @10 iters n=1944 FP32",
        "value": value,
        "unit": "Mbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "qc1944: seeded QC code, 12x24 base, Z=81, n=1944, rate 1/2, 4096 frames/step, "
                               "10 iterations (no early stop), BPSK/AWGN at 1.0/1.5/2.0/2.5 dB"
                               + (" (layered schedule: 10 passes)" if args.path == "layered" else ""),
                   "path": args.path, "frames": F, "n": n, "edges": E, "iterations": T},
        "info_mbps": k_info * F * args.steps / elapsed / 1e6,
        "per_step": per_step,
        "roofline": roofline,
        "kernels": kernels,
        "batch_path": other_path,
        "other_workloads": extra,
        "layered": layered,
        "min_sum": minsum,
        "multi_stream_baseline": mstream,
        "copy_probe": copy,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def floor_frac(E, n, tsize, frame_iters, ms):
    """Fraction of HBM peak that the whole step's algorithmic floor traffic
    would need: per frame-iteration one stored message per edge read and
    written once (2 tsize E) and one posterior per variable (tsize n),
    summed over the iterations each frame actually ran, divided by the
    measured time."""
    floor_bytes = frame_iters * (2 * tsize * E + tsize * n)
    gbs = floor_bytes / (ms * 1e-3) / 1e9
    return {"floor_bytes": floor_bytes, "achieved_gbs": gbs, "frac": gbs / HBM_PEAK_GBS}


def _time_ms(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batch_path_run(h, llrs, bits, iters, post, F, n, T, steps):
    """The same workload through ldpc_decode_batch (the fused frame-resident
    persistent kernel), timed on its own after the headline region."""
    import torch

    import paper_1812_06545_amd as L
    jobs = [[L.ldpc_job(h.handle, F, T, 0, llrs[i].data_ptr(), bits.data_ptr(), iters.data_ptr(), post.data_ptr())]
            for i in range(4)]
    wsb = L.ldpc_batch_workspace_bytes(jobs[0], torch.float32)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device="cuda")
    k = [0]

    def step():
        if L.ldpc_decode_batch(jobs[k[0] % 4], torch.float32, ws, wsb) != 0:
            raise RuntimeError("ldpc_decode_batch failed")
        k[0] += 1
    ms = _time_ms(step, steps)
    return {"entry": "ldpc_decode_batch (fused frame-resident persistent kernel)", "ms_per_step": ms,
            "mbps": F * n / (ms * 1e-3) / 1e6, "step_floor": floor_frac(h.edges, n, 4, F * T, ms)}


def extra_workloads(only=None):
    """The other seeded workloads, each timed with HIP events on the device:
    - gallager504 (FP64, 1000 frames, 20 iterations, early stop): plain and batch;
    - qc_mix (12 codes, 16384 frames, 10 iterations, early stop): one batched
      launch vs twelve plain per-code launches (identical outputs), the batch
      with the default launch shape, after ldpc_autotune_batch, and replayed
      from a HIP-graph plan;
    - stair64800 (256 frames, 50 iterations, early stop): plain path and
      ldpc_decode_batch (which takes the plain kernels for this code).
    `only` names one of them to time alone.
    Each carries the whole step's algorithmic-floor fraction (floor_frac)
    over the iterations its frames actually ran."""
    import torch

    import paper_1812_06545_amd as L
    from workloads import configs
    out = {}

    def plain_and_batch(batches, dtype, reps, tune=False):
        hs = [L.Code.from_workload(b.code) for b in batches]
        jobs = [L.Job(hh, torch.from_numpy(b.llr).cuda(), b.max_iter, early_stop=b.early_stop)
                for hh, b in zip(hs, batches)]
        wsz = max(L.ldpc_workspace_bytes(hh, dtype, b.llr.shape[0], b.max_iter) for hh, b in zip(hs, batches))
        ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")

        def plain():
            for hh, j in zip(hs, jobs):
                L.decode(hh, j.llr, j.max_iter, early_stop=j.early_stop, workspace=ws)
        cj = [j.c_struct() for j in jobs]
        bw = L.ldpc_batch_workspace_bytes(cj, dtype)
        bws = torch.empty(max(bw, 1), dtype=torch.uint8, device="cuda")

        def batched():
            if L.ldpc_decode_batch(cj, dtype, bws, bw) != 0:
                raise RuntimeError("ldpc_decode_batch failed")
        bits = sum(b.llr.shape[0] * b.code.n for b in batches)
        tp, tb = _time_ms(plain, reps), _time_ms(batched, reps)
        frames = sum(b.llr.shape[0] for b in batches)
        frame_iters = [float(j.iters.float().sum().item()) for j in jobs]
        mean_it = sum(frame_iters) / frames
        tsize = 8 if dtype == torch.float64 else 4
        # floor bytes summed over the jobs' codes
        fb = sum(fi * (2 * tsize * b.code.edges + tsize * b.code.n) for fi, b in zip(frame_iters, batches))

        def frac(ms):
            return {"floor_bytes": fb, "achieved_gbs": fb / (ms * 1e-3) / 1e9,
                    "frac": fb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        res = {"plain_ms": tp, "plain_mbps": bits / (tp * 1e-3) / 1e6, "batch_ms": tb,
               "batch_mbps": bits / (tb * 1e-3) / 1e6, "mean_iters": mean_it,
               "plain_floor": frac(tp), "batch_floor": frac(tb)}
        if tune:
            L.ldpc_autotune_batch(cj, dtype, bws, bw)
            chosen = L.ldpc_batch_launch_config(cj, dtype)
            per_job = L.ldpc_batch_job_threads(cj, dtype)
            tt = _time_ms(batched, reps)
            plan = L.Plan(jobs)
            tg = _time_ms(plan.launch, reps)
            plan.close()
            L.ldpc_tuning_clear()  # later workloads are measured with the defaults
            res.update({"batch_tuned_ms": tt, "batch_tuned_mbps": bits / (tt * 1e-3) / 1e6,
                        "tuned_threads": chosen["threads"], "tuned_threads_per_job": per_job,
                        "tuned_frames_per_group": chosen["frames_per_group"],
                        "plan_replay_ms": tg, "plan_replay_mbps": bits / (tg * 1e-3) / 1e6,
                        "batch_tuned_floor": frac(tt)})
        return res

    if only in (None, "gallager504_f64"):
        out["gallager504_f64"] = plain_and_batch([configs.gallager504()], torch.float64, 5)
    if only in (None, "qc_mix_16384"):
        out["qc_mix_16384"] = plain_and_batch(configs.qc_mix(), torch.float32, 5, tune=True)
    if only in (None, "stair64800"):
        st = plain_and_batch([configs.stair64800()], torch.float32, 3)
        st["batch_entry"] = "ldpc_decode_batch routes this code to the plain kernels (too large for one workgroup's LDS)"
        out["stair64800"] = st
    return out


def layered_workloads(steps):
    """The layered schedule (LDPC_LAYERED), timed with HIP events:
    - qc1944 at 2.0 dB, 4096 frames, 10 passes fixed, on the plain path (one
      launch per layer; the layer kernel's achieved bandwidth: per edge and
      frame a layer reads r and L and writes both, 16 bytes, 12 on the first
      pass, which reads no r) and on the fused frame-resident kernel;
    - time to decode with early stop (max 20) against flooding on the same
      inputs, both paths: qc1944 code at 3.5 dB and gallager504 (FP64) at 2.0 dB.
    Fused-kernel timings here follow ldpc_autotune_batch for their shape."""
    import torch

    import paper_1812_06545_amd as L
    from workloads import configs
    out = {}
    b = configs.qc1944(2.0)
    F, n, E = b.llr.shape[0], b.code.n, b.code.edges
    h = L.Code.from_workload(b.code)
    llr = torch.from_numpy(b.llr).cuda()
    ws = torch.empty(L.ldpc_workspace_bytes(h, torch.float32, F, 10), dtype=torch.uint8, device="cuda")
    # the step time without per-launch events (120 short launches per decode
    # make their cost visible), then the kernel times in a separate profiled run
    ms = _time_ms(lambda: L.decode(h, llr, 10, layered=True, workspace=ws), steps)
    torch.cuda.synchronize()
    L.ldpc_profile_collect()
    L.ldpc_profile_enable(True)
    _time_ms(lambda: L.decode(h, llr, 10, layered=True, workspace=ws), steps)
    L.ldpc_profile_enable(False)
    prof = L.ldpc_profile_collect()
    kms, kcount = prof["check"]
    fp = (F + 63) // 64 * 64
    layers = L.ldpc_code_layers(h)[0]
    per_decode = fp * (12 * E + 9 * 16 * E)
    achieved = per_decode * (kcount / (10 * layers)) / (kms * 1e-3) / 1e9 if kcount else None
    fused_ms = _batch_ms(L, [(h, llr, 10, False, True)], torch.float32, steps, tune=True)
    chain = copy_chain(per_decode / (10 * layers), 10 * layers) if kcount else None
    out["qc1944_2dB_10passes"] = {
        "plain_ms": ms, "plain_mbps": F * n / (ms * 1e-3) / 1e6, "layers": layers,
        "layer_kernel": {"launches": kcount, "avg_us": kms * 1e3 / max(kcount, 1),
                         "bytes_per_decode": per_decode, "achieved_gbs": achieved,
                         "frac_of_peak": achieved / HBM_PEAK_GBS if achieved else None,
                         "copy_chain": chain,
                         "frac_of_copy_chain": achieved / chain["gbs"] if chain and achieved else None},
        "batch_ms": fused_ms, "batch_mbps": F * n / (fused_ms * 1e-3) / 1e6}

    def converge(batch, dtype, T, reps):
        hh = L.Code.from_workload(batch.code)
        x = torch.from_numpy(batch.llr).cuda()
        wsz = torch.empty(L.ldpc_workspace_bytes(hh, dtype, x.shape[0], T), dtype=torch.uint8, device="cuda")
        bits = x.shape[0] * batch.code.n
        res = {}
        for name, lay in (("flooding", False), ("layered", True)):
            got = {}

            def run():
                got["o"] = L.decode(hh, x, T, early_stop=True, layered=lay, workspace=wsz)
            t = _time_ms(run, reps)
            tb = _batch_ms(L, [(hh, x, T, True, lay)], dtype, reps, tune=True)
            it = got["o"][1].float()
            res[name] = {"plain_ms": t, "plain_mbps": bits / (t * 1e-3) / 1e6, "batch_ms": tb,
                         "batch_mbps": bits / (tb * 1e-3) / 1e6, "mean_iters": float(it.mean().item()),
                         "unconverged": float((it == T).float().mean().item())}
        return res
    out["qc1944_3.5dB_early_stop20"] = converge(configs.qc1944(3.5), torch.float32, 20, 5)
    out["gallager504_f64_early_stop20"] = converge(configs.gallager504(), torch.float64, 20, 5)
    return out


def minsum_workloads(steps):
    """The min-sum check rule (LDPC_MIN_SUM), HIP-event timed:
    - qc1944 2.0 dB, 4096 frames, 10 iterations, normalised min-sum (scale
      0.75), plain flooding path: Mbit/s and the min-sum check kernel's
      achieved bandwidth on the sum-product check kernel's algorithmic bytes
      (no transcendentals: the kernel is a pure HBM stream); the fused path
      and the layered schedule on the same input;
    - early stop (max 20) at 3.5 dB against sum-product, plain flooding."""
    import torch

    import paper_1812_06545_amd as L
    from workloads import configs
    out = {}
    b = configs.qc1944(2.0)
    F, n, E = b.llr.shape[0], b.code.n, b.code.edges
    h = L.Code.from_workload(b.code)
    x = torch.from_numpy(b.llr).cuda()
    ws = torch.empty(L.ldpc_workspace_bytes(h, torch.float32, F, 20), dtype=torch.uint8, device="cuda")

    def plain(layered=False, T=10, es=False, llr=x, rule="minsum"):
        return lambda: L.decode(h, llr, T, early_stop=es, layered=layered, rule=rule, ms_scale=0.75, workspace=ws)
    ms = _time_ms(plain(), steps)
    L.ldpc_profile_collect()
    L.ldpc_profile_enable(True)
    _time_ms(plain(), steps)
    L.ldpc_profile_enable(False)
    kms, kcount = L.ldpc_profile_collect()["check"]
    bytes_per_launch = F * ((4 * E + 4 * n) + 9 * (8 * E + 4 * n)) / 10
    achieved = bytes_per_launch / (kms / kcount * 1e-3) / 1e9 if kcount else None
    fused = _batch_ms(L, [(h, x, 10, False, False, "minsum", 0.75)], torch.float32, steps, tune=True)
    lay = _time_ms(plain(layered=True), steps)
    out["qc1944_2dB_10it_nms0.75"] = {
        "plain_ms": ms, "plain_mbps": F * n / (ms * 1e-3) / 1e6,
        "check_kernel": {"avg_us": kms * 1e3 / max(kcount, 1), "bytes_per_launch": bytes_per_launch,
                         "achieved_gbs": achieved, "frac_of_peak": achieved / HBM_PEAK_GBS if achieved else None},
        "batch_ms": fused, "batch_mbps": F * n / (fused * 1e-3) / 1e6,
        "layered_plain_ms": lay, "layered_plain_mbps": F * n / (lay * 1e-3) / 1e6}
    hi = torch.from_numpy(configs.qc1944(3.5).llr).cuda()
    res = {}
    for name, rule in (("sum_product", "spa"), ("min_sum_0.75", "minsum")):
        got = {}

        def run():
            got["o"] = plain(T=20, es=True, llr=hi, rule=rule)()
        t = _time_ms(run, 5)
        it = got["o"][1].float()
        res[name] = {"plain_ms": t, "mean_iters": float(it.mean().item()),
                     "unconverged": float((it == 20).float().mean().item())}
    out["qc1944_3.5dB_early_stop20"] = res
    return out


def mstream_run():
    """The paper's multi-stream structure (ldpc_mstream_run: W host workers,
    each with its own stream and F frames per batch; host LLRs in, host bits
    out, copies included) on qc1944 frames at 2.0 dB, 10 iterations, against
    the same frames through one ldpc_decode_batch launch per 32768-frame
    batch with the same host copies around it; throughput and the host CPU
    time the structure costs (workers wait on blocking events)."""
    import numpy as np
    import torch

    import paper_1812_06545_amd as L
    from workloads import configs
    b = configs.qc1944(2.0)
    h = L.Code.from_workload(b.code)
    total = 32768
    llr = np.ascontiguousarray(np.tile(b.llr, (total // b.llr.shape[0], 1)))
    bits = np.zeros((total, b.code.n), np.uint8)
    iters = np.zeros(total, np.int32)
    rows = []
    for W, F in ((1, 4096), (2, 4096), (4, 2048), (8, 1024), (4, 4096), (8, 4096)):
        L.ldpc_mstream_run(h, W, F, min(2 * W, total // F), 10, 0, 1, llr, bits, iters)  # warm-up
        rc, st = L.ldpc_mstream_run(h, W, F, total // F, 10, 0, 1, llr, bits, iters)
        if rc != 0:
            raise RuntimeError(f"ldpc_mstream_run failed: {rc}")
        rows.append({"workers": W, "frames_per_batch": F, "mbps": st["mbps"], "wall_ms": st["wall_ms"],
                     "host_cores_busy": st["cpu_cores_busy"], "host_cpu_load": st["cpu_load"]})
    # one device-side launch over all frames, with the same host copies around it
    x = torch.empty((total, b.code.n), dtype=torch.float32, pin_memory=True)
    job = L.Job(h, torch.empty((total, b.code.n), dtype=torch.float32, device="cuda"), 10, want_posterior=False)
    cj = [job.c_struct()]
    nb = L.ldpc_batch_workspace_bytes(cj, torch.float32)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")
    out_bits = torch.empty((total, b.code.n), dtype=torch.uint8, pin_memory=True)

    def one():
        x.numpy()[:] = llr
        job.llr.copy_(x, non_blocking=True)
        if L.ldpc_decode_batch(cj, torch.float32, ws, nb) != 0:
            raise RuntimeError("ldpc_decode_batch failed")
        out_bits.copy_(job.bits, non_blocking=True)
        torch.cuda.synchronize()
        bits[:] = out_bits.numpy()
    one()
    t0 = time.perf_counter()
    one()
    wall = time.perf_counter() - t0
    return {"workload": "qc1944 2.0 dB frames (4096 tiled to 32768), 10 iterations, FP32, host LLRs in and host "
                        "bits out",
            "multi_stream": rows,
            "one_launch_with_copies": {"mbps": total * b.code.n / wall / 1e6, "wall_ms": wall * 1e3}}


def _batch_ms(L, items, dtype, reps, tune=False):
    """HIP-event time of one ldpc_decode_batch over items (handle, llr tensor,
    max_iter, early_stop, layered[, rule, min-sum scale]); with tune, after
    ldpc_autotune_batch has picked the workgroup size for this batch shape."""
    import torch
    jobs = [L.Job(hh, x, T, early_stop=es, layered=lay, rule=rest[0] if rest else "spa",
                  ms_scale=rest[1] if rest else 1.0) for hh, x, T, es, lay, *rest in items]
    if tune:
        L.autotune_batch(jobs)
    cj = [j.c_struct() for j in jobs]
    nb = L.ldpc_batch_workspace_bytes(cj, dtype)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda")

    def run():
        if L.ldpc_decode_batch(cj, dtype, ws, nb) != 0:
            raise RuntimeError("ldpc_decode_batch failed")
    t = _time_ms(run, reps)
    if tune:
        L.ldpc_tuning_clear()  # later workloads are measured with the defaults
    return t


def copy_chain(bytes_moved, count):
    """The same streaming copy as copy_probe, as `count` dependent launches
    that each move `bytes_moved` bytes (read + write), timed between two HIP
    events (median of 5): the rate a chain of launches of that size can reach,
    ramp-up and drain included."""
    import torch

    import paper_1812_06545_amd as L
    nbytes = max(16, int(bytes_moved) // 2 // 16 * 16)
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        L.ldpc_copy_probe(dst, src, nbytes)
    torch.cuda.synchronize()
    times = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(count):
            if L.ldpc_copy_probe(dst, src, nbytes) != 0:
                raise RuntimeError("ldpc_copy_probe failed")
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / count)
    ms = sorted(times)[len(times) // 2]
    return {"bytes_per_launch": 2 * nbytes, "launches": count, "us_per_launch": ms * 1e3,
            "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def copy_probe(mb):
    """Achievable HBM bandwidth: the library's streaming copy kernel over `mb`
    MiB (read + write bytes per second), median of 5 HIP-event timings."""
    import torch

    import paper_1812_06545_amd as L
    nbytes = mb << 20
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    times = []
    for rep in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        if L.ldpc_copy_probe(dst, src, nbytes) != 0:
            raise RuntimeError("ldpc_copy_probe failed")
        e1.record()
        torch.cuda.synchronize()
        if rep:
            times.append(e0.elapsed_time(e1))
    ms = sorted(times)[len(times) // 2]
    return {"bytes": 2 * nbytes, "ms": ms, "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def serve_run(seconds, rate, max_group_frames=1024, max_inflight=3, warmup_s=0.0):
    """Open-loop serving run: Poisson arrivals of decode requests (1-64 frames
    of one of the 12 QC codes, Eb/N0 uniform in [1, 3] dB per frame, 10
    iterations with early stop) submitted at their scheduled times; latency is
    completion minus scheduled arrival, so a backlog is not hidden.  The
    first warmup_s seconds of the same traffic run before the measured window:
    the server's statistics are reset when the schedule crosses into it (a
    request admitted before and completed after counts in the window).  The
    submitter's own lateness (time past the scheduled arrival when a request
    is handed over) is reported beside the latencies: it is part of them."""
    import ctypes
    import gc

    import numpy as np

    import paper_1812_06545_amd as L
    from workloads import configs

    pool = configs.ServePool(per_code=512)
    handles = [L.Code.from_workload(c) for c in pool.codes]
    llr = [pool.llr_pool(i) for i in range(12)]
    outs = [(np.zeros((64, c.n), np.uint8), np.zeros(64, np.int32)) for c in pool.codes]
    sched = configs.serve_schedule(warmup_s + seconds, rate)
    # every request's host pointers are worked out before the clock starts
    plan = []
    for k, rq in enumerate(sched):
        n = pool.codes[rq.code_id].n
        start = (k * 37) % (512 - rq.frames + 1)
        plan.append((int(rq.t_arrival * 1e9), rq.code_id, rq.frames,
                     llr[rq.code_id].ctypes.data + start * n * llr[rq.code_id].itemsize,
                     outs[rq.code_id][0].ctypes.data, outs[rq.code_id][1].ctypes.data))
    lag = np.zeros(len(plan), np.int64)
    srv = L.ldpc_server_create(handles, 512 << 20, max_inflight=max_inflight, max_group_frames=max_group_frames)
    try:
        # warm-up: one request per code
        for cid in range(12):
            st, t = L.ldpc_server_submit(srv, cid, 8, 10, 1, llr[cid][:8], outs[cid][0][:8], outs[cid][1][:8])
            L.ldpc_server_wait(srv, t)
        L.ldpc_server_stats_get(srv, reset=True)
        submit, ticket, mono = L._lib.ldpc_server_submit, ctypes.c_uint64(), time.monotonic_ns
        ticket_ref = ctypes.byref(ticket)
        rejected = 0
        gc.collect()
        gc.disable()
        reset_at = int(warmup_s * 1e9)
        window = warmup_s <= 0
        first = pending = 0
        try:
            t0 = mono() + 2_000_000
            t_window = t0
            for i, (off, cid, frames, lp, bp, ip) in enumerate(plan):
                at = t0 + off
                if not window and off >= reset_at:
                    t_window = t0 + reset_at
                    while mono() < t_window:
                        pass
                    s0 = L.ldpc_server_stats_get(srv, reset=True)  # the counts up to the reset
                    pending = s0["submitted"] - s0["completed"] - s0["failed"] - s0["cancelled"]
                    rejected, first, window = 0, i, True
                now = mono()
                while now < at:
                    now = mono()
                lag[i] = now - at
                rejected += submit(srv, cid, frames, 10, 1, lp, bp, ip, None, at, ticket_ref) != 0
        finally:
            gc.enable()
        while True:  # requests still in flight at the reset complete inside the window
            s = L.ldpc_server_stats_get(srv)
            if s["completed"] + s["failed"] >= s["submitted"] + pending:
                break
            time.sleep(0.001)
        wall = (time.monotonic_ns() - t_window) / 1e9
    finally:
        L.ldpc_server_destroy(srv)
    lag_ms = np.sort(lag[first:]) / 1e6
    return {"workload": "serve: Poisson arrivals, 1-64 frames of one of 12 QC codes (Z 27/54/81 x rate 1/2..5/6), "
                        "Eb/N0 U[1,3] dB, 10 iterations with early stop",
            "offered_req_per_s": rate, "duration_s": seconds, "warmup_s": warmup_s, "requests": s["completed"],
            "rejected": rejected,
            "failed": s["failed"], "p50_ms": s["p50_ms"], "p99_ms": s["p99_ms"], "p999_ms": s["p999_ms"],
            "max_ms": s["max_ms"],
            "max_ms_breakdown": {k: s["worst_" + k + "_ms"] for k in ("submit", "queue", "stage", "device", "copyout")},
            "max_step_ms": s["max_step_ms"],
            "max_host_ms": {k: s["max_" + k + "_ms"] for k in ("copy", "launch", "query")},
            "mbps": s["bits_completed"] / wall / 1e6, "launches": s["launches"],
            "mean_group_frames": s["mean_group_frames"], "max_queue_depth": s["max_queue_depth"],
            "submit_lag_p99_ms": float(lag_ms[int(0.99 * (lag_ms.size - 1))]) if lag_ms.size else 0.0,
            "submit_lag_max_ms": float(lag_ms[-1]) if lag_ms.size else 0.0}


def cpu_baseline(batches, T, seconds):
    """The oracle (plain FP64 C, as committed) on the host cores, over the
    step's Eb/N0 batches in turn, frame blocks of each, until about `seconds`
    of wall time have been spent (or every frame of every batch decoded)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS") or min(16, os.cpu_count() or 1))
    code = batches[0].code
    probe = 2 * threads
    t0 = time.perf_counter()
    oracle.decode(code, batches[0].llr[:probe], T, False, nthreads=threads, want_trace=False)
    per_frame = (time.perf_counter() - t0) / probe
    per_batch = int(min(batches[0].llr.shape[0], max(probe, seconds / len(batches) / max(per_frame, 1e-9))))
    frames = 0
    t0 = time.perf_counter()
    for b in batches:
        oracle.decode(code, b.llr[:per_batch], T, False, nthreads=threads, want_trace=False)
        frames += per_batch
    wall = time.perf_counter() - t0
    snrs = "/".join(f"{b.ebn0_db:g}" for b in batches)
    # the same oracle on one thread, over a smaller sample (about a tenth of the time)
    one = max(1, int(seconds / 10 / max(per_frame * threads, 1e-9)))
    one = min(one, batches[0].llr.shape[0])
    t1 = time.perf_counter()
    oracle.decode(code, batches[2].llr[:one], T, False, nthreads=1, want_trace=False)
    wall1 = time.perf_counter() - t1
    return {"value": frames * code.n / wall / 1e6, "unit": "Mbit/s", "cores": threads, "kind": "oracle",
            "sample": f"first {per_batch} of 4096 frames of each of the {snrs} dB batches ({frames} frames), "
                      f"{T} iterations, FP64, {threads} OpenMP threads, {wall:.1f} s wall "
                      f"({wall * threads:.0f} core-seconds)",
            "single_thread": {"value": one * code.n / wall1 / 1e6, "unit": "Mbit/s", "cores": 1,
                              "sample": f"first {one} frames of the {batches[2].ebn0_db:g} dB batch, {T} iterations, "
                                        f"FP64, 1 thread, {wall1:.1f} s wall"}}

if __name__ == "__main__":
    main()
