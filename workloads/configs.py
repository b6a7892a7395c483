"""The five seeded decoding workloads (codes, codewords, channel LLRs).

Synthetic stand-ins for the paper's test codes (lengths 576 to 9972 at 5 or
10 iterations, Section IV), whose matrices are not published with it.

  gallager504   (3,6)-regular n=504, FP64, 1000 frames, 2.0 dB, 20 iters, early stop
  qc1944        QC 12x24 base, Z=81 (n=1944), FP32, 4096 frames, 1.0/1.5/2.0/2.5 dB, 10 iters fixed
  qc_mix        12 QC codes (Z in 27/54/81 x rate 1/2, 2/3, 3/4, 5/6), 16384 frames, 2.0 dB, 10 iters, early stop
  serve         Poisson request stream (20k req/s, 1-64 frames, one of the 12 QC codes, 1-3 dB)
  stair64800    staircase irregular n=64800, 256 frames, 1.0 dB, 50 iters, early stop
"""
from __future__ import annotations

import dataclasses
import functools
from typing import List, Optional

import numpy as np

from . import channel, codes, gf2

QC_MIX_Z = (27, 54, 81)
QC_MIX_MB = (12, 8, 6, 4)
RATE_OF_MB = {12: 1 / 2, 8: 2 / 3, 6: 3 / 4, 4: 5 / 6}


@dataclasses.dataclass
class Batch:
    code: codes.Code
    codewords: np.ndarray       # (F, n) uint8
    llr: np.ndarray             # (F, n) float32 / float64
    rate: float                 # nominal rate used for Eb/N0 -> sigma
    ebn0_db: float
    max_iter: int
    early_stop: bool
    k: int                      # true information length n - rank(H)


@functools.lru_cache(maxsize=None)
def _encoder(code_key):
    kind, args = code_key
    code = _make_code(kind, args)
    if kind == "stair":
        return code, None
    return code, gf2.SystematicEncoder(code.to_dense())


def _make_code(kind, args):
    if kind == "gallager":
        return codes.gallager_regular(*args)
    if kind == "qc":
        return codes.qc_code(*args)
    if kind == "stair":
        return codes.staircase_irregular(*args)
    raise ValueError(kind)


def _codewords(code_key, count, seed):
    code, enc = _encoder(code_key)
    if enc is None:
        rng = np.random.Generator(np.random.PCG64(seed))
        u = rng.integers(0, 2, size=(count, code.m), dtype=np.uint8)
        return code, codes.staircase_encode(code, u), code.n - code.m
    return code, enc.random_codewords(count, seed), enc.k


def gallager504(frames: int = 1000) -> Batch:
    code, cw, k = _codewords(("gallager", (504, 3, 6, 101)), frames, 102)
    llr = channel.bpsk_awgn_llr(cw, 2.0, 0.5, 103, dtype=np.float64)
    return Batch(code, cw, llr, 0.5, 2.0, 20, True, k)


QC1944_SNRS = (1.0, 1.5, 2.0, 2.5)


def qc1944(ebn0_db: float = 2.0, frames: int = 4096) -> Batch:
    code, cw, k = _codewords(("qc", (12, 24, 81, 201)), frames, 202)
    noise_seed = 203 + QC1944_SNRS.index(ebn0_db) if ebn0_db in QC1944_SNRS else 207
    llr = channel.bpsk_awgn_llr(cw, ebn0_db, 0.5, noise_seed, dtype=np.float32)
    return Batch(code, cw, llr, 0.5, ebn0_db, 10, False, k)


def qc_mix_codes() -> List[codes.Code]:
    out = []
    for zi, Z in enumerate(QC_MIX_Z):
        for mi, mb in enumerate(QC_MIX_MB):
            out.append(_encoder(("qc", (mb, 24, Z, 301 + zi * 4 + mi)))[0])
    return out


def _qc_mix_key(idx):
    zi, mi = divmod(idx, 4)
    return ("qc", (QC_MIX_MB[mi], 24, QC_MIX_Z[zi], 301 + idx))


def qc_mix_counts(total: int = 16384) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(313))
    w = rng.permutation(np.arange(1, 13))
    counts = (total * w) // w.sum()
    counts[np.argsort(-w)[: total - counts.sum()]] += 1
    return counts.astype(np.int64)


def qc_mix(total: int = 16384, ebn0_db: float = 2.0) -> List[Batch]:
    out = []
    for idx, cnt in enumerate(qc_mix_counts(total)):
        mb = QC_MIX_MB[idx % 4]
        rate = RATE_OF_MB[mb]
        code, cw, k = _codewords(_qc_mix_key(idx), int(cnt), 320 + idx)
        llr = channel.bpsk_awgn_llr(cw, ebn0_db, rate, 340 + idx, dtype=np.float32)
        out.append(Batch(code, cw, llr, rate, ebn0_db, 10, True, k))
    return out


@dataclasses.dataclass
class ServeRequest:
    t_arrival: float            # scheduled arrival (s from start)
    code_id: int                # index into qc_mix_codes()
    frames: int
    ebn0_db: float


def serve_schedule(duration_s: float, rate_hz: float = 20000.0) -> List[ServeRequest]:
    rng_t = np.random.Generator(np.random.PCG64(401))
    rng_c = np.random.Generator(np.random.PCG64(402))
    rng_s = np.random.Generator(np.random.PCG64(403))
    n_est = int(duration_s * rate_hz * 1.2) + 64
    gaps = rng_t.exponential(1.0 / rate_hz, size=n_est)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    cnt = t.size
    code_id = rng_c.integers(0, 12, size=cnt)
    frames = rng_c.integers(1, 65, size=cnt)
    snr = rng_s.uniform(1.0, 3.0, size=cnt)
    return [ServeRequest(float(t[i]), int(code_id[i]), int(frames[i]), float(snr[i])) for i in range(cnt)]


class ServePool:
    """Pre-drawn codewords per QC code; a request takes a slice and gets noise
    from its own seed, so every request's LLRs are reproducible in isolation."""

    def __init__(self, per_code: int = 512):
        self.codes = qc_mix_codes()
        self.cw = []
        for idx in range(12):
            self.cw.append(_codewords(_qc_mix_key(idx), per_code, 360 + idx)[1])
        self.per_code = per_code

    def llr_pool(self, code_id: int) -> np.ndarray:
        """All pre-drawn frames of one code as LLRs, each frame at its own
        Eb/N0 drawn uniformly from [1, 3] dB (seeded); for load generation."""
        if not hasattr(self, "_llr"):
            self._llr = {}
        if code_id not in self._llr:
            rng = np.random.Generator(np.random.PCG64(405 + code_id))
            snr = rng.uniform(1.0, 3.0, size=self.per_code)
            rate = RATE_OF_MB[QC_MIX_MB[code_id % 4]]
            self._llr[code_id] = channel.bpsk_awgn_llr(self.cw[code_id], snr, rate, 420 + code_id, np.float32)
        return self._llr[code_id]

    def request_llr(self, req_index: int, req: ServeRequest) -> np.ndarray:
        cw_all = self.cw[req.code_id]
        start = (req_index * 37) % (self.per_code - req.frames + 1)
        cw = cw_all[start:start + req.frames]
        rate = RATE_OF_MB[QC_MIX_MB[req.code_id % 4]]
        return channel.bpsk_awgn_llr(cw, req.ebn0_db, rate, 404_000_000 + req_index, np.float32), cw


def stair64800(frames: int = 256) -> Batch:
    code, cw, k = _codewords(("stair", (64800, 501)), frames, 502)
    llr = channel.bpsk_awgn_llr(cw, 1.0, 0.5, 503, dtype=np.float32)
    return Batch(code, cw, llr, 0.5, 1.0, 50, True, k)
