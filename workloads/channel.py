"""BPSK over AWGN: channel LLRs for the decoder's inputs.

Conventions: bit 0 -> +1, bit 1 -> -1; y = x + sigma * N(0, 1) with
sigma^2 = 1 / (2 R 10^(Eb/N0 / 10)); the channel LLR is
L = ln P(c=0|y) / P(c=1|y) = 2 y / sigma^2 (positive favours bit 0).
"""
from __future__ import annotations

import numpy as np


def sigma2(ebn0_db: float, rate: float) -> float:
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def bpsk_awgn_llr(codewords: np.ndarray, ebn0_db, rate: float, seed: int,
                  dtype=np.float32) -> np.ndarray:
    """LLRs (F, n) for codewords (F, n) uint8.  ``ebn0_db`` may be a scalar or a
    per-frame array (the serving workload draws one SNR per request)."""
    c = np.asarray(codewords, dtype=np.uint8)
    F, n = c.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    eb = np.broadcast_to(np.asarray(ebn0_db, dtype=np.float64).reshape(-1, 1) if np.ndim(ebn0_db) else
                         np.float64(ebn0_db), (F, 1))
    s2 = 1.0 / (2.0 * rate * 10.0 ** (eb / 10.0))
    y = (1.0 - 2.0 * c) + np.sqrt(s2) * rng.standard_normal((F, n))
    return (2.0 * y / s2).astype(dtype)


def noiseless_llr(codewords: np.ndarray, amplitude: float, dtype=np.float64) -> np.ndarray:
    c = np.asarray(codewords, dtype=np.float64)
    return (amplitude * (1.0 - 2.0 * c)).astype(dtype)
