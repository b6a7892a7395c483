"""Seeded parity inputs on codes chosen for their row and column degrees, so
that every kernel body the library instantiates is reached (the list and
what each case covers are in test_gpu_degrees).  No decoder arithmetic."""
import functools

import numpy as np

from workloads import channel, codes, gf2

FRAMES = 200

# name -> (code builder, Eb/N0 dB)
CASES = {
    "qc_d16": (lambda: codes.qc_row_degrees([16, 14, 12, 10, 9, 9], 16, 27, 701), 3.0),
    "qc_d24": (lambda: codes.qc_row_degrees([24, 22, 20, 18, 17], 24, 27, 702), 3.5),
    "qc_d32": (lambda: codes.qc_row_degrees([32, 30, 28, 26, 25, 20], 32, 27, 703), 3.0),
    "qc_d64": (lambda: codes.qc_row_degrees([64, 57, 48, 40, 33], 64, 11, 704), 4.0),
    "csr_d25_32": (lambda: codes.random_rows(40, 400, 25, 32, 705, dense_col=True), 3.5),
    "csr_d33_64": (lambda: codes.random_rows(24, 600, 33, 64, 706, dense_col=True), 4.5),
    "spc30": (lambda: codes.single_parity_check(30), 3.0),
    "spc40": (lambda: codes.single_parity_check(40), 3.0),
    "spc64": (lambda: codes.single_parity_check(64), 3.0),
}
NAMES = list(CASES)
FUSED_FITS = {"qc_d16", "qc_d24", "qc_d32", "csr_d25_32", "spc30"}


@functools.lru_cache(maxsize=None)
def workload(name, dtype):
    build, ebn0 = CASES[name]
    code = build()
    cw = gf2.SystematicEncoder(code.to_dense()).random_codewords(FRAMES, 710 + NAMES.index(name))
    rate = 1.0 - code.m / code.n
    llr = channel.bpsk_awgn_llr(cw, ebn0, rate, 730 + NAMES.index(name), dtype=np.float64)
    return code, (llr.astype(np.float32) if dtype == "f32" else llr)
