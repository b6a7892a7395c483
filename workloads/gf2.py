"""GF(2) linear algebra for building test inputs: rank, systematic encoder.

Input generation only: this module turns a parity-check matrix H into an
encoder so that random codewords (the transmitted words of Section II) can be
drawn.  It holds none of the decoder's arithmetic.

Matrices are handled bit-packed (rows of uint64 words) so that the 972 x 1944
quasi-cyclic matrices eliminate in well under a second.
"""
from __future__ import annotations

import numpy as np


def pack_rows(H: np.ndarray) -> np.ndarray:
    """Pack a dense 0/1 matrix (m, n) into (m, ceil(n/64)) uint64 words (bit j of word w = column 64w+j)."""
    H = np.asarray(H, dtype=np.uint8)
    m, n = H.shape
    nw = (n + 63) // 64
    padded = np.zeros((m, nw * 64), dtype=np.uint8)
    padded[:, :n] = H
    bits = padded.reshape(m, nw, 64).astype(np.uint64)
    weights = (np.uint64(1) << np.arange(64, dtype=np.uint64))
    return (bits * weights).sum(axis=2, dtype=np.uint64)


def unpack_rows(P: np.ndarray, n: int) -> np.ndarray:
    m, nw = P.shape
    shifts = np.arange(64, dtype=np.uint64)
    bits = ((P[:, :, None] >> shifts) & np.uint64(1)).astype(np.uint8)
    return bits.reshape(m, nw * 64)[:, :n]


def rref(H: np.ndarray):
    """Reduced row echelon form over GF(2).

    Returns (R, pivots): R is the dense (rank, n) reduced matrix, pivots the
    pivot column of each of its rows (strictly increasing).
    """
    H = np.asarray(H, dtype=np.uint8)
    m, n = H.shape
    P = pack_rows(H)
    pivots = []
    row = 0
    for c in range(n):
        if row == m:
            break
        w, b = divmod(c, 64)
        bit = np.uint64(1) << np.uint64(b)
        col_set = (P[row:, w] & bit) != 0
        idx = np.flatnonzero(col_set)
        if idx.size == 0:
            continue
        p = row + idx[0]
        if p != row:
            P[[row, p]] = P[[p, row]]
        hit = (P[:, w] & bit) != 0
        hit[row] = False
        P[hit] ^= P[row]
        pivots.append(c)
        row += 1
    return unpack_rows(P[:row], n), np.asarray(pivots, dtype=np.int64)


def rank(H: np.ndarray) -> int:
    return int(rref(H)[1].size)


class SystematicEncoder:
    """Encoder for the code {c : H c = 0 (mod 2)} built from the RREF of H.

    The non-pivot columns carry the k = n - rank(H) information bits; each
    pivot bit is the GF(2) sum of the information bits its RREF row selects.
    A rank-deficient H (k > n - m) is handled naturally.
    """

    def __init__(self, H: np.ndarray):
        H = np.asarray(H, dtype=np.uint8)
        self.m, self.n = H.shape
        R, piv = rref(H)
        self.pivots = piv
        mask = np.ones(self.n, dtype=bool)
        mask[piv] = False
        self.info = np.flatnonzero(mask)
        self.k = int(self.info.size)
        # pivot_bits = A @ info_bits (mod 2); A is (rank, k)
        self.A = R[:, self.info].astype(np.float32)

    def encode(self, u: np.ndarray) -> np.ndarray:
        u = np.atleast_2d(np.asarray(u, dtype=np.uint8))
        assert u.shape[1] == self.k
        c = np.zeros((u.shape[0], self.n), dtype=np.uint8)
        c[:, self.info] = u
        if self.pivots.size:
            par = (u.astype(np.float32) @ self.A.T)  # exact: sums stay far below 2^24
            c[:, self.pivots] = (par.astype(np.int64) & 1).astype(np.uint8)
        return c

    def random_codewords(self, count: int, seed: int) -> np.ndarray:
        rng = np.random.Generator(np.random.PCG64(seed))
        u = rng.integers(0, 2, size=(count, self.k), dtype=np.uint8)
        return self.encode(u)


def nullspace_basis(H: np.ndarray) -> np.ndarray:
    """Rows form a basis of the code (k, n)."""
    enc = SystematicEncoder(H)
    return enc.encode(np.eye(enc.k, dtype=np.uint8))
