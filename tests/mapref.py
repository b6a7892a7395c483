"""Independent references for pinning the oracle: exact bitwise MAP by brute
force over all 2^n words, and a dense GF(2) syndrome.  Written without the
oracle and without the sum-product rule."""
from __future__ import annotations

import itertools

import numpy as np


def all_codewords(code) -> np.ndarray:
    """Every word c in {0,1}^n with H c = 0 (mod 2), by enumeration (n <= 20)."""
    n = code.n
    assert n <= 20
    H = code.to_dense().astype(np.int64)
    words = np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.int64)
    ok = ((words @ H.T) % 2 == 0).all(axis=1)
    return words[ok].astype(np.uint8)


def map_llr(code, llr: np.ndarray) -> np.ndarray:
    """Exact bitwise MAP posterior LLRs.

    With L_j = ln P(c_j=0|y_j)/P(c_j=1|y_j), the likelihood of a word c is
    proportional to exp(-sum_j c_j L_j); the posterior LLR of bit n is
    LSE over codewords with c_n = 0 minus LSE over codewords with c_n = 1.
    """
    C = all_codewords(code).astype(np.float64)
    llr = np.atleast_2d(np.asarray(llr, dtype=np.float64))
    out = np.zeros_like(llr)
    for f in range(llr.shape[0]):
        metric = -(C @ llr[f])
        for j in range(code.n):
            a = metric[C[:, j] == 0]
            b = metric[C[:, j] == 1]
            out[f, j] = _lse(a) - _lse(b)
    return out


def _lse(v):
    mx = np.max(v)
    return mx + np.log(np.sum(np.exp(v - mx)))


def dense_syndrome(code, bits: np.ndarray) -> np.ndarray:
    H = code.to_dense().astype(np.int64)
    return (np.atleast_2d(bits).astype(np.int64) @ H.T) % 2


def depth1_tree(code, root: int):
    """The depth-1 computation tree of variable `root`: the root joined to
    each of its checks, and every other variable of those checks as a fresh
    leaf (a variable met through two checks appears twice).  Returns the tree
    as a code (the root is variable 0) and, per tree variable, the variable
    of `code` it copies.  One flooding iteration at the root sees exactly
    this tree, so its posterior there is the tree's exact MAP."""
    from workloads.codes import Code

    H = code.to_dense()
    src = [root]
    rows = []
    for m in np.flatnonzero(H[:, root]):
        members = [0]
        for j in np.flatnonzero(H[m]):
            if j == root:
                continue
            members.append(len(src))
            src.append(int(j))
        rows.append(members)
    tree = Code.from_row_lists(len(rows), len(src), rows, f"depth-1 tree of {root}")
    return tree, np.array(src)
