"""The oracle against its pins (mathematics, not itself).  CPU only."""
import numpy as np
import pytest

import pins
from mapref import all_codewords
from workloads import codes, gf2


def _dec(oracle):
    return lambda code, llr, T, es: oracle.decode(code, llr, T, es)


@pytest.mark.parametrize("check", pins.ALL, ids=lambda f: f.__name__)
def test_pin(check, oracle_mod):
    check(_dec(oracle_mod))


def _paper_H():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_eq1_H.txt")
    return np.loadtxt(path, comments="#", dtype=np.uint8)


def test_paper_eq1_structure():
    """Section II, eq. (1): 5 checks x 10 variables, every variable in two
    checks, every check on four variables; GF(2) rank 4 (the five rows sum to
    zero), hence 2^6 = 64 codewords by enumeration; girth 6."""
    H = _paper_H()
    assert H.shape == (5, 10)
    assert (H.sum(axis=0) == 2).all() and (H.sum(axis=1) == 4).all()
    code = codes.Code.from_dense(H)
    assert gf2.rank(H) == 4
    assert len(all_codewords(code)) == 64
    assert codes.count_4cycles(code) == 0
    enc = gf2.SystematicEncoder(H)
    assert enc.k == 6
    basis = gf2.nullspace_basis(H)
    assert ((basis.astype(int) @ H.T.astype(int)) % 2 == 0).all()


def test_paper_eq1_decodes(oracle_mod):
    """Noiseless codewords of the eq. (1) code decode at iteration 0; a single
    flipped bit at moderate reliability is corrected."""
    code = codes.Code.from_dense(_paper_H())
    cw = all_codewords(code)
    out = oracle_mod.decode(code, 2.0 * (1.0 - 2.0 * cw.astype(float)), 10, True)
    assert (out["iters"] == 0).all() and (out["bits"] == cw).all()
    llr = 2.0 * (1.0 - 2.0 * cw.astype(float))
    llr[:, 0] = -0.5 * (1.0 - 2.0 * cw[:, 0])  # weak wrong-sign channel value on bit 0
    out = oracle_mod.decode(code, llr, 10, True)
    assert (out["bits"] == cw).all()


def test_hamming74_structure():
    code = codes.hamming74()
    assert gf2.rank(code.to_dense()) == 3
    assert len(all_codewords(code)) == 16
    assert codes.count_4cycles(code) > 0


def test_oracle_rejects_duplicate_edges(oracle_mod):
    code = codes.Code(1, 3, np.array([0, 3], np.int32), np.array([0, 1, 1], np.int32))
    with pytest.raises(ValueError):
        oracle_mod.decode(code, np.zeros((1, 3)), 1, False)


def test_oracle_threads_identical(oracle_mod):
    code, cw, llr = pins._gallager_noisy(16, 40)
    a = oracle_mod.decode(code, llr, 20, True, nthreads=1)
    b = oracle_mod.decode(code, llr, 20, True, nthreads=4)
    for k in ("bits", "iters", "posterior", "cond"):
        assert (a[k] == b[k]).all()
