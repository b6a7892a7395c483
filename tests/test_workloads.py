"""Pins for the seeded workload generators (CPU only): the stated structure of
every code (degrees, empty blocks, no 4-cycles), that the generated
codewords satisfy H by an independent dense GF(2) product, and that the
generators are deterministic."""
import numpy as np
import pytest

from mapref import dense_syndrome
from workloads import codes, configs, gf2


def _assert_codewords(code, cw):
    assert cw.dtype == np.uint8 and cw.shape[1] == code.n
    assert set(np.unique(cw).tolist()) <= {0, 1}
    assert (dense_syndrome(code, cw) == 0).all(), "a generated codeword violates H"
    assert cw.any(axis=1).sum() >= len(cw) - 1, "codewords should be random, not all-zero"


def test_gallager504_structure():
    """(3,6)-regular, n = 504, m = 252, no 4-cycles, k = n - rank(H)."""
    b = configs.gallager504(frames=64)
    code = b.code
    assert (code.m, code.n) == (252, 504)
    assert (code.row_degrees() == 6).all() and (code.col_degrees() == 3).all()
    assert codes.count_4cycles(code) == 0
    assert b.k == code.n - gf2.rank(code.to_dense())
    _assert_codewords(code, b.codewords)


def _check_qc(code, mb, Z):
    q = code.qc
    assert q is not None and (q["mb"], q["nb"], q["Z"]) == (mb, 24, Z)
    s = np.asarray(q["shifts"]).reshape(mb, 24)
    assert ((s == -1) | ((s >= 0) & (s < Z))).all()
    assert int((s == -1).sum()) == round(0.3 * mb * 24), "about 30% empty: exactly round(0.3 mb nb) blocks"
    assert ((s >= 0).sum(axis=0) > 0).all(), "an empty base column"
    assert (code.m, code.n) == (mb * Z, 24 * Z)
    # every block row contributes its non-empty block count to each of its Z rows
    deg = code.row_degrees().reshape(mb, Z)
    assert (deg == (s >= 0).sum(axis=1)[:, None]).all()
    # circulant structure: block (i, j) with shift t joins row i*Z + r to column j*Z + (r + t) mod Z
    H = code.to_dense()
    for i in range(mb):
        for j in range(24):
            blk = H[i * Z:(i + 1) * Z, j * Z:(j + 1) * Z]
            if s[i, j] < 0:
                assert not blk.any()
            else:
                want = np.roll(np.eye(Z, dtype=np.uint8), s[i, j], axis=1)
                assert (blk == want).all()


def test_qc1944_structure():
    b = configs.qc1944(2.0, frames=32)
    _check_qc(b.code, 12, 81)
    _assert_codewords(b.code, b.codewords)
    assert b.max_iter == 10 and not b.early_stop


def test_qc_mix_structure():
    mix = configs.qc_mix(total=240)
    assert len(mix) == 12
    seen = set()
    for idx, m in enumerate(mix):
        Z = configs.QC_MIX_Z[idx // 4]
        mb = configs.QC_MIX_MB[idx % 4]
        seen.add((Z, mb))
        _check_qc(m.code, mb, Z)
        _assert_codewords(m.code, m.codewords)
        assert m.rate == configs.RATE_OF_MB[mb]
    assert len(seen) == 12
    counts = configs.qc_mix_counts()
    assert counts.sum() == 16384 and len(set(counts.tolist())) >= 10, "uneven per-code counts"


def test_stair64800_structure():
    """n = 64800, rate 1/2: info columns of degree 8 (n/5) and 3 (3n/10), a
    dual-diagonal parity part (degree 2, the last column degree 1), check
    degrees {6: 1, 7: m - 1}, no 4-cycles; staircase-encoded codewords
    satisfy H."""
    b = configs.stair64800(frames=8)
    code = b.code
    n, m = 64800, 32400
    assert (code.m, code.n) == (m, n)
    cd = code.col_degrees()
    vals, cnt = np.unique(cd, return_counts=True)
    assert dict(zip(vals.tolist(), cnt.tolist())) == {1: 1, 2: m - 1, 3: 3 * n // 10, 8: n // 5}
    rd = code.row_degrees()
    vals, cnt = np.unique(rd, return_counts=True)
    assert dict(zip(vals.tolist(), cnt.tolist())) == {6: 1, 7: m - 1}
    assert code.edges == 226799
    assert codes.count_4cycles(code) == 0
    _assert_codewords(code, b.codewords)


def test_generators_deterministic():
    a = codes.qc_code(6, 24, 27, seed=305)
    b = codes.qc_code(6, 24, 27, seed=305)
    c = codes.qc_code(6, 24, 27, seed=306)
    assert np.array_equal(a.col_idx, b.col_idx) and np.array_equal(a.row_ptr, b.row_ptr)
    assert not np.array_equal(np.asarray(a.qc["shifts"]), np.asarray(c.qc["shifts"]))
    g1 = codes.gallager_regular(504, 3, 6, 101)
    g2 = codes.gallager_regular(504, 3, 6, 101)
    assert np.array_equal(g1.col_idx, g2.col_idx)
    x = configs.qc1944(1.5, frames=16).llr
    y = configs.qc1944(1.5, frames=16).llr
    assert np.array_equal(x, y)


def test_serve_schedule_shape():
    sched = configs.serve_schedule(0.5)
    gaps = np.diff([r.t_arrival for r in sched])
    assert abs(len(sched) / 0.5 - 20000) < 600, "Poisson arrivals at 20k requests/s"
    assert 0.8 < gaps.mean() * 20000 < 1.2 and gaps.std() / gaps.mean() == pytest.approx(1.0, abs=0.1)
    assert min(r.frames for r in sched) == 1 and max(r.frames for r in sched) == 64
    assert {r.code_id for r in sched} == set(range(12))
    assert all(1.0 <= r.ebn0_db <= 3.0 for r in sched)
