"""C ABI contract checks that need no GPU: the library loads, exports every
function include/ldpc.h declares, and rejects bad arguments before touching
the device (no compute call is made here)."""
import ctypes

import numpy as np
import pytest

import paper_1812_06545_amd as L


def test_exports_every_header_function():
    names = L.header_functions()
    assert len(names) >= 9
    lib = L.library()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    for s in (0, -1, -2, -3, -4, -5):
        assert L.ldpc_status_str(s) not in ("", "unknown status")
    assert L.ldpc_status_str(7) == "unknown status"


def _csr_status(m, n, row_ptr, col_idx):
    out = ctypes.c_void_p()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    return L.library().ldpc_code_from_csr(m, n, rp.ctypes.data, ci.ctypes.data if ci.size else None,
                                          ctypes.byref(out)), out.value


@pytest.mark.parametrize("m,n,rp,ci,want", [
    (0, 4, [0], [], L.LDPC_EINVAL),                       # no rows
    (1, 0, [0, 0], [], L.LDPC_EINVAL),                    # no columns
    (1, 4, [1, 2], [0, 1], L.LDPC_EINVAL),                # row_ptr[0] != 0
    (2, 4, [0, 2, 1], [0, 1], L.LDPC_EINVAL),             # decreasing row_ptr
    (1, 4, [0, 2], [0, 4], L.LDPC_EINVAL),                # column out of range
    (1, 4, [0, 2], [-1, 2], L.LDPC_EINVAL),               # negative column
    (1, 4, [0, 3], [1, 2, 1], L.LDPC_EINVAL),             # duplicate edge
    (1, 100, [0, 65], list(range(65)), L.LDPC_EUNSUPPORTED),  # row degree above the limit
])
def test_code_from_csr_rejects(m, n, rp, ci, want):
    st, handle = _csr_status(m, n, rp, ci)
    assert st == want
    assert handle is None


def test_code_from_csr_null_out():
    rp = np.array([0, 1], np.int32)
    ci = np.array([0], np.int32)
    assert L.library().ldpc_code_from_csr(1, 1, rp.ctypes.data, ci.ctypes.data, None) == L.LDPC_EINVAL


@pytest.mark.parametrize("shifts,Z", [([[0, 5]], 5), ([[-2, 0]], 5), ([[0, 1]], 0)])
def test_code_from_qc_rejects(shifts, Z):
    s = np.ascontiguousarray(shifts, dtype=np.int32)
    out = ctypes.c_void_p()
    st = L.library().ldpc_code_from_qc(s.shape[0], s.shape[1], Z, s.ctypes.data, ctypes.byref(out))
    assert st == L.LDPC_EINVAL and out.value is None


def test_decode_rejects_null_code():
    lib = L.library()
    st = lib.ldpc_decode(None, 0, 4, 10, 0, None, None, None, None, None, 0, None)
    assert st == L.LDPC_EINVAL
    b = ctypes.c_size_t()
    assert lib.ldpc_workspace_bytes(None, 0, 4, 10, ctypes.byref(b)) == L.LDPC_EINVAL


def test_batch_rejects_and_empty():
    lib = L.library()
    b = ctypes.c_size_t(123)
    assert lib.ldpc_batch_workspace_bytes(None, -1, 0, ctypes.byref(b)) == L.LDPC_EINVAL
    assert lib.ldpc_batch_workspace_bytes(None, 0, 0, ctypes.byref(b)) == L.LDPC_OK and b.value == 0
    assert lib.ldpc_decode_batch(None, 0, 0, None, 0, None) == L.LDPC_OK
    assert lib.ldpc_decode_batch(None, 0, 7, None, 0, None) == L.LDPC_EINVAL  # bad dtype
    job = L.ldpc_job(None, 4, 10, 0, None, None, None, None)
    assert L.library().ldpc_decode_batch(ctypes.byref(job), 1, 0, None, 0, None) == L.LDPC_EINVAL


def test_minsum_and_mstream_argument_errors_without_device():
    """Argument errors of the min-sum entry point and the multi-stream
    baseline are reported before any device call."""
    lib = L.library()
    assert lib.ldpc_decode_minsum(None, 0, 1, 10, L.LDPC_MIN_SUM, 1.0, 0.0, None, None, None, None, None, 0,
                                  None) == L.LDPC_EINVAL
    assert lib.ldpc_mstream_run(None, 1, 64, 1, 10, 0, 1, None, None, None, None) == L.LDPC_EINVAL



def test_code_limits_of_32bit_offsets():
    """Codes whose chunk offsets would overflow the kernels' 32-bit index
    arithmetic are refused at creation (before any device call)."""
    lib = L.library()
    out = ctypes.c_void_p()
    ci = np.arange(4, dtype=np.int32)
    rp = np.array([0, 1 << 25], np.int32)  # 2^25 edges: one more than LDPC_MAX_EDGES
    assert lib.ldpc_code_from_csr(1, 10, rp.ctypes.data, ci.ctypes.data, ctypes.byref(out)) == L.LDPC_EUNSUPPORTED
    rp = np.array([0, 2], np.int32)
    assert lib.ldpc_code_from_csr(1, 1 << 22, rp.ctypes.data, ci.ctypes.data,
                                  ctypes.byref(out)) == L.LDPC_EUNSUPPORTED
    assert out.value is None


def test_noalloc_batch_argument_errors_without_device():
    lib = L.library()
    assert lib.ldpc_decode_batch_noalloc(None, 0, 0, None) == L.LDPC_OK
    assert lib.ldpc_decode_batch_noalloc(None, -1, 0, None) == L.LDPC_EINVAL
    assert lib.ldpc_decode_batch_noalloc(None, 0, 7, None) == L.LDPC_EINVAL
    job = L.ldpc_job(None, 4, 10, 0, None, None, None, None)
    assert lib.ldpc_decode_batch_noalloc(ctypes.byref(job), 1, 0, None) == L.LDPC_EINVAL


def test_tuning_file_round_trip_without_device(tmp_path):
    """The tuning table's file format: valid lines load (and count), a
    malformed line is refused; saving writes one line per entry."""
    lib = L.library()
    good = tmp_path / "tune.txt"
    good.write_text("gfx950 00000000000000ab 256 2 1.250000\ngfx950 00000000000000cd 512 1 0.500000\n")
    n = ctypes.c_int32(-1)
    assert lib.ldpc_tuning_load(str(good).encode(), ctypes.byref(n)) == L.LDPC_OK and n.value == 2
    bad = tmp_path / "bad.txt"
    bad.write_text("gfx950 00000000000000ef 100 1 1.0\n")  # 100 threads: not a multiple of 64
    assert lib.ldpc_tuning_load(str(bad).encode(), ctypes.byref(n)) == L.LDPC_EINVAL
    assert lib.ldpc_tuning_load(str(tmp_path / "missing.txt").encode(), None) == L.LDPC_EINVAL
    out = tmp_path / "saved.txt"
    assert lib.ldpc_tuning_save(str(out).encode()) == L.LDPC_OK
    saved = out.read_text().splitlines()
    assert len(saved) >= 2 and all(len(s.split()) == 5 for s in saved)
    assert {s.split()[1] for s in saved} >= {"00000000000000ab", "00000000000000cd"}
    assert lib.ldpc_batch_set_frames_per_group(3) == L.LDPC_EINVAL
    assert lib.ldpc_batch_set_frames_per_group(1) == L.LDPC_OK
