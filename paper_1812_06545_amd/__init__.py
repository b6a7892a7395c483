"""Python binding of libldpc (flooding sum-product LDPC decoding on MI355X).

A thin ctypes layer over the C ABI declared in include/ldpc.h: the functions
``ldpc_*`` below take the same arguments as their C namesakes (device memory
as torch tensors or raw pointers, the stream as a torch stream) and only
marshal them; every step of decoding runs in the HIP kernels of libldpc.so.
PyTorch supplies device memory and streams, nothing else.

There is no CPU fallback: importing this package fails loudly when the
library has not been built (``python -m paper_1812_06545_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
import re

import torch  # loads the HIP runtime that libldpc.so then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldpc.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "ldpc.h")

LDPC_OK, LDPC_EINVAL, LDPC_ENOMEM, LDPC_EDEVICE, LDPC_EBUSY, LDPC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
LDPC_F32, LDPC_F64 = 0, 1
LDPC_EARLY_STOP = 1
LDPC_LAYERED = 2
LDPC_MIN_SUM = 4
LDPC_R_MAX = 20.0
LDPC_NOALLOC_MAX_GROUPS = 16

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1812_06545_amd.build` "
                      "(there is no fallback decoder)")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_I32 = ctypes.c_int32


class ldpc_job(ctypes.Structure):
    _fields_ = [("code", _P), ("frames", _I32), ("max_iter", _I32), ("flags", ctypes.c_uint32),
                ("llr", _P), ("bits", _P), ("iters", _P), ("posterior", _P),
                ("ms_scale", ctypes.c_float), ("ms_offset", ctypes.c_float)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("ldpc_status_str", ctypes.c_char_p, [ctypes.c_int])
_sig("ldpc_code_from_csr", ctypes.c_int, [_I32, _I32, _P, _P, ctypes.POINTER(_P)])
_sig("ldpc_code_from_qc", ctypes.c_int, [_I32, _I32, _I32, _P, ctypes.POINTER(_P)])
_sig("ldpc_code_info", ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_int64)])
_sig("ldpc_code_layers", ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)])
_sig("ldpc_code_destroy", None, [_P])
_sig("ldpc_workspace_bytes", ctypes.c_int, [_P, ctypes.c_int, _I32, _I32, ctypes.POINTER(ctypes.c_size_t)])
_sig("ldpc_decode", ctypes.c_int, [_P, ctypes.c_int, _I32, _I32, ctypes.c_uint32, _P, _P, _P, _P, _P,
                                   ctypes.c_size_t, _P])
_sig("ldpc_decode_minsum", ctypes.c_int, [_P, ctypes.c_int, _I32, _I32, ctypes.c_uint32, ctypes.c_float,
                                          ctypes.c_float, _P, _P, _P, _P, _P, ctypes.c_size_t, _P])
_sig("ldpc_batch_workspace_bytes", ctypes.c_int, [ctypes.POINTER(ldpc_job), _I32, ctypes.c_int,
                                                  ctypes.POINTER(ctypes.c_size_t)])
_sig("ldpc_decode_batch", ctypes.c_int, [ctypes.POINTER(ldpc_job), _I32, ctypes.c_int, _P, ctypes.c_size_t, _P])
_sig("ldpc_decode_batch_noalloc", ctypes.c_int, [ctypes.POINTER(ldpc_job), _I32, ctypes.c_int, _P])
class ldpc_server_cfg(ctypes.Structure):
    _fields_ = [("ncodes", _I32), ("codes", ctypes.POINTER(_P)), ("mem_budget_bytes", ctypes.c_size_t),
                ("max_inflight", _I32), ("max_group_frames", _I32), ("max_queue", _I32)]


class ldpc_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("launches", ctypes.c_int64), ("frames_completed", ctypes.c_int64),
                ("bits_completed", ctypes.c_int64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("p999_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("mean_group_frames", ctypes.c_double),
                ("max_queue_depth", ctypes.c_int64), ("worst_submit_ms", ctypes.c_double),
                ("worst_queue_ms", ctypes.c_double), ("worst_stage_ms", ctypes.c_double),
                ("worst_device_ms", ctypes.c_double), ("worst_copyout_ms", ctypes.c_double),
                ("max_step_ms", ctypes.c_double), ("max_copy_ms", ctypes.c_double),
                ("max_launch_ms", ctypes.c_double), ("max_query_ms", ctypes.c_double)]


_sig("ldpc_server_create", ctypes.c_int, [ctypes.POINTER(ldpc_server_cfg), ctypes.POINTER(_P)])
_sig("ldpc_server_submit", ctypes.c_int, [_P, _I32, _I32, _I32, ctypes.c_uint32, _P, _P, _P, _P, ctypes.c_int64,
                                          ctypes.POINTER(ctypes.c_uint64)])
_sig("ldpc_server_poll", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(_I32)])
_sig("ldpc_server_wait", ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_double])
_sig("ldpc_server_cancel", ctypes.c_int, [_P, ctypes.c_uint64])
_sig("ldpc_server_stats_get", ctypes.c_int, [_P, ctypes.POINTER(ldpc_server_stats), ctypes.c_int])
_sig("ldpc_server_destroy", None, [_P])
_sig("ldpc_plan_create", ctypes.c_int, [ctypes.POINTER(ldpc_job), _I32, ctypes.c_int, _P, ctypes.c_size_t,
                                        ctypes.POINTER(_P)])
_sig("ldpc_plan_launch", ctypes.c_int, [_P, _P])
_sig("ldpc_plan_destroy", None, [_P])
_sig("ldpc_batch_set_threads", ctypes.c_int, [_I32])
_sig("ldpc_batch_set_frames_per_group", ctypes.c_int, [_I32])
_sig("ldpc_batch_launch_config", ctypes.c_int, [ctypes.POINTER(ldpc_job), _I32, ctypes.c_int, ctypes.POINTER(_I32),
                                                ctypes.POINTER(_I32), ctypes.POINTER(_I32)])
_sig("ldpc_tuning_save", ctypes.c_int, [ctypes.c_char_p])
_sig("ldpc_tuning_clear", None, [])
_sig("ldpc_batch_job_threads", ctypes.c_int, [ctypes.POINTER(ldpc_job), _I32, ctypes.c_int, ctypes.POINTER(_I32)])
_sig("ldpc_tuning_load", ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_I32)])
_sig("ldpc_autotune_batch", ctypes.c_int, [ctypes.POINTER(ldpc_job), _I32, ctypes.c_int, _P, ctypes.c_size_t, _P,
                                           ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_double)])
_sig("ldpc_batch_fits_fused", ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)])
_sig("ldpc_profile_enable", ctypes.c_int, [ctypes.c_int])
_sig("ldpc_copy_probe", ctypes.c_int, [_P, _P, ctypes.c_size_t, _P])
_sig("ldpc_profile_collect", ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)])

KERNEL_KINDS = ("ingest", "check", "variable", "output", "fused", "other")


class LdpcError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {ldpc_status_str(status)} ({status})")


def header_functions():
    """Names of the functions include/ldpc.h declares."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ldpc_[a-z0-9_]+)\s*\(", text)))


def library():
    return _lib


def _check(st, where):
    if st != LDPC_OK:
        raise LdpcError(st, where)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _handle(code):
    """A code handle from a Code (kept alive by the caller) or a raw handle."""
    return code.handle if isinstance(code, Code) else code


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dtype_code(dt):
    if dt in (torch.float32, LDPC_F32):
        return LDPC_F32
    if dt in (torch.float64, LDPC_F64):
        return LDPC_F64
    raise ValueError(f"unsupported dtype {dt}")


# ---------------------------------------------------------------- C names --

def ldpc_status_str(status: int) -> str:
    return _lib.ldpc_status_str(int(status)).decode()


def ldpc_code_from_csr(m, n, row_ptr, col_idx) -> int:
    import numpy as np
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    out = _P()
    _check(_lib.ldpc_code_from_csr(int(m), int(n), rp.ctypes.data, ci.ctypes.data if ci.size else None,
                                   ctypes.byref(out)), "ldpc_code_from_csr")
    return out.value


def ldpc_code_from_qc(mb, nb, Z, shifts) -> int:
    import numpy as np
    s = np.ascontiguousarray(shifts, dtype=np.int32)
    out = _P()
    _check(_lib.ldpc_code_from_qc(int(mb), int(nb), int(Z), s.ctypes.data, ctypes.byref(out)), "ldpc_code_from_qc")
    return out.value


def ldpc_code_info(handle):
    m, n, e = _I32(), _I32(), ctypes.c_int64()
    _check(_lib.ldpc_code_info(_handle(handle), ctypes.byref(m), ctypes.byref(n), ctypes.byref(e)), "ldpc_code_info")
    return m.value, n.value, e.value


def ldpc_code_layers(handle):
    """(number of layers, fewest rows in a layer, most rows in a layer)."""
    nl, lo, hi = _I32(), _I32(), _I32()
    _check(_lib.ldpc_code_layers(_handle(handle), ctypes.byref(nl), ctypes.byref(lo), ctypes.byref(hi)),
           "ldpc_code_layers")
    return nl.value, lo.value, hi.value


def ldpc_code_destroy(handle):
    _lib.ldpc_code_destroy(handle)


def ldpc_workspace_bytes(handle, dtype, frames, max_iter) -> int:
    b = ctypes.c_size_t()
    _check(_lib.ldpc_workspace_bytes(_handle(handle), _dtype_code(dtype), int(frames), int(max_iter), ctypes.byref(b)),
           "ldpc_workspace_bytes")
    return b.value


def ldpc_decode(handle, dtype, frames, max_iter, flags, llr, bits, iters, posterior, workspace, workspace_bytes,
                stream=None) -> int:
    return _lib.ldpc_decode(_handle(handle), _dtype_code(dtype), int(frames), int(max_iter), int(flags), _ptr(llr),
                            _ptr(bits), _ptr(iters), _ptr(posterior), _ptr(workspace), int(workspace_bytes),
                            _stream_handle(stream))


def ldpc_decode_minsum(handle, dtype, frames, max_iter, flags, ms_scale, ms_offset, llr, bits, iters, posterior,
                       workspace, workspace_bytes, stream=None) -> int:
    return _lib.ldpc_decode_minsum(_handle(handle), _dtype_code(dtype), int(frames), int(max_iter), int(flags),
                                   float(ms_scale), float(ms_offset), _ptr(llr), _ptr(bits), _ptr(iters),
                                   _ptr(posterior), _ptr(workspace), int(workspace_bytes), _stream_handle(stream))


class ldpc_mstream_stats(ctypes.Structure):
    _fields_ = [("wall_ms", ctypes.c_double), ("frames_per_s", ctypes.c_double), ("mbps", ctypes.c_double),
                ("cpu_ms", ctypes.c_double), ("cpu_cores_busy", ctypes.c_double), ("cpu_load", ctypes.c_double),
                ("online_cores", _I32)]


_sig("ldpc_mstream_run", ctypes.c_int, [_P, _I32, _I32, _I32, _I32, ctypes.c_uint32, _I32, _P, _P, _P,
                                        ctypes.POINTER(ldpc_mstream_stats)])


def ldpc_mstream_run(handle, workers, frames_per_batch, batches, max_iter, flags, blocking_sync, llr, bits, iters):
    """The multi-stream baseline over host numpy arrays (llr float32
    [batches * frames_per_batch, n]); returns (status, stats dict)."""
    def hp(a):
        if a is None or isinstance(a, int):
            return a
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    need = int(batches) * int(frames_per_batch)
    if need > 0 and not isinstance(llr, int):
        n = ldpc_code_info(handle)[1]
        if llr.size < need * n or bits.size < need * n or iters.size < need:
            raise ValueError("host arrays smaller than batches * frames_per_batch frames")
    st = ldpc_mstream_stats()
    rc = _lib.ldpc_mstream_run(_handle(handle), int(workers), int(frames_per_batch), int(batches), int(max_iter),
                               int(flags), int(bool(blocking_sync)), hp(llr), hp(bits), hp(iters), ctypes.byref(st))
    return rc, {name: getattr(st, name) for name, _ in st._fields_}


def _jobs_array(jobs):
    arr = (ldpc_job * max(len(jobs), 1))()
    for i, j in enumerate(jobs):
        arr[i] = j
    return arr


def ldpc_batch_workspace_bytes(jobs, dtype) -> int:
    arr = _jobs_array(jobs)
    b = ctypes.c_size_t()
    _check(_lib.ldpc_batch_workspace_bytes(arr, len(jobs), _dtype_code(dtype), ctypes.byref(b)),
           "ldpc_batch_workspace_bytes")
    return b.value


def ldpc_decode_batch(jobs, dtype, workspace, workspace_bytes, stream=None) -> int:
    arr = _jobs_array(jobs)
    return _lib.ldpc_decode_batch(arr, len(jobs), _dtype_code(dtype), _ptr(workspace), int(workspace_bytes),
                                  _stream_handle(stream))


def ldpc_decode_batch_noalloc(jobs, dtype, stream=None) -> int:
    arr = _jobs_array(jobs)
    return _lib.ldpc_decode_batch_noalloc(arr, len(jobs), _dtype_code(dtype), _stream_handle(stream))


def ldpc_plan_create(jobs, dtype, workspace, workspace_bytes) -> int:
    arr = _jobs_array(jobs)
    out = _P()
    _check(_lib.ldpc_plan_create(arr, len(jobs), _dtype_code(dtype), _ptr(workspace), int(workspace_bytes),
                                 ctypes.byref(out)), "ldpc_plan_create")
    return out.value


def ldpc_plan_launch(plan, stream=None) -> int:
    return _lib.ldpc_plan_launch(plan, _stream_handle(stream))


def ldpc_plan_destroy(plan):
    _lib.ldpc_plan_destroy(plan)


def ldpc_autotune_batch(jobs, dtype, workspace, workspace_bytes, stream=None):
    """-> (best_threads, best_ms)."""
    arr = _jobs_array(jobs)
    t, ms = _I32(), ctypes.c_double()
    _check(_lib.ldpc_autotune_batch(arr, len(jobs), _dtype_code(dtype), _ptr(workspace), int(workspace_bytes),
                                    _stream_handle(stream), ctypes.byref(t), ctypes.byref(ms)), "ldpc_autotune_batch")
    return t.value, ms.value


def autotune_batch(jobs, stream=None):
    """Autotune ldpc_decode_batch for these Jobs; returns (threads, ms)."""
    cj = [j.c_struct() for j in jobs]
    dt = jobs[0].llr.dtype
    need = ldpc_batch_workspace_bytes(cj, dt)
    ws = _workspace(need, jobs[0].llr.device)
    return ldpc_autotune_batch(cj, dt, ws, ws.numel(), stream)


def ldpc_batch_set_threads(threads: int) -> int:
    return _lib.ldpc_batch_set_threads(int(threads))


def ldpc_batch_set_frames_per_group(frames: int) -> int:
    return _lib.ldpc_batch_set_frames_per_group(int(frames))


def ldpc_batch_launch_config(jobs, dtype):
    """-> {"threads", "frames_per_group", "tuned"} that ldpc_decode_batch would use for these jobs."""
    arr = _jobs_array(jobs)
    t, f, tu = _I32(), _I32(), _I32()
    _check(_lib.ldpc_batch_launch_config(arr, len(jobs), _dtype_code(dtype), ctypes.byref(t), ctypes.byref(f),
                                         ctypes.byref(tu)), "ldpc_batch_launch_config")
    return {"threads": t.value, "frames_per_group": f.value, "tuned": bool(tu.value)}


def ldpc_batch_job_threads(jobs, dtype):
    """-> list of the fused workgroup size of each job (0: no frames, or the plain path)."""
    arr = _jobs_array(jobs)
    out = (_I32 * max(len(jobs), 1))()
    _check(_lib.ldpc_batch_job_threads(arr, len(jobs), _dtype_code(dtype), out), "ldpc_batch_job_threads")
    return [out[i] for i in range(len(jobs))]


def ldpc_tuning_clear():
    _lib.ldpc_tuning_clear()


def ldpc_tuning_save(path) -> int:
    return _lib.ldpc_tuning_save(os.fsencode(path))


def ldpc_tuning_load(path):
    """-> (status, entries read)."""
    n = _I32()
    st = _lib.ldpc_tuning_load(os.fsencode(path), ctypes.byref(n))
    return st, n.value


def ldpc_batch_fits_fused(handle, dtype):
    """(fits, lds_bytes) for the fused frame-resident kernel."""
    b = ctypes.c_size_t()
    st = _lib.ldpc_batch_fits_fused(_handle(handle), _dtype_code(dtype), ctypes.byref(b))
    if st not in (LDPC_OK, LDPC_EUNSUPPORTED):
        raise LdpcError(st, "ldpc_batch_fits_fused")
    return st == LDPC_OK, b.value


def ldpc_copy_probe(dst, src, nbytes, stream=None) -> int:
    return _lib.ldpc_copy_probe(_ptr(dst), _ptr(src), int(nbytes), _stream_handle(stream))


def ldpc_profile_enable(enable: bool) -> int:
    return _lib.ldpc_profile_enable(int(bool(enable)))


def ldpc_profile_collect():
    """{kind: (total_ms, launches)} since the last collect (waits for the events)."""
    ms = (ctypes.c_double * len(KERNEL_KINDS))()
    cnt = (ctypes.c_int64 * len(KERNEL_KINDS))()
    _check(_lib.ldpc_profile_collect(ms, cnt), "ldpc_profile_collect")
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS)}


# ------------------------------------------------------------ conveniences --

class Code:
    """Owns an ldpc_code handle on the current device."""

    def __init__(self, handle: int):
        self.handle = handle
        self.m, self.n, self.edges = ldpc_code_info(handle)

    @classmethod
    def from_csr(cls, m, n, row_ptr, col_idx):
        return cls(ldpc_code_from_csr(m, n, row_ptr, col_idx))

    @classmethod
    def from_qc(cls, mb, nb, Z, shifts):
        return cls(ldpc_code_from_qc(mb, nb, Z, shifts))

    @classmethod
    def from_workload(cls, code):
        """From a workloads.codes.Code (QC layout when it carries one)."""
        if code.qc is not None:
            q = code.qc
            return cls.from_qc(q["mb"], q["nb"], q["Z"], q["shifts"])
        return cls.from_csr(code.m, code.n, code.row_ptr, code.col_idx)

    def close(self):
        if self.handle:
            ldpc_code_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _workspace(nbytes, device):
    # 256-byte alignment is required; torch's allocator gives at least 512.
    ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def _flags(early_stop: bool, layered: bool, rule: str = "spa") -> int:
    if rule not in ("spa", "minsum"):
        raise ValueError(f"unknown check rule {rule!r}")
    return ((LDPC_EARLY_STOP if early_stop else 0) | (LDPC_LAYERED if layered else 0)
            | (LDPC_MIN_SUM if rule == "minsum" else 0))


def decode(code: Code, llr: torch.Tensor, max_iter: int, early_stop: bool = False, want_posterior: bool = True,
           stream=None, workspace: torch.Tensor = None, layered: bool = False, rule: str = "spa",
           ms_scale: float = 1.0, ms_offset: float = 0.0):
    """Decode llr [frames, n] (float32 or float64, on the GPU), flooding or
    (layered=True) layered schedule, sum-product or (rule="minsum") min-sum
    check rule with magnitude max(ms_scale * min - ms_offset, 0).  Returns
    (bits uint8 [frames, n], iters int32 [frames], posterior or None)."""
    assert llr.is_cuda and llr.dim() == 2 and llr.shape[1] == code.n and llr.is_contiguous()
    frames = llr.shape[0]
    dev = llr.device
    bits = torch.empty((frames, code.n), dtype=torch.uint8, device=dev)
    iters = torch.empty(frames, dtype=torch.int32, device=dev)
    post = torch.empty_like(llr) if want_posterior else None
    need = ldpc_workspace_bytes(code.handle, llr.dtype, frames, max_iter)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, dev)
    flags = _flags(early_stop, layered, rule)
    _check(ldpc_decode_minsum(code.handle, llr.dtype, frames, max_iter, flags, ms_scale, ms_offset, llr, bits, iters,
                              post, workspace, workspace.numel(), stream), "ldpc_decode_minsum")
    return bits, iters, post


class Job:
    """One job of a batch, holding its output tensors."""

    def __init__(self, code: Code, llr: torch.Tensor, max_iter: int, early_stop: bool = False,
                 want_posterior: bool = True, layered: bool = False, rule: str = "spa", ms_scale: float = 1.0,
                 ms_offset: float = 0.0):
        assert llr.is_cuda and llr.dim() == 2 and llr.shape[1] == code.n and llr.is_contiguous()
        self.code, self.llr, self.max_iter, self.early_stop = code, llr, max_iter, early_stop
        self.layered, self.rule, self.ms_scale, self.ms_offset = layered, rule, ms_scale, ms_offset
        dev = llr.device
        self.bits = torch.empty((llr.shape[0], code.n), dtype=torch.uint8, device=dev)
        self.iters = torch.empty(llr.shape[0], dtype=torch.int32, device=dev)
        self.posterior = torch.empty_like(llr) if want_posterior else None

    def c_struct(self) -> ldpc_job:
        return ldpc_job(self.code.handle, self.llr.shape[0], self.max_iter,
                        _flags(self.early_stop, self.layered, self.rule), _ptr(self.llr), _ptr(self.bits),
                        _ptr(self.iters), _ptr(self.posterior), float(self.ms_scale), float(self.ms_offset))


class Plan:
    """A captured ldpc_decode_batch over fixed Job buffers (replay with launch())."""

    def __init__(self, jobs):
        self.jobs = jobs
        dt = jobs[0].llr.dtype
        cj = [j.c_struct() for j in jobs]
        need = ldpc_batch_workspace_bytes(cj, dt)
        self.workspace = _workspace(need, jobs[0].llr.device)
        self.handle = ldpc_plan_create(cj, dt, self.workspace, self.workspace.numel())

    def launch(self, stream=None):
        _check(ldpc_plan_launch(self.handle, stream), "ldpc_plan_launch")

    def close(self):
        if self.handle:
            ldpc_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decode_batch(jobs, stream=None, workspace: torch.Tensor = None):
    """Decode a list of Job in one ldpc_decode_batch call (outputs land in the Jobs)."""
    assert jobs
    dt = jobs[0].llr.dtype
    cj = [j.c_struct() for j in jobs]
    need = ldpc_batch_workspace_bytes(cj, dt)
    if workspace is None or workspace.numel() < need:
        workspace = _workspace(need, jobs[0].llr.device)
    _check(ldpc_decode_batch(cj, dt, workspace, workspace.numel(), stream), "ldpc_decode_batch")
    return jobs


# ------------------------------------------------------------------ serving --

def ldpc_server_create(codes, mem_budget_bytes, max_inflight=3, max_group_frames=1024, max_queue=1 << 20):
    arr = (_P * len(codes))(*[_handle(c) for c in codes])
    cfg = ldpc_server_cfg(len(codes), arr, int(mem_budget_bytes), int(max_inflight), int(max_group_frames),
                          int(max_queue))
    out = _P()
    _check(_lib.ldpc_server_create(ctypes.byref(cfg), ctypes.byref(out)), "ldpc_server_create")
    return out.value


def ldpc_server_submit(server, code_id, frames, max_iter, flags, llr, bits, iters, posterior=None, arrival_ns=0):
    """Host pointers (ints) or contiguous numpy arrays.  Returns (status, ticket)."""
    def hp(a):
        if a is None or isinstance(a, int):
            return a
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    t = ctypes.c_uint64()
    st = _lib.ldpc_server_submit(server, int(code_id), int(frames), int(max_iter), int(flags), hp(llr), hp(bits),
                                 hp(iters), hp(posterior), int(arrival_ns), ctypes.byref(t))
    return st, t.value


def ldpc_server_poll(server, ticket):
    d = _I32()
    _check(_lib.ldpc_server_poll(server, ctypes.c_uint64(ticket), ctypes.byref(d)), "ldpc_server_poll")
    return bool(d.value)


def ldpc_server_wait(server, ticket, timeout_ms=60000.0) -> int:
    return _lib.ldpc_server_wait(server, ctypes.c_uint64(ticket), float(timeout_ms))


def ldpc_server_cancel(server, ticket) -> int:
    return _lib.ldpc_server_cancel(server, ctypes.c_uint64(ticket))


def ldpc_server_stats_get(server, reset=False):
    s = ldpc_server_stats()
    _check(_lib.ldpc_server_stats_get(server, ctypes.byref(s), int(bool(reset))), "ldpc_server_stats_get")
    return {name: getattr(s, name) for name, _ in s._fields_}


def ldpc_server_destroy(server):
    _lib.ldpc_server_destroy(server)
