"""Build libldpc.so (HIP for gfx950) in-tree.

Every source under csrc/ is compiled by hipcc to an object (in parallel; the
check-node kernels are split into one translation unit per degree bucket),
then linked into one shared library next to this file.  FP contraction is
off so that every kernel evaluates the check rule with the same rounding;
packed FP32 instructions are disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libldpc.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-ffp-contract=off", "-Wall", "-Wno-unused-result", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    assert srcs, "no sources"
    return srcs


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _stale(src, obj, headers):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(p) > t for p in [src, *headers])


def build(force: bool = True, verbose: bool = False, jobs: int = 0) -> str:
    """Compile (all objects if force, else only stale ones) and link libldpc.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    headers = glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(ROOT, "include", "ldpc.h")]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    todo, objs = [], []
    for src in sources():
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        objs.append(obj)
        if force or _stale(src, obj, headers):
            todo.append((src, obj))

    def compile_one(item):
        src, obj = item
        cmd = [_hipcc(), *HIPCC_FLAGS, *inc, "-c", src, "-o", obj + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msgs = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
        if msgs.strip() and verbose:
            print(msgs, file=sys.stderr)
        os.replace(obj + ".tmp", obj)

    workers = jobs or min(16, os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(compile_one, todo))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--incremental" not in sys.argv, verbose=True))
