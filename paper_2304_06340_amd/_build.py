"""Build the HIP libraries for gfx950 with hipcc, in-tree.

libhsd.so            every HIP source of csrc/: the product library (the C
                     ABI of include/hsd.h and nothing else callable)
libhsd_testhooks.so  the same sources with HSD_TEST_HOOKS defined: also the
                     CPU runs of the kernels' lane bodies, the FFT and the
                     simulated serving executor that the tests call

Sources compile one per process (objects under _build/), then link; a source
without test hooks is compiled once and linked into both.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhsd.so")
TEST_LIB = os.path.join(HERE, "libhsd_testhooks.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _has_hooks(path: str) -> bool:
    with open(path) as fh:
        return "HSD_TEST_HOOKS" in fh.read()


def _run(cmd: list[str]) -> None:
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP source (always recompiles) and link both libraries."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(HERE, "..", "include")]
    tasks = []   # (source, object, extra flags)
    prod, test = [], []
    for src in sources():
        name = os.path.splitext(os.path.basename(src))[0]
        obj = os.path.join(OBJ, name + ".o")
        tasks.append((src, obj, []))
        prod.append(obj)
        if _has_hooks(src):
            tobj = os.path.join(OBJ, name + ".hooks.o")
            tasks.append((src, tobj, ["-DHSD_TEST_HOOKS"]))
            test.append(tobj)
        else:
            test.append(obj)

    def compile_one(t):
        src, obj, extra = t
        cmd = [hipcc, *HIPCC_FLAGS, *extra, *inc, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        _run(cmd)

    n = jobs or max(1, min(len(tasks), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(n) as ex:
        list(ex.map(compile_one, tasks))
    for lib, objs in ((LIB, prod), (TEST_LIB, test)):
        tmp = lib + ".tmp%d" % os.getpid()
        _run([hipcc, *HIPCC_FLAGS, "-shared", "-o", tmp, *objs, "-lpthread"])
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
