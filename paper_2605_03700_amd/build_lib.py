"""Build the HIP library libcfqmc.so for gfx950 (hipcc, in-tree).

Every source is compiled with packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops) and linked into one
shared library next to this file; the kernel microbenchmark driver kbench
(csrc/kbench.cpp) is linked against it.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libcfqmc.so")
SOURCES = ["gemm.hip", "linalg.hip", "qmc.hip", "slmc.hip", "engine.hip"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(os.path.dirname(HERE), "include")]


def _compile(src, objdir):
    obj = os.path.join(objdir, src.replace(".hip", ".o"))
    cmd = ["hipcc"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-6000:]))
    return obj


def build(verbose=True):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir), SOURCES))
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-o", OUT + ".tmp"] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(OUT + ".tmp", OUT)
    # the kernel microbenchmark driver (timing and hardware-counter runs of single kernels)
    kb = os.path.join(HERE, "kbench")
    cmd = ["hipcc"] + FLAGS + [os.path.join(CSRC, "kbench.cpp"), "-L", HERE, "-lcfqmc", "-Wl,-rpath,$ORIGIN",
                               "-o", kb + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for kbench.cpp:\n" + r.stderr[-4000:])
    os.replace(kb + ".tmp", kb)
    if verbose:
        print("built", OUT, "and", kb)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
