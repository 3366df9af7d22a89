"""Builds libllama_mi.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libllama_mi.so")
SOURCES = ["host.cpp", "batch.cpp", "k_raw.hip", "k_raw4.hip", "k_conv.hip", "k_pack.hip", "k_unpack.hip", "k_batch.hip", "k_zero.hip", "k_count.hip", "k_xpose.hip", "k_mixed.hip", "k_generic.hip", "k_pack_planar.hip",
           "nbody.hip"]
ARCH = os.environ.get("LLAMA_MI_ARCH", "gfx950")
# Packed FP32 instructions are disabled for every HIP translation unit.
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    raise RuntimeError("hipcc not found")


def _deps_mtime():
    """Newest modification time of the headers every translation unit may include."""
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    heads.append(os.path.join(os.path.dirname(HERE), "include", "llama_mi.h"))
    return max(os.path.getmtime(h) for h in heads)


def _compile(src, incremental=False, deps=0.0):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    if incremental and os.path.exists(obj):
        if os.path.getmtime(obj) >= max(deps, os.path.getmtime(os.path.join(CSRC, src))):
            return obj
    cmd = [_hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, err))
    return obj


def build(verbose=False, jobs=None, incremental=False):
    """Compiles every source (incremental=True: only those older than their
    source or any header) and links the library."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 16)
    deps = _deps_mtime()
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental, deps), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)
