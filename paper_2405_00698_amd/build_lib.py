"""Compiles the HIP library (csrc/*.hip) for gfx950 into libsoftrobot.so, in-tree."""
import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsoftrobot.so")
OBJ = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         # no packed FP32 instructions anywhere in the library
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # the step kernels' slot and direction loops must unroll completely
         # (their per-slot arrays then live in registers, not scratch)
         "-mllvm", "-pragma-unroll-threshold=1000000",
         "-Wno-unused-command-line-argument"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    subprocess.check_call([HIPCC] + FLAGS + ["-c", src, "-o", obj])
    return obj


def build(jobs=8):
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, sources()))
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
    # every kernel must fit one gfx950 CU (LDS, registers, scratch) before the
    # library replaces the previous build
    from paper_2405_00698_amd import codeobj
    try:
        codeobj.check(tmp, OBJ)
    except Exception:
        os.remove(tmp)
        raise
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
