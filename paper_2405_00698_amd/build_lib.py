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


# debug build: the exchange kernels poison their LDS entries with NaN at the
# start of each phase (tests compare it bit for bit with the product build)
LIB_POISON = os.path.join(HERE, "libsoftrobot_poison.so")
OBJ_POISON = os.path.join(HERE, "_build", "poison")
POISONED = ("sim.hip", "adjoint.hip")


def _compile(src, objdir=OBJ, extra=()):
    obj = os.path.join(objdir, os.path.basename(src)[:-4] + ".o")
    subprocess.check_call([HIPCC] + FLAGS + list(extra) + ["-c", src, "-o", obj])
    return obj


def _link(objs, lib, workdir):
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
    # every kernel must fit one gfx950 CU (LDS, registers, scratch) before the
    # library replaces the previous build
    from paper_2405_00698_amd import codeobj
    try:
        codeobj.check(tmp, workdir)
    except Exception:
        os.remove(tmp)
        raise
    os.replace(tmp, lib)
    return lib


def build(jobs=8):
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(OBJ_POISON, exist_ok=True)
    srcs = sources()
    poisoned = [f for f in srcs if os.path.basename(f) in POISONED]
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
        pobjs = list(ex.map(lambda f: _compile(f, OBJ_POISON, ["-DSR_POISON_LDS=1"]), poisoned))
    _link(objs, LIB, OBJ)
    by_name = {os.path.basename(o): o for o in pobjs}
    _link([by_name.get(os.path.basename(o), o) for o in objs], LIB_POISON, OBJ_POISON)
    return LIB


if __name__ == "__main__":
    print(build())
