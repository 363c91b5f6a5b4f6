"""Resource check of the built gfx950 code objects.

Reads the AMDGPU metadata note of every kernel in libsoftrobot.so (the
offload bundles in its .hip_fatbin section) and checks what a workgroup needs
against one gfx950 compute unit: LDS (group segment) within 160 KiB, vector
registers (architected + accumulation, one unified file of 512 per SIMD lane)
within the share each wave gets when the largest workgroup the kernel admits
is resident, a bounded private segment, no dynamic stack, wave64.  The build
runs it on every link, so a configuration that a CU cannot hold never reaches
a kernel launch or a runtime attribute query.
"""
import os
import struct
import subprocess

import yaml

READELF = os.environ.get("LLVM_READELF", "/opt/rocm/llvm/bin/llvm-readelf")
TARGET = "gfx950"

LDS_PER_CU = 160 * 1024       # bytes of LDS one workgroup may use
VGPRS_PER_SIMD_LANE = 512     # unified VGPR + AGPR file, per lane, wave64
SIMDS_PER_CU = 4
MAX_PRIVATE = 16 * 1024       # bound this library sets on per-lane scratch
MAX_WORKGROUP = 1024
_BUNDLE_MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"


def _section(path, name):
    out = subprocess.run([READELF, "-S", "-W", path], capture_output=True, text=True, check=True).stdout
    for line in out.splitlines():
        if "]" in line and name in line.split("]")[1].split()[:1]:
            f = line.split("]")[1].split()
            off, size = int(f[3], 16), int(f[4], 16)
            with open(path, "rb") as fh:
                fh.seek(off)
                return fh.read(size)
    raise RuntimeError("%s has no %s section" % (path, name))


def code_objects(lib_path):
    """The gfx950 code objects (ELF bytes) bundled in lib_path."""
    data = _section(lib_path, ".hip_fatbin")
    cos, pos = [], 0
    while True:
        i = data.find(_BUNDLE_MAGIC, pos)
        if i < 0:
            return cos
        (n,) = struct.unpack_from("<Q", data, i + len(_BUNDLE_MAGIC))
        p = i + len(_BUNDLE_MAGIC) + 8
        for _ in range(n):
            off, size, tlen = struct.unpack_from("<QQQ", data, p)
            p += 24
            triple = data[p:p + tlen].decode()
            p += tlen
            if triple.endswith(TARGET) and size > 0:
                cos.append(data[i + off:i + off + size])
        pos = i + 1


def kernels(lib_path, workdir):
    """Metadata dicts of every kernel in the library (one per kernel symbol)."""
    out = []
    for k, co in enumerate(code_objects(lib_path)):
        path = os.path.join(workdir, "co%d.elf" % k)
        with open(path, "wb") as fh:
            fh.write(co)
        notes = subprocess.run([READELF, "--notes", path], capture_output=True, text=True, check=True).stdout
        doc = notes[notes.index("---"):notes.rindex("...")]
        out.extend(yaml.safe_load(doc)["amdhsa.kernels"])
    return out


def vgpr_budget(workgroup):
    """VGPRs (with AGPRs) a wave may hold when a workgroup of this size is resident."""
    waves = (workgroup + 63) // 64
    per_simd = (waves + SIMDS_PER_CU - 1) // SIMDS_PER_CU
    return VGPRS_PER_SIMD_LANE // per_simd


def violations(ks):
    bad = []
    for k in ks:
        name, wg = k[".name"], k[".max_flat_workgroup_size"]
        if k[".wavefront_size"] != 64:
            bad.append("%s: wave%d" % (name, k[".wavefront_size"]))
        if wg > MAX_WORKGROUP:
            bad.append("%s: workgroup %d" % (name, wg))
        if k[".group_segment_fixed_size"] > LDS_PER_CU:
            bad.append("%s: LDS %d B > %d" % (name, k[".group_segment_fixed_size"], LDS_PER_CU))
        if k[".vgpr_count"] > vgpr_budget(wg):
            bad.append("%s: %d VGPRs > %d at workgroup %d" % (name, k[".vgpr_count"], vgpr_budget(wg), wg))
        if k[".private_segment_fixed_size"] > MAX_PRIVATE:
            bad.append("%s: private segment %d B" % (name, k[".private_segment_fixed_size"]))
        if k.get(".uses_dynamic_stack"):
            bad.append("%s: dynamic stack" % name)
    return bad


def check(lib_path, workdir):
    ks = kernels(lib_path, workdir)
    bad = violations(ks)
    if bad:
        raise RuntimeError("kernels outside the gfx950 per-CU limits:\n  " + "\n  ".join(bad))
    return ks
