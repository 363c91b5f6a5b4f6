"""CPU checks of the C ABI: the HIP library loads and exports every entry
point that include/*.h declares, and the ctypes mirrors of the parameter
structs match the C layout (no device call is made)."""
import ctypes as C
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:int|const char\s*\*)\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("pop_create", "pop_destroy", "pop_build_from_genomes", "pop_build_from_voxels", "pop_step",
                 "pop_fitness", "ga_generation", "pop_backward"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2405_00698_amd import _lib
    L = _lib.load()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_struct_layouts_match_c(tmp_path):
    from paper_2405_00698_amd import _lib
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "softrobot.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(sr_sim_params), sizeof(sr_ga_params),'
                   ' offsetof(sr_sim_params, flags), offsetof(sr_ga_params, p_mut_thr), offsetof(sr_ga_params, mut_sigma),'
                   ' offsetof(sr_sim_params, mu_static), offsetof(sr_sim_params, zeta_ground));'
                   ' return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = [int(t) for t in subprocess.check_output([str(exe)]).split()]
    assert out == [C.sizeof(_lib.SimParams), C.sizeof(_lib.GAParams), _lib.SimParams.flags.offset,
                   _lib.GAParams.p_mut_thr.offset, _lib.GAParams.mut_sigma.offset,
                   _lib.SimParams.mu_static.offset, _lib.SimParams.zeta_ground.offset]


def test_defaults_and_errors_without_device():
    from paper_2405_00698_amd import _lib
    L = _lib.load()
    p = _lib.default_params()
    assert abs(p.dt - 1e-4) < 1e-18 and p.mass == pytest.approx(0.1) and p.k_ground == 1e5
    assert list(p.k_class) == [0.0, 1e4, 1e4, 3e3, 3e4]
    # argument validation happens before any device work
    h = C.c_void_p()
    sides = (C.c_int32 * 1)(13)
    assert L.pop_create(C.byref(p), 1, sides, None, C.byref(h)) == _lib.SR_EINVAL
    assert b"grid_side" in L.sr_last_error()
    assert L.pop_step(None, 1) == _lib.SR_EINVAL


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2405_00698_amd")
    for f in glob.glob(os.path.join(pkg, "**", "*.*"), recursive=True):
        if f.endswith((".py", ".hip", ".h", ".cpp")):
            txt = open(f).read()
            assert "import oracle" not in txt and "from oracle" not in txt and "oracle.c" not in txt, f


def test_voxel_order_of_rebuilt_parameters_matches_mesh_ranges(tmp_path):
    """The kernels that rebuild spring parameters from voxels must add a
    spring's voxels in the mesh build's order.  The build takes, per axis, the
    voxel range [min(a, a2) - (step == 0), min(a, a2)] (z: [c - 1 + dz, c]) and
    loops z, y, x ascending; the helpers in internal.h are compiled on the host
    and compared with that enumeration for all 13 directions."""
    src = tmp_path / "vox.cpp"
    src.write_text('#include <cstdio>\n#include "internal.h"\nusing namespace sr;\n'
                   'int main(){for(int d=0;d<NDIR;++d){printf("%d %d %d %d",dir_dx(d),dir_dy(d),dir_dz(d),vox_cnt(d));'
                   'for(int i=0;i<vox_cnt(d);++i)printf(" %d",vox_idx(d,i));printf("\\n");}'
                   'for(int i=0;i<8;++i)printf("%d ",vox_off(i,11));printf("\\n");return 0;}\n')
    exe = tmp_path / "vox"
    subprocess.check_call(["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-I",
                           os.path.join(ROOT, "paper_2405_00698_amd", "csrc"), str(src), "-o", str(exe)])
    lines = subprocess.check_output([str(exe)]).decode().split("\n")
    for line in lines[:13]:
        dx, dy, dz, cnt, *idx = [int(t) for t in line.split()]
        a = b = c = 5
        a2, b2 = a + dx, b + dy
        want = [(vx - a, vy - b, vz - c)
                for vz in range(c - 1 + dz, c + 1)
                for vy in range(min(b, b2) - (dy == 0), min(b, b2) + 1)
                for vx in range(min(a, a2) - (dx == 0), min(a, a2) + 1)]
        got = [((i & 1) - 1, ((i >> 1) & 1) - 1, (i >> 2) - 1) for i in idx]
        assert cnt == len(want) and got == want, (dx, dy, dz, got, want)
    offs = [int(t) for t in lines[13].split()]
    assert offs == [((i & 1) - 1) + 11 * (((i >> 1) & 1) - 1) + 121 * ((i >> 2) - 1) for i in range(8)]


def test_every_kernel_fits_one_cu(tmp_path):
    """Every kernel of the built library, as the compiler emitted it (LDS it
    added itself included), fits one gfx950 CU at the largest workgroup it
    admits: group segment <= 160 KiB, VGPRs + AGPRs within each wave's share
    of the 512-register file, bounded scratch, no dynamic stack, wave64.  The
    step, recording and adjoint kernels of every grid side are among them."""
    from paper_2405_00698_amd import codeobj, _lib
    ks = codeobj.kernels(_lib.LIB_PATH, str(tmp_path))
    assert not codeobj.violations(ks)
    names = [k[".name"] for k in ks]
    for stem in ("k_persist", "k_adjoint", "k_query", "k_build_mesh", "k_ga_child"):
        assert any(stem in nm for nm in names), stem
    # adjoint kernels for every side 1..12 (template argument N = n + 1)
    for n in range(1, 13):
        assert any("k_adjointILi%dE" % (n + 1) in nm for nm in names), n


def test_resource_check_rejects_oversized_kernels():
    from paper_2405_00698_amd import codeobj
    ok = {".name": "k", ".max_flat_workgroup_size": 512, ".wavefront_size": 64, ".group_segment_fixed_size": 130000,
          ".vgpr_count": 256, ".private_segment_fixed_size": 0, ".uses_dynamic_stack": False}
    assert codeobj.violations([ok]) == []
    assert codeobj.vgpr_budget(256) == 512 and codeobj.vgpr_budget(512) == 256 and codeobj.vgpr_budget(1024) == 128
    for field, val in ((".group_segment_fixed_size", 160 * 1024 + 16), (".vgpr_count", 264),
                       (".private_segment_fixed_size", 1 << 20), (".uses_dynamic_stack", True),
                       (".wavefront_size", 32)):
        assert len(codeobj.violations([dict(ok, **{field: val})])) == 1, field
    assert any("workgroup 2048" in v for v in codeobj.violations([dict(ok, **{".max_flat_workgroup_size": 2048})]))


def test_noalloc_step_allocates_nothing():
    """pop_step_noalloc and what it calls contain no allocating HIP call and
    capture no graph (a source check: the device table is a static array)."""
    src = open(os.path.join(ROOT, "paper_2405_00698_amd", "csrc", "runtime.hip")).read()

    def body(name):
        i = src.index(name)
        i = src.index("{", i)
        depth, j = 0, i
        while True:
            depth += {"{": 1, "}": -1}.get(src[j], 0)
            if depth == 0:
                return src[i:j + 1]
            j += 1

    bad = re.compile(r"hipMalloc|hipFree|hipHostMalloc|dalloc|ensure_sc|ensure_adj|hipGraphInstantiate|"
                     r"hipStreamBeginCapture|hipMemset|new |malloc\(")
    for fn in ("int pop_step_noalloc(", "int recorded_steps(", "int enqueue_steps(", "int noalloc_table("):
        b = body(fn)
        assert not bad.search(b), (fn, bad.search(b).group(0))
    assert "static __device__ __align__(256) float2 scratch[SR_NOALLOC_MAX_STEPS]" in src
    assert "hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))" in src
