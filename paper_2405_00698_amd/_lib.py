"""ctypes loader for libsoftrobot.so (the HIP library).  No fallback: when the
library is missing or fails to load, every call raises."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsoftrobot.so")

SR_OK, SR_EINVAL, SR_ENOMEM, SR_EHIP, SR_ESTATE, SR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SR_NO_GRAVITY, SR_NO_GROUND, SR_NO_ACTUATION, SR_WEIGHT_ACTUATION = 1, 2, 4, 8
SR_NOALLOC_MAX_STEPS = 65536
SR_QUERY_FP32, SR_QUERY_BF16 = 0, 1
SR_STEP_AUTO, SR_STEP_PERSISTENT, SR_STEP_PLAIN = 0, 1, 2
GENOME_LEN = 8710


class SimParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("gravity", C.c_float), ("damping", C.c_float), ("mass", C.c_float),
                ("voxel_len", C.c_float), ("k_ground", C.c_float), ("mu", C.c_float), ("act_freq", C.c_float),
                ("k_class", C.c_float * 5), ("a_class", C.c_float * 5), ("phi_class", C.c_float * 5),
                ("flags", C.c_uint32), ("mu_static", C.c_float), ("zeta_spring", C.c_float),
                ("zeta_ground", C.c_float), ("reserved", C.c_float)]


class GAParams(C.Structure):
    _fields_ = [("elite_frac", C.c_double), ("tournament_k", C.c_int32), ("reserved", C.c_int32),
                ("p_cross_thr", C.c_uint64), ("p_mut_thr", C.c_uint64), ("mut_sigma", C.c_float),
                ("reserved2", C.c_float)]


class SoftRobotError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("softrobot error %d: %s" % (code, msg))
        self.code = code


_lib = None

# (name, argtypes) of every exported entry point
P = C.c_void_p
_SIGS = {
    "sr_last_error": ([], C.c_char_p),
    "sr_version": ([], C.c_int),
    "sr_default_params": ([C.POINTER(SimParams)], C.c_int),
    "sr_table2_params": ([C.POINTER(SimParams)], C.c_int),
    "pop_create": ([C.POINTER(SimParams), C.c_int32, C.POINTER(C.c_int32), P, C.POINTER(P)], C.c_int),
    "pop_destroy": ([P], C.c_int),
    "pop_build_from_voxels": ([P, P, P], C.c_int),
    "pop_build_from_genomes": ([P, P, P, C.c_int32], C.c_int),
    "pop_set_step_config": ([P, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    "pop_step": ([P, C.c_int32], C.c_int),
    "pop_step_noalloc": ([P, C.c_int32], C.c_int),
    "pop_fitness": ([P, P], C.c_int),
    "pop_get_counts": ([P, P, P, P, P], C.c_int),
    "pop_get_voxels": ([P, P, P], C.c_int),
    "pop_get_query": ([P, P, P], C.c_int),
    "pop_get_springs": ([P, P, P, P, P, P], C.c_int),
    "pop_set_spring_params": ([P, P, P, P], C.c_int),
    "pop_get_state": ([P, P, P, C.POINTER(C.c_int64)], C.c_int),
    "pop_set_state": ([P, P, P, C.c_int64], C.c_int),
    "pop_get_status": ([P, P], C.c_int),
    "pop_set_persist_variant": ([P, C.c_int32, C.c_int32, C.c_int32], C.c_int),
    "pop_reset": ([P], C.c_int),
    "pop_set_graphs": ([P, C.c_int32], C.c_int),
    "sr_microbench": ([C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
    "sr_persist_configs": ([C.c_int32, P, P, C.c_int32], C.c_int),
    "pop_get_persist_variant": ([P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "pop_set_schedule": ([P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "pop_get_schedule": ([P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)], C.c_int),
    "pop_record": ([P, C.c_int32, C.c_int32], C.c_int),
    "pop_backward": ([P, P, P, P, P, P, P, P], C.c_int),
    "ga_generation": ([P, P, P, C.c_int32, C.c_int32, C.POINTER(GAParams), C.c_uint64, C.c_uint64, P, P],
                      C.c_int),
}


def load(path=None):
    """The HIP library with every declared entry point typed (cached).  path:
    another build of the same library (the tests' poisoned debug build),
    loaded and returned without replacing the cached one."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    lib_path = LIB_PATH if path is None else path
    if not os.path.exists(lib_path):
        raise RuntimeError("%s is not built (run __graft_entry__.build()); "
                           "there is no fallback path" % os.path.basename(lib_path))
    L = C.CDLL(lib_path)
    missing = [name for name in _SIGS if not hasattr(L, name)]
    if missing:
        raise RuntimeError("libsoftrobot.so lacks the entry points %s declared in include/softrobot.h; "
                           "rebuild it (__graft_entry__.build())" % ", ".join(missing))
    for name, (args, res) in _SIGS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    if path is None:
        _lib = L
    return L


def check(rc):
    if rc != SR_OK:
        raise SoftRobotError(rc, load().sr_last_error().decode())
    return rc


def default_params(**overrides):
    p = SimParams()
    check(load().sr_default_params(C.byref(p)))
    return _override(p, overrides)


def table2_params(**overrides):
    """Table II material and contact model (sr_table2_params), with overrides."""
    p = SimParams()
    check(load().sr_table2_params(C.byref(p)))
    return _override(p, overrides)


def _override(p, overrides):
    for k, v in overrides.items():
        if k in ("k_class", "a_class", "phi_class"):
            setattr(p, k, (C.c_float * 5)(*v))
        else:
            setattr(p, k, v)
    return p
