"""Python handle on the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product path (the HIP library
and its binding) never imports this package.

Each wrapper names the part of arXiv 2405.00698 it follows; the C source
carries the details.
"""
import ctypes as C
import math
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

GENOME_LEN = 8710
NO_GRAVITY, NO_GROUND, NO_ACTUATION, WEIGHT_ACTUATION = 1, 2, 4, 8


LIB_NATIVE = os.path.join(HERE, "liboracle_native.so")
# no -ffast-math anywhere: the oracle keeps IEEE FP64 semantics
_FLAGS = ["-std=gnu11", "-fPIC", "-shared", "-fopenmp"]


def build(force=False):
    """Compile liboracle.so with gcc (-O3 for any x86-64 host, no fast-math,
    OpenMP over robots).  The tests load this build."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3"] + _FLAGS + [SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB)
    return LIB


def build_native():
    """Compile liboracle_native.so with -O3 -march=native for the host that
    runs it (always rebuilt: the library must match this machine's CPU)."""
    tmp = LIB_NATIVE + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", "-march=native"] + _FLAGS + [SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB_NATIVE)
    return LIB_NATIVE


def use_native():
    """Load the -march=native build instead of the portable one (for the CPU
    timing leg; robots created before the switch keep the old library)."""
    global _lib, _lib_path
    build_native()
    _lib, _lib_path = None, LIB_NATIVE
    return lib()


_lib = None
_lib_path = None


class _Params(C.Structure):
    _fields_ = [("dt", C.c_double), ("gravity", C.c_double), ("damping", C.c_double),
                ("mass", C.c_double), ("voxel_len", C.c_double), ("k_ground", C.c_double),
                ("mu", C.c_double), ("act_freq", C.c_double),
                ("k_class", C.c_double * 5), ("a_class", C.c_double * 5),
                ("phi_class", C.c_double * 5), ("flags", C.c_int32),
                ("mu_static", C.c_double), ("zeta_spring", C.c_double), ("zeta_ground", C.c_double)]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _u64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def lib():
    global _lib
    if _lib is None:
        if _lib_path is None:
            build()
        L = C.CDLL(_lib_path or LIB)
        vp = C.c_void_p
        L.or_robot_create.restype = vp
        L.or_robot_create.argtypes = [C.POINTER(_Params), C.c_int, C.POINTER(C.c_uint8), C.POINTER(C.c_double)]
        L.or_robot_destroy.argtypes = [vp]
        L.or_robot_counts.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.or_robot_voxels.argtypes = [vp, C.POINTER(C.c_uint8)]
        L.or_robot_nodes.argtypes = [vp, C.POINTER(C.c_int32)]
        L.or_robot_springs.argtypes = [vp, C.POINTER(C.c_int32)] + [C.POINTER(C.c_double)] * 4
        L.or_robot_set_springs.argtypes = [vp] + [C.POINTER(C.c_double)] * 3
        L.or_robot_get_state.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        L.or_robot_set_state.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int64]
        L.or_robot_get_x0.argtypes = [vp, C.POINTER(C.c_double)]
        L.or_robot_step.argtypes = [vp, C.c_int]
        L.or_pop_step.argtypes = [C.POINTER(vp), C.c_int, C.c_int]
        L.or_robot_fitness.restype = C.c_double
        L.or_robot_fitness.argtypes = [vp]
        L.or_robot_momentum.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_robot_energy.restype = C.c_double
        L.or_robot_energy.argtypes = [vp]
        L.or_robot_backward.restype = C.c_double
        L.or_robot_backward.argtypes = [vp, C.c_int, C.c_double] + [C.POINTER(C.c_double)] * 3
        L.or_robot_backward_z.restype = C.c_double
        L.or_robot_backward_z.argtypes = [vp, C.c_int, C.c_double] + [C.POINTER(C.c_double)] * 4
        L.or_robot_backward_c.restype = C.c_double
        L.or_robot_backward_c.argtypes = [vp, C.c_int, C.c_double, C.POINTER(C.c_double)]
        L.or_robot_dashpots.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_robot_dJdw.argtypes = [vp] + [C.POINTER(C.c_double)] * 5
        L.or_mlp_backward.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int,
                                      C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_encode.argtypes = [C.POINTER(C.c_double)] * 3
        L.or_mlp.argtypes = [C.POINTER(C.c_double)] * 5
        L.or_query.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double)]
        L.or_heads.argtypes = [C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_uint8), C.POINTER(C.c_double)]
        L.or_lcc.argtypes = [C.POINTER(C.c_uint8), C.c_int, C.POINTER(C.c_uint8)]
        L.or_philox4x64_10.argtypes = [C.POINTER(C.c_uint64)] * 3
        L.or_ga_generation.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.c_int, C.c_int, C.c_double, C.c_int, C.c_uint64, C.c_uint64,
                                       C.c_double, C.c_uint64, C.c_uint64, C.POINTER(C.c_int32)]
        L.or_num_threads.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


# Default parameters: the hot-path configuration (voxel edge 0.1 m, 0.1 kg per
# node and ground stiffness 1e5 N/m as in Table II; dt, damping, friction,
# stiffness per class and the 4 Hz, +-0.2 muscle law from the workload spec).
DEFAULTS = dict(dt=1e-4, gravity=9.81, damping=0.999, mass=0.1, voxel_len=0.1,
                k_ground=1e5, mu=0.5, act_freq=4.0,
                k_class=(0.0, 1e4, 1e4, 3e3, 3e4), a_class=(0.0, 0.2, -0.2, 0.0, 0.0),
                phi_class=(0.0,) * 5, flags=0, mu_static=0.0, zeta_spring=0.0, zeta_ground=0.0)

# Table II as printed: stiffness 2e3 (muscle), 1e3 (soft tissue), 1e4 (bone),
# dt 1e-5 s, muscle amplitude up to 0.25 and phase up to pi scaled by the
# sigmoid weight, damping ratio 0.1 for the spring dashpots and the ground,
# ground stiffness 1e5, static 0.6 / kinetic 1.0 friction.  No per-step velocity
# damping (the dashpots dissipate); 4 Hz muscles as in the base model.
TABLE2 = dict(dt=1e-5, gravity=9.81, damping=1.0, mass=0.1, voxel_len=0.1,
              k_ground=1e5, mu=1.0, act_freq=4.0,
              k_class=(0.0, 2e3, 2e3, 1e3, 1e4), a_class=(0.0, 0.25, -0.25, 0.0, 0.0),
              phi_class=(0.0, math.pi, math.pi, 0.0, 0.0), flags=WEIGHT_ACTUATION,
              mu_static=0.6, zeta_spring=0.1, zeta_ground=0.1)


def make_params(**kw):
    d = dict(DEFAULTS)
    d.update(kw)
    p = _Params()
    for k in ("dt", "gravity", "damping", "mass", "voxel_len", "k_ground", "mu", "act_freq",
              "mu_static", "zeta_spring", "zeta_ground"):
        setattr(p, k, float(d[k]))
    p.k_class = (C.c_double * 5)(*d["k_class"])
    p.a_class = (C.c_double * 5)(*d["a_class"])
    p.phi_class = (C.c_double * 5)(*d["phi_class"])
    p.flags = int(d["flags"])
    return p


class Robot:
    """One voxel robot in the oracle (Sec. II-A; build, step, fitness, adjoint)."""

    def __init__(self, n, cls, w, **params):
        self.n = int(n)
        self.params = dict(DEFAULTS, **params)
        cls = np.ascontiguousarray(cls, dtype=np.uint8).reshape(-1)
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
        assert cls.size == n ** 3 and w.size == n ** 3
        self._p = make_params(**params)
        self.h = lib().or_robot_create(C.byref(self._p), self.n, _up(cls), _dp(w))
        if not self.h:
            raise ValueError("robot has no occupied voxel")
        M, S = C.c_int32(), C.c_int32()
        lib().or_robot_counts(self.h, C.byref(M), C.byref(S))
        self.M, self.S = M.value, S.value

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.or_robot_destroy(h)
            self.h = None

    def kept(self):
        out = np.zeros(self.n ** 3, np.uint8)
        lib().or_robot_voxels(self.h, _up(out))
        return out

    def node_lattice(self):
        out = np.zeros(self.M, np.int32)
        lib().or_robot_nodes(self.h, _ip(out))
        return out

    def springs(self):
        ij = np.zeros((self.S, 2), np.int32)
        L0, k, a, phi = (np.zeros(self.S) for _ in range(4))
        lib().or_robot_springs(self.h, _ip(ij), _dp(L0), _dp(k), _dp(a), _dp(phi))
        return dict(ij=ij, L0=L0, k=k, a=a, phi=phi)

    def set_springs(self, k=None, a=None, phi=None):
        arr = [None if t is None else np.ascontiguousarray(t, dtype=np.float64) for t in (k, a, phi)]
        lib().or_robot_set_springs(self.h, *[_dp(t) if t is not None else None for t in arr])

    def state(self):
        x = np.zeros((self.M, 3))
        v = np.zeros((self.M, 3))
        st, dv = C.c_int64(), C.c_int32()
        lib().or_robot_get_state(self.h, _dp(x), _dp(v), C.byref(st), C.byref(dv))
        return x, v, st.value, bool(dv.value)

    def set_state(self, x, v, step):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        lib().or_robot_set_state(self.h, _dp(x), _dp(v), int(step))

    def x0(self):
        x = np.zeros((self.M, 3))
        lib().or_robot_get_x0(self.h, _dp(x))
        return x

    def step(self, n_steps):
        lib().or_robot_step(self.h, int(n_steps))

    def fitness(self):
        return lib().or_robot_fitness(self.h)

    def momentum(self):
        P = np.zeros(3)
        Lm = np.zeros(3)
        lib().or_robot_momentum(self.h, _dp(P), _dp(Lm))
        return P, Lm

    def energy(self):
        return lib().or_robot_energy(self.h)

    def backward(self, n_steps, g=1.0):
        """J = g * fitness after n_steps from the current state, and dJ/d(k, a, phi) per spring."""
        gk, ga, gp = (np.zeros(self.S) for _ in range(3))
        J = lib().or_robot_backward(self.h, int(n_steps), float(g), _dp(gk), _dp(ga), _dp(gp))
        return J, gk, ga, gp

    def backward_z(self, n_steps, g=1.0):
        """J, dJ/d(k, Zr, Zi) per spring, Z = k a e^{i phi} (k at fixed Z), and
        dJ/dc per spring dashpot coefficient."""
        gk, gr, gi, gc = (np.zeros(self.S) for _ in range(4))
        J = lib().or_robot_backward_z(self.h, int(n_steps), float(g), _dp(gk), _dp(gr), _dp(gi), _dp(gc))
        return J, gk, gr, gi, gc

    def backward_c(self, n_steps, g=1.0):
        """J and dJ/dc per spring dashpot coefficient (Table II model)."""
        gc = np.zeros(self.S)
        J = lib().or_robot_backward_c(self.h, int(n_steps), float(g), _dp(gc))
        return J, gc

    def dashpots(self, cd=None):
        """The springs' dashpot coefficients; with cd, sets them first."""
        if cd is not None:
            cin = np.ascontiguousarray(cd, dtype=np.float64)
            lib().or_robot_dashpots(self.h, None, _dp(cin))
        out = np.zeros(self.S)
        lib().or_robot_dashpots(self.h, _dp(out), None)
        return out

    def dJdw(self, gkz, gzr, gzi, gcd=None):
        """dJ/dw per voxel from dJ/d(k, Zr, Zi, c) through the parallel-sum rule."""
        out = np.zeros(self.n ** 3)
        arr = [np.ascontiguousarray(t, dtype=np.float64) for t in (gkz, gzr, gzi)]
        gc = None if gcd is None else np.ascontiguousarray(gcd, dtype=np.float64)
        rc = lib().or_robot_dJdw(self.h, *[_dp(t) for t in arr], None if gc is None else _dp(gc), _dp(out))
        if rc != 0:
            raise ValueError("the genome gradient with spring dashpots needs dJ/dc")
        return out


def pop_step(robots, n_steps):
    """Step many robots, one per host thread."""
    arr = (C.c_void_p * len(robots))(*[r.h for r in robots])
    lib().or_pop_step(arr, len(robots), int(n_steps))


def num_threads():
    return lib().or_num_threads()


def set_threads(n):
    """Threads of the OpenMP loop over robots in pop_step."""
    lib().or_set_threads(int(n))


def encode(B, v):
    B = np.ascontiguousarray(B, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    g = np.zeros(64)
    lib().or_encode(_dp(B), _dp(v), _dp(g))
    return g


def mlp(genome, g):
    genome = np.ascontiguousarray(genome, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    h1, h2, o = np.zeros(64), np.zeros(64), np.zeros(6)
    lib().or_mlp(_dp(genome), _dp(g), _dp(h1), _dp(h2), _dp(o))
    return h1, h2, o


def query(genome, B, n):
    """Logits [n^3, 6] of one genome over an n^3 grid (Eq. (1) + MLP)."""
    genome = np.ascontiguousarray(genome, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    out = np.zeros((n ** 3, 6))
    lib().or_query(_dp(genome), _dp(B), int(n), _dp(out))
    return out


def heads(logits):
    logits = np.ascontiguousarray(logits, dtype=np.float64)
    nv = logits.shape[0]
    cls = np.zeros(nv, np.uint8)
    w = np.zeros(nv)
    lib().or_heads(_dp(logits), nv, _up(cls), _dp(w))
    return cls, w


def lcc(cls, n):
    cls = np.ascontiguousarray(cls, dtype=np.uint8).reshape(-1)
    kept = np.zeros(n ** 3, np.uint8)
    lib().or_lcc(_up(cls), int(n), _up(kept))
    return kept


def mlp_backward(genome, B, n, dJdw):
    genome = np.ascontiguousarray(genome, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    dJdw = np.ascontiguousarray(dJdw, dtype=np.float64)
    out = np.zeros(GENOME_LEN)
    lib().or_mlp_backward(_dp(genome), _dp(B), int(n), _dp(dJdw), _dp(out))
    return out


def philox(ctr, key):
    c = np.array(ctr, dtype=np.uint64)
    k = np.array(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64_10(_u64p(c), _u64p(k), _u64p(out))
    return out


def prob_threshold(p):
    """floor(p * 2^64) as an unsigned 64-bit threshold (p in [0, 1])."""
    if p >= 1.0:
        return 2 ** 64 - 1
    return int(math.floor(p * 2.0 ** 64))


def ga_generation(fitness, genomes, elite_frac=0.3, k=4, p_cross=0.4, p_mut=0.1, sigma=0.02,
                  seed=3, generation=0, p_cross_thr=None, p_mut_thr=None):
    """One GA generation (Sec. II-C, Table I).  Returns (children, decisions[P,3])."""
    fit = np.ascontiguousarray(fitness, dtype=np.float64)
    gin = np.ascontiguousarray(genomes, dtype=np.float64)
    P, L = gin.shape
    gout = np.zeros_like(gin)
    dec = np.zeros((P, 3), np.int32)
    ct = prob_threshold(p_cross) if p_cross_thr is None else p_cross_thr
    mt = prob_threshold(p_mut) if p_mut_thr is None else p_mut_thr
    rc = lib().or_ga_generation(_dp(fit), _dp(gin), _dp(gout), P, L, float(elite_frac), int(k),
                                ct, mt, float(sigma), int(seed), int(generation), _ip(dec))
    assert rc == 0
    return gout, dec


def robot_from_genome(genome, B, n, **params):
    """Full build (Eq. (1) -> MLP -> heads -> robot)."""
    lg = query(genome, B, n)
    cls, w = heads(lg)
    return Robot(n, cls, w, **params)


def genome_fitness_grad(genome, B, n, n_steps, **params):
    """J = fitness after n_steps of the robot built from `genome`, and dJ/dgenome."""
    R = robot_from_genome(genome, B, n, **params)
    J, gk, gr, gi, gc = R.backward_z(n_steps)
    dJdw = R.dJdw(gk, gr, gi, gc)
    return J, mlp_backward(genome, B, n, dJdw)
