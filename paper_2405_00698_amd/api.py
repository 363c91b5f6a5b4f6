"""Python binding of the C ABI (include/softrobot.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Torch tensors supply device memory and the stream."""
import ctypes as C

import torch

from . import _lib
from ._lib import SoftRobotError, check  # noqa: F401


def _ptr(t, dtype, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Population:
    """A population of voxel robots on one GPU (pop_create ... pop_destroy)."""

    def __init__(self, grid_sides, params=None, stream=None, **param_overrides):
        L = _lib.load()
        self.sides = [int(n) for n in grid_sides]
        self.R = len(self.sides)
        self.params = params if params is not None else _lib.default_params(**param_overrides)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        arr = (C.c_int32 * self.R)(*self.sides)
        h = C.c_void_p()
        check(L.pop_create(C.byref(self.params), self.R, arr, _stream_handle(self.stream), C.byref(h)))
        self.h = h
        self.n_vox = sum(n ** 3 for n in self.sides)
        self._counts = None
        # spring dashpots select the +16 persistent kernels
        self.dashpots = self.params.zeta_spring != 0.0

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _lib.load().pop_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- build
    def build_from_voxels(self, cls, w):
        check(_lib.load().pop_build_from_voxels(self.h, _ptr(cls, torch.uint8, self.n_vox, "cls"),
                                                _ptr(w, torch.float32, self.n_vox, "w")))
        self._counts = None

    def build_from_genomes(self, genomes, B, precision=_lib.SR_QUERY_FP32):
        check(_lib.load().pop_build_from_genomes(self.h, _ptr(genomes, torch.float32, self.R * _lib.GENOME_LEN,
                                                              "genomes"),
                                                 _ptr(B, torch.float32, 96, "B"), int(precision)))
        self._counts = None

    # ---------------------------------------------------------------- stepping
    def set_step_config(self, mode=_lib.SR_STEP_AUTO, block=0, steps_per_launch=0):
        check(_lib.load().pop_set_step_config(self.h, int(mode), int(block), int(steps_per_launch)))

    def set_persist_variant(self, n, block, variant):
        check(_lib.load().pop_set_persist_variant(self.h, int(n), int(block), int(variant)))

    def set_graphs(self, enable):
        check(_lib.load().pop_set_graphs(self.h, 1 if enable else 0))

    def persist_variant(self, n):
        b, v = C.c_int32(), C.c_int32()
        check(_lib.load().pop_get_persist_variant(self.h, int(n), C.byref(b), C.byref(v)))
        return b.value, v.value

    def set_schedule(self, sides, lanes):
        """pop_set_schedule: launch order of the size groups and the stream
        (lane) of each; lane 0 is the population's stream."""
        n = len(sides)
        sa, la = (C.c_int32 * n)(*[int(q) for q in sides]), (C.c_int32 * n)(*[int(q) for q in lanes])
        check(_lib.load().pop_set_schedule(self.h, n, sa, la))

    def schedule(self):
        """(sides in launch order, their lanes)."""
        n = len(set(self.sides))
        sa, la = (C.c_int32 * n)(), (C.c_int32 * n)()
        check(_lib.load().pop_get_schedule(self.h, sa, la))
        return list(sa), list(la)

    def kernel_config(self, n):
        b, v = self.persist_variant(n)
        return "k_persist<%d, %d, %d>" % (n + 1, b, v)

    def step(self, n_steps):
        check(_lib.load().pop_step(self.h, int(n_steps)))

    def step_noalloc(self, n_steps):
        """pop_step_noalloc: the same steps without any device allocation (at
        most SR_NOALLOC_MAX_STEPS per call; calls on one device share its table)."""
        check(_lib.load().pop_step_noalloc(self.h, int(n_steps)))

    def fitness(self, out=None):
        if out is None:
            out = torch.empty(self.R, dtype=torch.float32, device=self.device)
        check(_lib.load().pop_fitness(self.h, _ptr(out, torch.float32, self.R, "fitness")))
        return out

    def reset(self):
        check(_lib.load().pop_reset(self.h))

    # ---------------------------------------------------------------- adjoint
    def record(self, checkpoint_every, max_steps):
        check(_lib.load().pop_record(self.h, int(checkpoint_every), int(max_steps)))

    def backward(self, dJ_dfitness, genomes=None, B=None, springs=True):
        """Gradients of sum_r dJ_dfitness[r] fitness_r over the recorded run."""
        S = self.counts()[3][-1]
        dev = self.device
        out = {}
        if springs:
            for key in ("k", "a", "phi"):
                out[key] = torch.empty(S, dtype=torch.float32, device=dev)
        g_gen = None
        if genomes is not None:
            g_gen = torch.empty((self.R, _lib.GENOME_LEN), dtype=torch.float32, device=dev)
            out["genome"] = g_gen
        check(_lib.load().pop_backward(self.h, _ptr(dJ_dfitness, torch.float32, self.R, "dJ_dfitness"),
                                       _ptr(out.get("k"), torch.float32), _ptr(out.get("a"), torch.float32),
                                       _ptr(out.get("phi"), torch.float32),
                                       _ptr(genomes, torch.float32, self.R * _lib.GENOME_LEN, "genomes"),
                                       _ptr(B, torch.float32, 96, "B"), _ptr(g_gen, torch.float32)))
        return out

    # ---------------------------------------------------------------- introspection
    def counts(self):
        if self._counts is None:
            M = (C.c_int32 * self.R)()
            S = (C.c_int32 * self.R)()
            mo = (C.c_int64 * (self.R + 1))()
            so = (C.c_int64 * (self.R + 1))()
            check(_lib.load().pop_get_counts(self.h, M, S, mo, so))
            self._counts = (list(M), list(S), list(mo), list(so))
        return self._counts

    def voxels(self):
        kept = torch.empty(self.n_vox, dtype=torch.uint8, device=self.device)
        w = torch.empty(self.n_vox, dtype=torch.float32, device=self.device)
        check(_lib.load().pop_get_voxels(self.h, _ptr(kept, torch.uint8), _ptr(w, torch.float32)))
        return kept, w

    def query(self):
        """Per-voxel class and weight the build started from (before the component step)."""
        cls = torch.empty(self.n_vox, dtype=torch.uint8, device=self.device)
        w = torch.empty(self.n_vox, dtype=torch.float32, device=self.device)
        check(_lib.load().pop_get_query(self.h, _ptr(cls, torch.uint8), _ptr(w, torch.float32)))
        return cls, w

    def springs(self):
        S = self.counts()[3][-1]
        dev = self.device
        ij = torch.empty((S, 2), dtype=torch.int32, device=dev)
        L0, k, a, phi = (torch.empty(S, dtype=torch.float32, device=dev) for _ in range(4))
        check(_lib.load().pop_get_springs(self.h, _ptr(ij, torch.int32), _ptr(L0, torch.float32),
                                          _ptr(k, torch.float32), _ptr(a, torch.float32),
                                          _ptr(phi, torch.float32)))
        return dict(ij=ij, L0=L0, k=k, a=a, phi=phi)

    def set_spring_params(self, k=None, a=None, phi=None):
        S = self.counts()[3][-1]
        check(_lib.load().pop_set_spring_params(self.h, _ptr(k, torch.float32, S, "k"),
                                                _ptr(a, torch.float32, S, "a"),
                                                _ptr(phi, torch.float32, S, "phi")))

    def state(self):
        M = self.counts()[2][-1]
        x = torch.empty((M, 3), dtype=torch.float32, device=self.device)
        v = torch.empty((M, 3), dtype=torch.float32, device=self.device)
        st = C.c_int64()
        check(_lib.load().pop_get_state(self.h, _ptr(x, torch.float32), _ptr(v, torch.float32), C.byref(st)))
        return x, v, st.value

    def set_state(self, x, v, step):
        M = self.counts()[2][-1]
        check(_lib.load().pop_set_state(self.h, _ptr(x, torch.float32, 3 * M, "x"),
                                        _ptr(v, torch.float32, 3 * M, "v"), int(step)))

    def status(self):
        out = torch.empty(self.R, dtype=torch.uint8, device=self.device)
        check(_lib.load().pop_get_status(self.h, _ptr(out, torch.uint8)))
        return out


def persist_configs(n):
    """(block, variant) persistent-kernel configurations compiled for side n."""
    L = _lib.load()
    cnt = L.sr_persist_configs(int(n), None, None, 0)
    if cnt < 0:
        check(cnt)
    b = (C.c_int32 * max(cnt, 1))()
    v = (C.c_int32 * max(cnt, 1))()
    L.sr_persist_configs(int(n), b, v, cnt)
    return [(b[i], v[i]) for i in range(cnt)]


MICRO = {"lds_read_16B": 0, "lds_read_12B": 1, "lds_read_4B": 2, "valu_fma": 3, "valu_rsq": 4, "hbm_copy": 5}


def microbench(name, iters=None):
    """Measured rate of one roofline microbenchmark: bytes/s (LDS, HBM) or lane ops/s (VALU)."""
    if iters is None:
        iters = 8 if name == "hbm_copy" else 4096
    sec, units = C.c_double(), C.c_double()
    check(_lib.load().sr_microbench(MICRO[name], int(iters), C.byref(sec), C.byref(units)))
    return units.value / sec.value


def prob_threshold(p):
    """floor(p * 2^64) as an unsigned 64-bit threshold (p in [0, 1])."""
    import math
    if p >= 1.0:
        return 2 ** 64 - 1
    return int(math.floor(p * 2.0 ** 64))


class GAConfig:
    """GA rates: Table I (mutation 0.1, crossover 0.4, elite 0.3) with tournament
    size 4 and mutation N(0, 0.02^2)."""

    def __init__(self, elite_frac=0.3, tournament_k=4, p_cross=0.4, p_mut=0.1, sigma=0.02,
                 p_cross_thr=None, p_mut_thr=None):
        self.params = _lib.GAParams()
        self.params.elite_frac = float(elite_frac)
        self.params.tournament_k = int(tournament_k)
        self.params.p_cross_thr = prob_threshold(p_cross) if p_cross_thr is None else int(p_cross_thr)
        self.params.p_mut_thr = prob_threshold(p_mut) if p_mut_thr is None else int(p_mut_thr)
        self.params.mut_sigma = float(sigma)


def ga_generation(fitness, genomes_in, genomes_out, cfg=None, seed=3, generation=0, decisions=None, stream=None):
    """One GA generation on the device (ga_generation of the C ABI)."""
    cfg = cfg if cfg is not None else GAConfig()
    P, L = genomes_in.shape
    check(_lib.load().ga_generation(_ptr(fitness, torch.float32, P, "fitness"),
                                    _ptr(genomes_in, torch.float32, P * L, "genomes_in"),
                                    _ptr(genomes_out, torch.float32, P * L, "genomes_out"), P, L,
                                    C.byref(cfg.params), int(seed), int(generation),
                                    _ptr(decisions, torch.int32, 3 * P, "decisions"), _stream_handle(stream)))
    return genomes_out


class SpringFitness(torch.autograd.Function):
    """fitness = F(k, a, phi): per-spring stiffness, amplitude and phase (canonical
    order) of a built population, n_steps from the build state; the backward runs
    the checkpointed adjoint (pop_backward)."""

    @staticmethod
    def forward(ctx, k, a, phi, pop, n_steps, checkpoint_every):
        pop.reset()
        pop.set_spring_params(k.detach().contiguous(), a.detach().contiguous(), phi.detach().contiguous())
        pop.record(checkpoint_every, n_steps)
        pop.step(n_steps)
        ctx.pop = pop
        return pop.fitness()

    @staticmethod
    def backward(ctx, gfit):
        g = ctx.pop.backward(gfit.detach().float().contiguous())
        return g["k"], g["a"], g["phi"], None, None, None


class GenomeFitness(torch.autograd.Function):
    """fitness = F(genomes): FP32 genome query and build, n_steps of simulation;
    the backward runs the adjoint through the sigmoid weight head, the
    parallel-sum rule and the MLP."""

    @staticmethod
    def forward(ctx, genomes, B, pop, n_steps, checkpoint_every):
        g = genomes.detach().contiguous()
        Bc = B.detach().contiguous()
        pop.build_from_genomes(g, Bc, _lib.SR_QUERY_FP32)
        pop.record(checkpoint_every, n_steps)
        pop.reset()
        pop.step(n_steps)
        ctx.pop = pop
        ctx.save_for_backward(g, Bc)
        return pop.fitness()

    @staticmethod
    def backward(ctx, gfit):
        g, Bc = ctx.saved_tensors
        out = ctx.pop.backward(gfit.detach().float().contiguous(), genomes=g, B=Bc, springs=False)
        return out["genome"], None, None, None, None
