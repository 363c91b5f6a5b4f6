"""The debug build that poisons the kernels' LDS exchange entries with NaN at
the start of every phase (libsoftrobot_poison.so) gives the same bits as the
product build: every coefficient or adjoint vector a thread reads was written
in the same phase, including where the balanced slot plan skips directions.
A missing barrier or a read of an entry left unwritten would surface as NaN."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, need_gpu, say, voxel_population
from paper_2405_00698_amd import _lib, api, build_lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _run(lib, sides, cls, w, configs, steps, params=None, record=False):
    """States after `steps` steps for each (side, block, variant) config (and
    the adjoint's spring gradients when record), with the given library."""
    saved = _lib._lib
    _lib._lib = lib
    try:
        out = []
        for cfg in configs:
            P = api.Population(sides, params=params)
            P.build_from_voxels(torch.from_numpy(cls).to(DEV), torch.from_numpy(w).to(DEV))
            if cfg is not None:
                P.set_persist_variant(*cfg)
            if record:
                P.record(50, steps)
            P.step(steps)
            x, v, _ = P.state()
            res = [x.cpu().numpy(), v.cpu().numpy()]
            if record:
                g = P.backward(torch.ones(len(sides), device=DEV))
                res += [g[k].cpu().numpy() for k in ("k", "a", "phi")]
            out.append(res)
            P.close()
        return out
    finally:
        _lib._lib = saved


@pytest.mark.parametrize("n", [4, 7, 8, 9, 10, 11, 12])
def test_poisoned_exchange_gives_the_same_bits(n):
    poison = _lib.load(build_lib.LIB_POISON)
    prod = _lib.load()
    sides = [n] * 3
    cls, w = voxel_population(sides, 120 + n)
    configs = [(n, b, v) for b, v in api.persist_configs(n) if not v & 16]
    a = _run(prod, sides, cls, w, configs, 120)
    b = _run(poison, sides, cls, w, configs, 120)
    for cfg, ra, rb in zip(configs, a, b):
        assert np.isfinite(rb[0]).all(), cfg
        assert all(np.array_equal(p, q) for p, q in zip(ra, rb)), cfg
    say("side", n, "configurations compared", len(configs))


@pytest.mark.parametrize("n", [3, 5, 8, 10, 12])
def test_poisoned_adjoint_exchange_gives_the_same_bits(n):
    """The exchange rows of the reverse step (one chunk of directions up to 8^3,
    three at 10^3, seven at 12^3) are all written before they are read."""
    poison = _lib.load(build_lib.LIB_POISON)
    prod = _lib.load()
    sides = [n] * 3
    cls, w = voxel_population(sides, 130 + n)
    a = _run(prod, sides, cls, w, [None], 150, record=True)[0]
    b = _run(poison, sides, cls, w, [None], 150, record=True)[0]
    for p, q in zip(a, b):
        assert np.isfinite(q).all() and np.array_equal(p, q)


@pytest.mark.parametrize("n", [4, 8, 10])
def test_poisoned_dashpot_adjoint_exchange_gives_the_same_bits(n):
    """The dashpot adjoint's four exchange rows per direction (one chunk at 4^3,
    two at 8^3, five at 10^3) are all written before they are read."""
    poison = _lib.load(build_lib.LIB_POISON)
    prod = _lib.load()
    sides = [n] * 3
    cls, w = voxel_population(sides, 150 + n)
    params = _lib.table2_params()
    a = _run(prod, sides, cls, w, [None], 120, params=params, record=True)[0]
    b = _run(poison, sides, cls, w, [None], 120, params=params, record=True)[0]
    for p, q in zip(a, b):
        assert np.isfinite(q).all() and np.array_equal(p, q)


def test_poisoned_dashpot_kernels_give_the_same_bits():
    poison = _lib.load(build_lib.LIB_POISON)
    prod = _lib.load()
    sides = [5, 8, 10]
    cls, w = voxel_population(sides, 140)
    params = _lib.table2_params()
    configs = []
    for n in sorted(set(sides)):
        configs += [(n, b, v) for b, v in api.persist_configs(n) if v & 16]
    a = _run(prod, sides, cls, w, configs, 120, params=params)
    b = _run(poison, sides, cls, w, configs, 120, params=params)
    for cfg, ra, rb in zip(configs, a, b):
        assert np.isfinite(rb[0]).all() and all(np.array_equal(p, q) for p, q in zip(ra, rb)), cfg
