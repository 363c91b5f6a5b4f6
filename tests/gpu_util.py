"""Shared helpers for the GPU parity tests: the same seeded inputs go to the
HIP library (through the C ABI) and to the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

from paper_2405_00698_amd import inputs

DEV = "cuda:0"


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this container")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def voxel_population(sides, seed, p_empty=0.2):
    cls, w = inputs.population_voxels(sides, seed, p_empty)
    return cls, w


def split(arr, offsets):
    return [arr[offsets[r]:offsets[r + 1]] for r in range(len(offsets) - 1)]


def gpu_population(sides, cls, w, **params):
    from paper_2405_00698_amd.api import Population
    P = Population(sides, **params)
    P.build_from_voxels(torch.from_numpy(cls).to(DEV), torch.from_numpy(w).to(DEV))
    return P


def oracle_robots(orc, sides, cls, w, **params):
    out, o = [], 0
    oparams = dict(params)
    if "flags" in oparams:
        oparams["flags"] = int(oparams["flags"])
    for n in sides:
        nv = n ** 3
        out.append(orc.Robot(n, cls[o:o + nv], w[o:o + nv].astype(np.float64), **oparams))
        o += nv
    return out


def rel_err(xg, xo):
    """max_i ||x_gpu,i - x_oracle,i||_inf / max_i ||x_oracle,i||_inf"""
    return float(np.abs(xg - xo).max() / max(np.abs(xo).max(), 1e-30))


def gpu_states(P):
    x, v, st = P.state()
    M, S, mo, so = P.counts()
    xs = split(x.cpu().numpy().astype(np.float64), mo)
    vs = split(v.cpu().numpy().astype(np.float64), mo)
    return xs, vs, st
