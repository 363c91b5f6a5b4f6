"""pop_step_noalloc, the allocation-free form of pop_step: the same results,
bit for bit, on two calls in a row, the second on a smaller input; sizes
beyond its static step table are rejected with an error."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, gpu_population, need_gpu, say, voxel_population
from paper_2405_00698_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _state(P):
    x, v, st = P.state()
    return x.cpu().numpy(), v.cpu().numpy(), st


def _same(A, B, label):
    xa, va, sa = _state(A)
    xb, vb, sb = _state(B)
    assert sa == sb, (label, sa, sb)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb), label
    assert torch.equal(A.fitness(), B.fitness()), label


def test_noalloc_step_matches_pop_step_on_two_calls():
    # first call: an uneven population (several size groups, persistent kernels)
    sides = [4, 7, 10, 12, 5, 10, 8, 4]
    cls, w = voxel_population(sides, 71)
    A = gpu_population(sides, cls, w)
    B = gpu_population(sides, cls, w)
    say("noalloc: uneven population", sides, "3000 steps")
    A.step(3000)
    B.step_noalloc(3000)
    _same(A, B, "first call")
    # second call, smaller input: fewer robots, fewer steps (the table keeps
    # the longer first call's entries beyond its end)
    small = [4, 6]
    cls2, w2 = voxel_population(small, 72)
    C = gpu_population(small, cls2, w2)
    D = gpu_population(small, cls2, w2)
    say("noalloc: small population", small, "250 steps")
    C.step(250)
    D.step_noalloc(250)
    _same(C, D, "second call")
    # the first populations continue, with the table rewritten in between
    A.step(100)
    B.step_noalloc(100)
    _same(A, B, "continued")


def test_noalloc_step_recording_and_per_step_form():
    sides = [4] * 8
    cls, w = voxel_population(sides, 73)
    from paper_2405_00698_amd import SR_STEP_PLAIN
    for mode in (None, SR_STEP_PLAIN):
        A = gpu_population(sides, cls, w)
        B = gpu_population(sides, cls, w)
        if mode is not None:
            A.set_step_config(mode)
            B.set_step_config(mode)
        A.record(50, 200)
        B.record(50, 200)
        A.step(200)
        B.step_noalloc(200)
        _same(A, B, "mode %s" % mode)
        dJ = torch.ones(8, device=DEV)
        ga, gb = A.backward(dJ), B.backward(dJ)
        for key in ("k", "a", "phi"):
            assert torch.equal(ga[key], gb[key]), (mode, key)


def test_noalloc_step_rejects_sizes_beyond_its_table():
    sides = [3] * 2
    cls, w = voxel_population(sides, 74, p_empty=0.0)
    P = gpu_population(sides, cls, w)
    with pytest.raises(_lib.SoftRobotError):
        P.step_noalloc(_lib.SR_NOALLOC_MAX_STEPS + 1)
    with pytest.raises(_lib.SoftRobotError):
        P.step_noalloc(-1)
    P.step_noalloc(0)
    x, v, st = P.state()
    assert st == 0 and torch.isfinite(x).all()
