"""Seeded synthetic inputs shared by the HIP path's tests, the benchmark and the
oracle's tests.

This module holds random draws and array layout only, none of the method's
arithmetic, so both sides can consume identical bytes without sharing code.
Every generator is a numpy Philox stream keyed by (seed, stream id).
"""
import numpy as np

GENOME_LEN = 8710
# flat genome layout: W1[64][64] b1[64] W2[64][64] b2[64] W3[6][64] b3[6]
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 4096, 4160, 8256, 8320, 8704

SEED_B, SEED_GENOME, SEED_SHAPE, SEED_GA = 0, 1, 2, 3


def rng(seed, stream=0):
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream)]))


def gaussian_B(seed=SEED_B, m=32, d=3, sigma=1.0):
    """Frequency matrix of the Gaussian positional encoding: [m, d], entries N(0, sigma^2)."""
    return (sigma * rng(seed, 11).standard_normal((m, d))).astype(np.float32)


def random_genomes(n_robots, seed=SEED_GENOME, empty_bias=None):
    """[R, 8710] float32 genomes: weights N(0, 1/fan_in) with fan_in = 64, biases 0.

    empty_bias (optional, [R]) is written into b3[0], the bias of the empty
    class logit, to move a robot's fraction of empty voxels up or down."""
    g = rng(seed, 12)
    out = np.zeros((n_robots, GENOME_LEN), np.float32)
    std = 1.0 / np.sqrt(64.0)
    out[:, OFF_W1:OFF_B1] = g.standard_normal((n_robots, OFF_B1 - OFF_W1)) * std
    out[:, OFF_W2:OFF_B2] = g.standard_normal((n_robots, OFF_B2 - OFF_W2)) * std
    out[:, OFF_W3:OFF_B3] = g.standard_normal((n_robots, OFF_B3 - OFF_W3)) * std
    if empty_bias is not None:
        out[:, OFF_B3] = np.asarray(empty_bias, np.float32)
    return out


def uniform(n, lo, hi, seed, stream=13):
    return rng(seed, stream).uniform(lo, hi, size=n)


def grid_sides(n_robots, lo, hi, seed=SEED_SHAPE):
    """Grid side per robot, uniform over the integers lo..hi."""
    return rng(seed, 14).integers(lo, hi + 1, size=n_robots).astype(np.int32)


def random_voxels(n, seed, p_empty=0.2, w_lo=0.05, w_hi=1.0, classes=(1, 2, 3, 4)):
    """Direct voxel input for one n^3 robot: class per voxel (0 = empty with
    probability p_empty, else uniform over `classes`) and a weight in [w_lo, w_hi).
    Linear voxel id = i + n (j + n k), x fastest."""
    g = rng(seed, 15)
    nv = n ** 3
    cls = np.asarray(classes, np.uint8)[g.integers(0, len(classes), size=nv)]
    cls[g.random(nv) < p_empty] = 0
    w = g.uniform(w_lo, w_hi, size=nv).astype(np.float32)
    return cls.astype(np.uint8), w


def population_voxels(sides, seed, p_empty=0.2, **kw):
    """Concatenated per-robot voxel arrays for a population (robot r uses seed + r)."""
    cls, w = [], []
    for r, n in enumerate(sides):
        c, ww = random_voxels(int(n), seed * 100003 + r, p_empty, **kw)
        cls.append(c)
        w.append(ww)
    return np.concatenate(cls), np.concatenate(w)
