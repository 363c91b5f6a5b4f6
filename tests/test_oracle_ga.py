"""Pins for the oracle's counter-based RNG and GA generation (Sec. II-C,
Table I: elites, crossover, mutation over a population of genomes)."""
import math

import numpy as np
import pytest

M64 = 2 ** 64 - 1


def _numpy_philox(ctr, key):
    """numpy's Philox-4x64-10 emits the block of counter+1, so step back one."""
    c = [int(x) for x in ctr]
    for i in range(4):                  # 256-bit decrement
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = M64
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4)


def test_philox_published_answer(orc):
    # Random123 known-answer vector for philox4x64-10, counter 0 / key 0
    out = orc.philox([0, 0, 0, 0], [0, 0])
    assert [int(x) for x in out] == [0x16554d9eca36314c, 0xdb20fe9d672d0fdc,
                                     0xd7e772cee186176b, 0x7e68b68aec7ba23b]


@pytest.mark.parametrize("seed", range(8))
def test_philox_matches_numpy(orc, seed):
    g = np.random.default_rng(seed)
    ctr = [int(x) for x in g.integers(0, 2 ** 63, 4)]
    ctr[0] |= 1
    key = [int(x) for x in g.integers(0, 2 ** 63, 2)]
    assert np.array_equal(orc.philox(ctr, key), _numpy_philox(ctr, key))


# ---------------------------------------------------------------- brute-force GA
def _word(seed, gen, child, purpose, block, word):
    return int(_numpy_philox([gen, child, purpose, block], [seed, 0])[word])


def _key(f, i):
    f = -math.inf if math.isnan(f) else f
    return (-f, i)


def _brute_ga(fit, G, elite_frac, k, pc_thr, pm_thr, sigma, seed, gen):
    """The GA generation spelled out with numpy's Philox, one draw at a time."""
    P, L = G.shape
    E = int(math.floor(elite_frac * P))
    order = sorted(range(P), key=lambda i: _key(fit[i], i))
    out = np.zeros_like(G)
    dec = []
    for c in range(E):
        out[c] = G[order[c]]
        dec.append((order[c], order[c], 0))
    for c in range(E, P):
        par = []
        for purpose in (0, 1):
            cands = [(_word(seed, gen, c, purpose, t // 4, t % 4) >> 32) * P >> 32 for t in range(k)]
            par.append(min(cands, key=lambda i: _key(fit[i], i)))
        A, B = par
        cx = _word(seed, gen, c, 2, 0, 0) < pc_thr
        dec.append((A, B, 2 if cx else 1))
        for q in range(L):
            src = A
            if cx and (_word(seed, gen, c, 3, q // 256, (q % 256) // 64) >> (q % 64)) & 1:
                src = B
            val = G[src, q]
            if _word(seed, gen, c, 4, q // 4, q % 4) < pm_thr:
                w0 = _word(seed, gen, c, 5, q // 2, 2 * (q % 2))
                w1 = _word(seed, gen, c, 5, q // 2, 2 * (q % 2) + 1)
                u1 = ((w0 >> 11) + 1) * 2.0 ** -53
                u2 = (w1 >> 11) * 2.0 ** -53
                val = val + sigma * math.sqrt(-2 * math.log(u1)) * math.cos(2 * math.pi * u2)
            out[c, q] = val
    return out, np.array(dec)


@pytest.mark.parametrize("P,L,gen", [(5, 3, 0), (8, 4, 7), (7, 2, 123456789)])
def test_ga_brute_force(orc, P, L, gen):
    g = np.random.default_rng(P * 100 + L)
    fit = g.normal(size=P)
    fit[1] = fit[3]                     # a tie
    if P > 6:
        fit[6] = np.nan
    G = g.normal(size=(P, L))
    pc, pm = orc.prob_threshold(0.5), orc.prob_threshold(0.4)
    out, dec = orc.ga_generation(fit, G, elite_frac=0.3, k=4, p_cross_thr=pc, p_mut_thr=pm,
                                 sigma=0.02, seed=99, generation=gen)
    ref, rdec = _brute_ga(fit, G, 0.3, 4, pc, pm, 0.02, 99, gen)
    assert np.array_equal(dec, rdec)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-15)


def test_elites_and_pure_selection_are_bitwise(orc):
    P, L = 40, 16
    g = np.random.default_rng(1)
    fit = g.normal(size=P)
    G = g.normal(size=(P, L))
    out, dec = orc.ga_generation(fit, G, elite_frac=0.3, p_cross=0.0, p_mut=0.0, seed=5, generation=2)
    E = int(math.floor(0.3 * P))
    order = np.lexsort((np.arange(P), -fit))
    assert np.array_equal(dec[:E, 0], order[:E])
    assert np.array_equal(out[:E], G[order[:E]])
    assert np.all(dec[E:, 2] == 1)
    assert np.array_equal(out[E:], G[dec[E:, 0]])


def test_tournament_rank_distribution(orc):
    """P(rank-r individual wins a k-tournament with replacement) = ((P-r+1)^k - (P-r)^k) / P^k."""
    P, k, gens = 16, 4, 400
    fit = np.random.default_rng(3).permutation(P).astype(float)
    rank_of = np.empty(P, int)
    rank_of[np.argsort(-fit)] = np.arange(1, P + 1)
    counts = np.zeros(P + 1)
    for gen in range(gens):
        _, dec = orc.ga_generation(fit, np.zeros((P, 1)), elite_frac=0.0, k=k, p_cross=0, p_mut=0,
                                   seed=11, generation=gen)
        for w in np.concatenate([dec[:, 0], dec[:, 1]]):
            counts[rank_of[w]] += 1
    n = counts.sum()
    r = np.arange(1, P + 1)
    p = ((P - r + 1.0) ** k - (P - r) ** k) / P ** k
    assert p.sum() == pytest.approx(1.0)
    chi2 = np.sum((counts[1:] - n * p) ** 2 / (n * p))
    assert chi2 < 40.0                     # 15 dof: p-value ~ 5e-4 at this bound


def test_crossover_and_mutation_statistics(orc):
    P, L = 64, 2048
    G = np.zeros((P, L))
    G[:] = np.arange(P)[:, None]           # gene value = parent id
    fit = np.zeros(P)
    out, dec = orc.ga_generation(fit, G, elite_frac=0.0, p_cross=1.0, p_mut=0.0, seed=4, generation=1)
    cx = dec[:, 2] == 2
    assert cx.all()
    fromB = []
    for c in range(P):
        A, B = dec[c, 0], dec[c, 1]
        assert np.all((out[c] == A) | (out[c] == B))
        if A != B:
            fromB.append(np.mean(out[c] == B))
    assert np.mean(fromB) == pytest.approx(0.5, abs=0.01)
    # mutation: rate 0.1 and N(0, 0.02^2) steps
    out, dec = orc.ga_generation(fit, np.zeros((P, L)), elite_frac=0.0, p_cross=0.0, p_mut=0.1,
                                 sigma=0.02, seed=4, generation=2)
    moved = out != 0
    assert moved.mean() == pytest.approx(0.1, abs=0.005)
    d = out[moved]
    assert d.mean() == pytest.approx(0.0, abs=0.001)
    assert d.std() == pytest.approx(0.02, rel=0.03)
    # crossover rate
    _, dec = orc.ga_generation(np.zeros(2000), np.zeros((2000, 1)), elite_frac=0.0, p_cross=0.4,
                               p_mut=0.0, seed=8, generation=0)
    assert np.mean(dec[:, 2] == 2) == pytest.approx(0.4, abs=0.035)


def test_tournament_ties_and_nan(orc):
    P = 32
    fit = np.full(P, np.nan)
    _, dec = orc.ga_generation(fit, np.zeros((P, 1)), elite_frac=0.25, p_cross=0, p_mut=0, seed=1)
    assert np.array_equal(dec[:8, 0], np.arange(8))       # all -inf: rank by index
    # the winner of an all-tie tournament is the smallest drawn index
    for c in range(8, P):
        cands = [(int(_numpy_philox([0, c, 0, 0], [1, 0])[t]) >> 32) * P >> 32 for t in range(4)]
        assert dec[c, 0] == min(cands)
