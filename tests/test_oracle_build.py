"""Pins for the oracle's build step: Eq. (1), the MLP and its two heads
(Sec. II-B, II-C), the largest-component morphology and the spring mesh
(Sec. II-A).  Each check is a special case, closed form, library routine or
brute-force count that does not re-run the oracle's own formula."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

from paper_2405_00698_amd import inputs


# ---------------------------------------------------------------- Eq. (1)
def test_encoding_zero_B(orc):
    g = orc.encode(np.zeros((32, 3)), np.array([0.3, 0.7, 0.1]))
    assert np.array_equal(g[:32], np.ones(32)) and np.array_equal(g[32:], np.zeros(32))


def test_encoding_integer_half_quarter_phases(orc):
    # B v = integer -> cos 1, sin 0; half-integer -> cos -1; quarter -> sin 1
    B = np.zeros((32, 3))
    B[0] = (2.0, 0.0, 0.0)      # v = (0.5, ...) -> Bv = 1
    B[1] = (0.0, 1.0, 0.0)      # v_y = 0.5 -> Bv = 0.5
    B[2] = (0.0, 0.0, 1.0)      # v_z = 0.25 -> Bv = 0.25
    B[3] = (1.0, 1.0, 0.0)      # 0.5 + 0.5 = 1
    g = orc.encode(B, np.array([0.5, 0.5, 0.25]))
    np.testing.assert_allclose(g[[0, 1, 2, 3]], [1.0, -1.0, 0.0, 1.0], atol=1e-15)
    np.testing.assert_allclose(g[[32, 33, 34, 35]], [0.0, 0.0, 1.0, 0.0], atol=1e-15)


def test_encoding_unit_norm_pairs(orc):
    B = inputs.gaussian_B().astype(np.float64)
    g = orc.encode(B, np.array([0.1, 0.45, 0.9]))
    np.testing.assert_allclose(g[:32] ** 2 + g[32:] ** 2, 1.0, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- MLP and heads
def _sparse_genome():
    """A genome whose network is a hand-traceable chain:
    h1[3] = tanh(gamma[5]);  h2[7] = tanh(2 h1[3]);  o2 = 0.1 - 1.5 h2[7];  o5 = 0.7 + 0.5 h2[7]."""
    G = np.zeros(inputs.GENOME_LEN)
    G[inputs.OFF_W1 + 3 * 64 + 5] = 1.0
    G[inputs.OFF_W2 + 7 * 64 + 3] = 2.0
    G[inputs.OFF_W3 + 2 * 64 + 7] = -1.5
    G[inputs.OFF_B3 + 2] = 0.1
    G[inputs.OFF_W3 + 5 * 64 + 7] = 0.5
    G[inputs.OFF_B3 + 5] = 0.7
    return G


def test_mlp_chain_layout(orc):
    G = _sparse_genome()
    g = np.linspace(-1.0, 1.0, 64)
    h1, h2, o = orc.mlp(G, g)
    e1 = math.tanh(g[5])
    e2 = math.tanh(2.0 * e1)
    assert h1[3] == pytest.approx(e1, abs=1e-15)
    assert np.count_nonzero(h1) == 1 and np.count_nonzero(h2) == 1
    assert h2[7] == pytest.approx(e2, abs=1e-15)
    np.testing.assert_allclose(o, [0, 0, 0.1 - 1.5 * e2, 0, 0, 0.7 + 0.5 * e2], atol=1e-15)


def test_mlp_zero_weights_gives_bias(orc):
    G = np.zeros(inputs.GENOME_LEN)
    G[inputs.OFF_B3:inputs.OFF_B3 + 6] = [0.2, -1.0, 0.9, 0.3, 0.9, math.log(3.0)]
    lg = orc.query(G, inputs.gaussian_B(), 3)
    assert np.array_equal(lg, np.tile(G[inputs.OFF_B3:], (27, 1)))
    cls, w = orc.heads(lg)
    assert np.all(cls == 2)                 # tie between classes 2 and 4 -> lowest id
    np.testing.assert_allclose(w, 0.75, atol=1e-15)  # sigmoid(log 3) = 3/4


def test_heads_argmax_and_sigmoid(orc):
    lg = np.array([[5.0, 1, 2, 3, 4, 0.0],
                   [0.0, 1, 7, 3, 4, -50.0],
                   [1.0, 1, 1, 1, 1, 50.0]])
    cls, w = orc.heads(lg)
    assert cls.tolist() == [0, 2, 0]
    np.testing.assert_allclose(w, [0.5, 1.0 / (1.0 + math.exp(50.0)), 1.0 / (1.0 + math.exp(-50.0))], rtol=1e-15)


def test_query_voxel_centres(orc):
    # B row 0 = (1,0,0): cos(2 pi (i+1/2)/n) at voxel (i, j, k) with the x index fastest
    n = 4
    B = np.zeros((32, 3))
    B[0] = (1.0, 0.0, 0.0)
    B[1] = (0.0, 0.0, 1.0)
    G = np.zeros(inputs.GENOME_LEN)
    G[inputs.OFF_W1 + 0 * 64 + 0] = 1.0       # h1[0] = tanh(cos(2 pi v_x))
    G[inputs.OFF_W1 + 1 * 64 + 33] = 1.0      # h1[1] = tanh(sin(2 pi v_z))
    G[inputs.OFF_W2 + 0 * 64 + 0] = 1.0
    G[inputs.OFF_W2 + 1 * 64 + 1] = 1.0
    G[inputs.OFF_W3 + 0 * 64 + 0] = 1.0
    G[inputs.OFF_W3 + 1 * 64 + 1] = 1.0
    lg = orc.query(G, B, n)
    for vid in range(n ** 3):
        i, j, k = vid % n, (vid // n) % n, vid // (n * n)
        ex = math.tanh(math.tanh(math.cos(2 * math.pi * (i + 0.5) / n)))
        ez = math.tanh(math.tanh(math.sin(2 * math.pi * (k + 0.5) / n)))
        assert lg[vid, 0] == pytest.approx(ex, abs=1e-14)
        assert lg[vid, 1] == pytest.approx(ez, abs=1e-14)


# ---------------------------------------------------------------- largest component
def _scipy_lcc(cls, n):
    occ = (cls.reshape(n, n, n) != 0)          # [k][j][i]
    lab, nl = ndi.label(occ)                   # default structure = face connectivity
    if nl == 0:
        return np.zeros_like(cls)
    sizes = np.bincount(lab.ravel())[1:]
    flat = lab.ravel()
    best = max(range(1, nl + 1), key=lambda L: (sizes[L - 1], -np.flatnonzero(flat == L)[0]))
    return np.where(flat == best, cls, 0).astype(np.uint8)


@pytest.mark.parametrize("seed", range(12))
def test_lcc_matches_scipy_label(orc, seed):
    n = 3 + seed % 6
    cls, _ = inputs.random_voxels(n, seed, p_empty=0.35 + 0.03 * (seed % 5))
    assert np.array_equal(orc.lcc(cls, n), _scipy_lcc(cls, n))


def test_lcc_hand_cases(orc):
    n = 3
    cls = np.zeros(27, np.uint8)
    cls[0] = 1                      # (0,0,0)
    cls[1 + 3 * 1 + 9 * 1] = 2      # (1,1,1): touches (0,0,0) only at a corner
    kept = orc.lcc(cls, n)
    assert kept.tolist() == [1] + [0] * 26   # tie of size 1 -> smallest voxel id
    cls = np.zeros(27, np.uint8)
    cls[[0, 1]] = 3                 # blob of 2 along x
    cls[[24, 25, 26]] = 4           # blob of 3 in the top layer
    kept = orc.lcc(cls, n)
    assert np.flatnonzero(kept).tolist() == [24, 25, 26]


# ---------------------------------------------------------------- mesh
def _full(orc, n, c=4, w=0.5):
    return orc.Robot(n, np.full(n ** 3, c, np.uint8), np.full(n ** 3, w))


@pytest.mark.parametrize("n,M,S", [(1, 8, 28), (2, 27, 3 * 2 * 9 + 6 * 4 * 3 + 32), (4, 125, 1036),
                                   (8, 729, 7448), (10, 1331, 14230), (12, 2197, 24228)])
def test_full_grid_counts(orc, n, M, S):
    R = _full(orc, n)
    assert (R.M, R.S) == (M, S)
    assert S == 3 * n * (n + 1) ** 2 + 6 * n * n * (n + 1) + 4 * n ** 3


def test_two_face_adjacent_voxels(orc):
    cls = np.zeros(8, np.uint8)
    cls[[0, 1]] = 3
    R = orc.Robot(2, cls, np.ones(8))
    assert (R.M, R.S) == (12, 50)


def test_rest_lengths_degree_and_order(orc):
    n = 4
    R = _full(orc, n)
    sp = R.springs()
    L = np.round(sp["L0"] / 0.1, 12)
    assert (np.sum(L == 1.0), np.sum(L == round(math.sqrt(2), 12)), np.sum(L == round(math.sqrt(3), 12))) == \
        (3 * n * (n + 1) ** 2, 6 * n * n * (n + 1), 4 * n ** 3)
    ij = sp["ij"]
    assert np.all(ij[:, 0] < ij[:, 1])
    keys = ij[:, 0].astype(np.int64) * R.M + ij[:, 1]
    assert np.all(np.diff(keys) > 0)                       # canonical (min id, max id) order
    deg = np.bincount(ij.ravel(), minlength=R.M)
    assert deg.max() == 26 and deg.min() == 7


def test_sum_rule_homogeneous_grid(orc):
    # every spring of a homogeneous grid is shared by 1, 2 or 4 voxels (edges),
    # 1 or 2 (face diagonals) or exactly 1 (body diagonals)
    n, kc, w = 3, 3e4, 0.5
    R = _full(orc, n, c=4, w=w)
    sp = R.springs()
    mult = np.round(sp["k"] / (kc * w), 9)
    L = np.round(sp["L0"] / 0.1, 9)
    assert set(mult[L == 1.0]) == {1.0, 2.0, 4.0}
    assert set(mult[L == round(math.sqrt(2), 9)]) == {1.0, 2.0}
    assert set(mult[L == round(math.sqrt(3), 9)]) == {1.0}
    # brute force: number of kept voxels holding both endpoints of each spring
    nl = R.node_lattice()
    N = n + 1
    coords = np.stack([nl % N, (nl // N) % N, nl // (N * N)], 1)
    for s in range(0, R.S, 7):
        a, b = coords[sp["ij"][s, 0]], coords[sp["ij"][s, 1]]
        cnt = 0
        for vid in range(n ** 3):
            v = np.array([vid % n, (vid // n) % n, vid // (n * n)])
            if np.all((a >= v) & (a <= v + 1) & (b >= v) & (b <= v + 1)):
                cnt += 1
        assert mult[s] == cnt
    assert np.all(sp["a"] == 0) and np.all(sp["phi"] == 0)


def test_sum_rule_mixed_muscle_tissue(orc):
    # expanding muscle (k 1e4, a +0.2) beside soft tissue (k 3e3, a 0) sharing a face
    cls = np.zeros(8, np.uint8)
    cls[0], cls[1] = 1, 3
    w = np.zeros(8)
    w[0], w[1] = 0.8, 0.4
    R = orc.Robot(2, cls, w)
    sp = R.springs()
    k1, k3 = 1e4 * 0.8, 3e3 * 0.4
    shared = np.isclose(sp["k"], k1 + k3, rtol=1e-14)
    assert shared.sum() == 6          # 4 edges + 2 face diagonals of the shared face
    np.testing.assert_allclose(sp["a"][shared], 0.2 * k1 / (k1 + k3), rtol=1e-14)
    only_m = np.isclose(sp["k"], k1, rtol=1e-14)
    np.testing.assert_allclose(sp["a"][only_m], 0.2, rtol=1e-14)
    assert only_m.sum() == 22 and np.isclose(sp["k"], k3).sum() == 22


def test_contracting_muscle_negative_amplitude(orc):
    R = orc.Robot(1, np.array([2], np.uint8), np.array([1.0]))
    sp = R.springs()
    assert np.all(sp["a"] == -0.2) and np.all(sp["k"] == 1e4)


def test_initial_state_on_ground(orc):
    cls = np.zeros(27, np.uint8)
    cls[9 + 4] = 4                    # only the voxel (1,1,1)
    R = orc.Robot(3, cls, np.ones(27))
    x, v, step, _ = R.state()
    assert R.M == 8 and step == 0 and np.all(v == 0)
    assert x[:, 2].min() == 0.0
    np.testing.assert_allclose(sorted(set(np.round(x[:, 0], 12))), [0.1, 0.2])
    assert R.fitness() == 0.0
