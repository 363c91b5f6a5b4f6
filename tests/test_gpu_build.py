"""GPU genome query (Eq. (1) encoding, MLP, softmax/sigmoid heads) in FP32 and
in BF16-on-MFMA, against the FP64 oracle, and the full genome -> robot ->
simulation path.  Classes must agree wherever the oracle's top-two logit
margin exceeds the precision's bound (1e-4 for FP32, 0.1 for BF16); the
sigmoid weight within 1e-5 (FP32) or 1e-2 (BF16)."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, gpu_states, need_gpu, rel_err, say
from paper_2405_00698_amd import SR_QUERY_BF16, SR_QUERY_FP32, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _oracle_heads(orc, G, B, sides):
    out = []
    for r, n in enumerate(sides):
        lg = orc.query(G[r].astype(np.float64), B.astype(np.float64), n)
        cls, w = orc.heads(lg)
        srt = np.sort(lg[:, :5], axis=1)
        out.append((cls, w, srt[:, -1] - srt[:, -2]))
    return out


def _gpu_query(sides, G, B, prec):
    from paper_2405_00698_amd.api import Population
    P = Population(sides)
    P.build_from_genomes(torch.from_numpy(G).to(DEV), torch.from_numpy(B).to(DEV), prec)
    cls, w = P.query()
    return P, cls.cpu().numpy(), w.cpu().numpy()


@pytest.mark.parametrize("prec,margin,wtol", [(SR_QUERY_FP32, 1e-4, 1e-5), (SR_QUERY_BF16, 0.1, 1e-2)])
def test_query_matches_oracle(orc, prec, margin, wtol):
    sides = [4] * 8 + [1, 2, 3, 5, 6, 7, 8, 9, 10, 11, 12] + [5] * 17   # 36 robots, partial last MFMA tiles
    R = len(sides)
    B = inputs.gaussian_B()
    G = inputs.random_genomes(R, seed=41, empty_bias=inputs.uniform(R, -0.2, 0.4, seed=41))
    say("query precision", prec)
    P, cls, w = _gpu_query(sides, G, B, prec)
    ref = _oracle_heads(orc, G, B, sides)
    o = 0
    agree = total = 0
    for r, n in enumerate(sides):
        c_o, w_o, m_o = ref[r]
        sl = slice(o, o + n ** 3)
        clear = m_o > margin
        assert np.array_equal(cls[sl][clear], c_o[clear]), r
        np.testing.assert_allclose(w[sl], w_o, atol=wtol, rtol=0)
        agree += np.sum(cls[sl] == c_o)
        total += n ** 3
        o += n ** 3
    say("class agreement %.5f over %d voxels" % (agree / total, total))
    assert agree / total > (0.9999 if prec == SR_QUERY_FP32 else 0.98)


def test_bf16_and_fp32_builds_are_close():
    sides = [10] * 64
    B = inputs.gaussian_B()
    G = inputs.random_genomes(64, seed=43)
    _, c32, w32 = _gpu_query(sides, G, B, SR_QUERY_FP32)
    _, c16, w16 = _gpu_query(sides, G, B, SR_QUERY_BF16)
    assert np.mean(c32 == c16) > 0.98
    assert np.abs(w32 - w16).max() < 1e-2


def test_genome_pipeline_parity(orc):
    """Genome -> FP32 query -> robot -> 200 contact steps, against the oracle pipeline,
    on the robots whose every voxel has a clear class decision."""
    sides = [4] * 8
    B = inputs.gaussian_B()
    G = inputs.random_genomes(8, seed=1)
    P, cls, w = _gpu_query(sides, G, B, SR_QUERY_FP32)
    ref = _oracle_heads(orc, G, B, sides)
    P.step(200)
    xs, _, _ = gpu_states(P)
    fit = P.fitness().cpu().numpy()
    checked = 0
    for r, (c_o, w_o, m_o) in enumerate(ref):
        if m_o.min() <= 1e-4:
            continue
        Ro = orc.Robot(4, c_o, w_o)
        Ro.step(200)
        xo = Ro.state()[0]
        assert rel_err(xs[r], xo) <= 1e-3
        assert abs(fit[r] - Ro.fitness()) <= 1e-3 * np.abs(xo).max()
        checked += 1
    assert checked >= 6
