"""Host-side logic of the co-design driver: the diversity measure and the
rule-based supervisor stand-in (no device work)."""
import numpy as np

from paper_2405_00698_amd.evolve import diversity, rule_supervisor


def test_diversity_identical_and_opposite():
    sides = [2, 2, 2]
    a = np.zeros(8, np.uint8)
    b = np.ones(8, np.uint8)
    kept = np.concatenate([a, a, b])
    G = np.array([[0.0, 0.0], [0.0, 0.0], [3.0, 4.0]])
    dm, dg = diversity(kept, sides, G)
    assert dm == (0 + 1 + 1) / 3
    assert dg == (0 + 5 + 5) / 3


def test_diversity_compares_equal_sides_only():
    sides = [2, 3]
    kept = np.concatenate([np.zeros(8, np.uint8), np.ones(27, np.uint8)])
    dm, _ = diversity(kept, sides, np.zeros((2, 3)))
    assert dm == 0.0


def test_rule_supervisor_raises_mutation_on_stall():
    base = dict(elite_frac=0.3, tournament_k=4, p_cross=0.4, p_mut=0.1, sigma=0.02)
    hist = [{"params": base, "fit_max": 1.0, "div_morph": 0.3}] * 3
    out = rule_supervisor(hist)
    assert out["p_mut"] > 0.1 and out["sigma"] > 0.02
    hist = [{"params": base, "fit_max": f, "div_morph": 0.3} for f in (1.0, 1.1, 1.2)]
    out = rule_supervisor(hist)
    assert out["p_mut"] == 0.1 and out["sigma"] == 0.02
