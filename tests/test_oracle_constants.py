"""The oracle's default constants against the values the paper prints
(Table I and Table II, stored in tests/golden/paper_tables.json).  Where the
hot-path workload overrides a table value (time step, stiffness per class,
damping and friction), the override is named here explicitly."""
import json
import os

import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


def test_table_values_used_on_the_hot_path(orc):
    t = json.load(open(GOLD))
    d = orc.DEFAULTS
    assert d["gravity"] == t["table_II_physics"]["gravity_m_s2"]
    assert d["mass"] == t["table_II_physics"]["mass_per_index_kg"]
    assert d["voxel_len"] == t["table_II_physics"]["original_rest_length_m"]
    assert d["k_ground"] == t["table_II_plane"]["elastic_coefficient_N_m"]
    # workload overrides of Table II
    assert d["dt"] == 1e-4 and d["damping"] == 0.999 and d["mu"] == 0.5
    assert tuple(d["k_class"]) == (0.0, 1e4, 1e4, 3e3, 3e4)
    assert tuple(d["a_class"]) == (0.0, 0.2, -0.2, 0.0, 0.0)


def test_table_I_rates_are_the_ga_defaults(orc):
    import inspect
    t = json.load(open(GOLD))["table_I_general"]
    sig = inspect.signature(orc.ga_generation).parameters
    assert sig["p_mut"].default == t["initial_mutation_rate"]
    assert sig["p_cross"].default == t["initial_crossover_rate"]
    assert sig["elite_frac"].default == t["initial_elite_percentage"]
    assert sig["sigma"].default == 0.02          # workload's N(0, 0.02) overrides the 0.1 scale
