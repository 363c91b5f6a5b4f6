"""Batching and launch machinery: captured step graphs (with one parallel
branch per grid side) against direct launches, the tuner, and the uneven
co-design loop (sides 4..12, BF16 query, GA) run end to end twice."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, gpu_population, need_gpu, say, voxel_population
from paper_2405_00698_amd import SR_QUERY_BF16, SR_STEP_PLAIN, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("plain", [False, True])
def test_graphs_match_direct_launches_bitwise(plain):
    sides = [int(n) for n in inputs.grid_sides(24, 4, 12)]
    cls, w = voxel_population(sides, 61)
    outs = []
    for graphs in (True, False):
        P = gpu_population(sides, cls, w)
        if plain:
            P.set_step_config(SR_STEP_PLAIN)
        P.set_graphs(graphs)
        for n in (37, 37, 100, 1):    # repeated keys replay the cached graph
            P.step(n)
        x, v, st = P.state()
        assert st == 175
        outs.append((x.cpu().numpy(), v.cpu().numpy(), P.fitness().cpu().numpy()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_launch_schedules_give_the_same_bits():
    """Every size group computes only its own robots, so the order of the
    groups' launches and the streams they go to change no result; the
    schedule travels into captured graphs and is validated."""
    from paper_2405_00698_amd import SoftRobotError
    sides = [int(n) for n in inputs.grid_sides(40, 4, 12)]
    cls, w = voxel_population(sides, 63)
    P = gpu_population(sides, cls, w)
    desc = sorted(set(sides), reverse=True)
    assert P.schedule() == (desc, list(range(len(desc))))
    P.set_step_config(steps_per_launch=40)
    P.step(120)
    ref = P.state()[0].cpu().numpy()
    scheds = [(desc, [i % 2 for i in range(len(desc))]), (desc[::-1], [0] * len(desc)),
              (desc, [(3 * i) % len(desc) for i in range(len(desc))])]
    for order, lanes in scheds:
        P.set_schedule(order, lanes)
        assert P.schedule() == (list(order), list(lanes))
        for graphs in (True, False):
            P.set_graphs(graphs)
            P.reset()
            P.step(120)
            assert np.array_equal(P.state()[0].cpu().numpy(), ref), (order, lanes, graphs)
    for order, lanes in ((desc[1:], list(range(len(desc) - 1))), (desc, [len(desc)] * len(desc)),
                         ([desc[0]] * len(desc), list(range(len(desc)))), ([13] + desc[1:], list(range(len(desc))))):
        with pytest.raises(SoftRobotError):
            P.set_schedule(order, lanes)


def test_tuner_picks_a_compiled_config_and_keeps_results(tmp_path):
    from paper_2405_00698_amd import tune, api
    sides = [6] * 16 + [10] * 16
    cls, w = voxel_population(sides, 62)
    P = gpu_population(sides, cls, w)
    P.step(150)
    ref = P.state()[0].cpu().numpy()
    res = tune.tune(P, steps=50, cache_path=str(tmp_path / "tune.json"), verbose=True)
    for n, (b, v, t) in res.items():
        assert (b, v) in api.persist_configs(n)
        assert P.persist_variant(n) == (b, v)
    P.step(150)
    assert np.array_equal(P.state()[0].cpu().numpy(), ref)
    sched = P.schedule()
    res2 = tune.tune(P, steps=50, cache_path=str(tmp_path / "tune.json"))
    assert {n: r[:2] for n, r in res.items()} == {n: r[:2] for n, r in res2.items()}
    assert P.schedule() == sched


def test_uneven_codesign_loop_is_reproducible():
    """1024 robots with sides 4..12 and empty fractions spread 0.1..0.5:
    build (BF16 MFMA) -> 500 steps -> fitness -> GA, three generations, twice."""
    from paper_2405_00698_amd.api import GAConfig, Population, ga_generation
    R = 1024
    sides = [int(n) for n in inputs.grid_sides(R, 4, 12)]
    B = torch.from_numpy(inputs.gaussian_B()).to(DEV)
    G0 = inputs.random_genomes(R, seed=1, empty_bias=inputs.uniform(R, -0.2, 0.4, seed=2))
    finals = []
    for rep in range(2):
        P = Population(sides)
        G = [torch.from_numpy(G0).to(DEV), torch.empty((R, inputs.GENOME_LEN), device=DEV)]
        fits = []
        for g in range(3):
            P.build_from_genomes(G[g % 2], B, SR_QUERY_BF16)
            P.step(500)
            f = P.fitness()
            fits.append(f.cpu().numpy())
            ga_generation(f, G[g % 2], G[(g + 1) % 2], GAConfig(), seed=3, generation=g)
        finals.append((G[1].cpu().numpy(), np.array(fits)))
        M, S, _, _ = P.counts()
        say("uneven loop rep", rep, "mean springs %.0f max %d" % (np.mean(S), max(S)))
        assert np.all(np.isfinite(fits[-1]))
    assert np.array_equal(finals[0][0], finals[1][0])
    assert np.array_equal(finals[0][1], finals[1][1])


def test_microbenchmarks_report_positive_rates():
    from paper_2405_00698_amd import api
    rates = {k: api.microbench(k, iters=256) for k in api.MICRO}
    say("microbenchmarks", {k: "%.3g" % v for k, v in rates.items()})
    assert all(v > 0 for v in rates.values())


def test_codesign_driver_paper_shape_short():
    """The paper's experiment shape (30 robots of 5^3, Table I rates), 4
    generations of 2000 steps with the supervisor stand-in: statistics logged,
    best fitness never lost (elites are re-simulated at their slot's side,
    equal here), reproducible."""
    from paper_2405_00698_amd.evolve import evolve, rule_supervisor
    h1 = evolve([5] * 30, generations=4, sim_steps=2000, supervisor=rule_supervisor)
    h2 = evolve([5] * 30, generations=4, sim_steps=2000, supervisor=rule_supervisor)
    assert [r["fit_max"] for r in h1] == [r["fit_max"] for r in h2]
    best = [r["fit_max"] for r in h1]
    assert all(b2 >= b1 for b1, b2 in zip(best, best[1:]))
    say("paper-shape run", [("%.4f" % r["fit_max"], "%.3f" % r["div_morph"]) for r in h1])


def test_codesign_driver_table2_model_and_sigma_sweep():
    """The co-design loop under the Table II model (weighted muscles, dashpots,
    dt 1e-5 s) and a two-value sweep of the encoding scale sigma_B."""
    from paper_2405_00698_amd._lib import table2_params
    from paper_2405_00698_amd.evolve import sigma_sweep
    res = sigma_sweep([0.5, 2.0], [5] * 30, generations=3, sim_steps=3000, sim_params=table2_params())
    for s, runs in res.items():
        best = [r["fit_max"] for r in runs[0]]
        assert all(np.isfinite(best)) and all(b2 >= b1 for b1, b2 in zip(best, best[1:]))
        say("sigma_B", s, "best", ["%.5f" % b for b in best], "diversity %.3f" % runs[0][-1]["div_morph"])


def test_codesign_loop_resumes_at_a_generation_bitwise():
    """A run stopped after generation g - 1 and resumed from its genomes at
    generation g repeats generations g..G of the uninterrupted run bit for bit
    (the GA draws depend only on (seed, generation, child)); two resume points,
    an uneven population."""
    from paper_2405_00698_amd.evolve import evolve
    sides = [4, 5, 6, 4, 7, 5, 6, 8, 4, 5, 6, 4, 7, 5, 6, 8]
    R, G, steps = len(sides), 6, 400
    full = torch.empty((R, inputs.GENOME_LEN), device=DEV)
    h_full = evolve(sides, generations=G, sim_steps=steps, out_genomes=full)
    for g in (2, 4):
        mid = torch.empty((R, inputs.GENOME_LEN), device=DEV)
        h_a = evolve(sides, generations=g, sim_steps=steps, out_genomes=mid)
        end = torch.empty((R, inputs.GENOME_LEN), device=DEV)
        h_b = evolve(sides, generations=G - g, sim_steps=steps, start_generation=g, genomes=mid, out_genomes=end)
        assert [r["generation"] for r in h_b] == list(range(g, G))
        for key in ("fit_max", "fit_mean", "fit_min", "div_morph", "div_genome"):
            assert [r[key] for r in h_a + h_b] == [r[key] for r in h_full], (g, key)
        assert torch.equal(end, full), g
    say("resume: best fitness per generation", ["%.4f" % r["fit_max"] for r in h_full])
