"""Co-design loop driver (Sec. II-C, Table I): each generation builds every
robot from its genome (Eq. (1) encoding, MLP, heads), simulates it, scores
it, and breeds the next genomes on the device.

The paper steers the GA with an LLM that reads the parameters and the
population of the previous three generations and proposes new parameters
(Sec. II-D).  Here that role is a plain callback, `supervisor(history) ->
GAConfig`, called once per generation with the last three generations'
parameters and statistics; `rule_supervisor` is a deterministic stand-in.
Every step of the hot path runs in the HIP library; this module only
sequences the calls and logs per-generation statistics (fitness min / mean /
max and a diversity measure) on the host.
"""
import json
import time

import numpy as np
import torch

from . import SR_QUERY_BF16, inputs
from .api import GAConfig, Population, ga_generation


def diversity(kept_cls, sides, genomes):
    """Mean pairwise Hamming distance between the robots' kept-class grids
    (robots of equal side only; a class differs or a voxel is kept in one and
    not the other), and the mean pairwise L2 distance between genomes."""
    out_h, pairs = 0.0, 0
    offs = np.concatenate([[0], np.cumsum([n ** 3 for n in sides])])
    by_side = {}
    for r, n in enumerate(sides):
        by_side.setdefault(n, []).append(kept_cls[offs[r]:offs[r + 1]])
    for n, grids in by_side.items():
        g = np.stack(grids)
        for i in range(len(g)):
            d = (g[i + 1:] != g[i]).mean(axis=1)
            out_h += d.sum()
            pairs += len(d)
    G = genomes.astype(np.float64)
    sq = (G * G).sum(1)
    d2 = np.maximum(sq[:, None] + sq[None, :] - 2 * G @ G.T, 0.0)
    iu = np.triu_indices(len(G), 1)
    return (out_h / pairs if pairs else 0.0), float(np.sqrt(d2[iu]).mean()) if len(iu[0]) else 0.0


def rule_supervisor(history):
    """Deterministic stand-in for the LLM supervisor: when the best fitness
    stalls for the last three generations or the morphology diversity falls,
    raise the mutation rate and scale; otherwise relax them towards Table I."""
    cur = history[-1]["params"]
    rate, sigma = cur["p_mut"], cur["sigma"]
    if len(history) >= 3:
        best = [h["fit_max"] for h in history[-3:]]
        div = [h["div_morph"] for h in history[-3:]]
        if best[-1] <= best[0] or div[-1] < 0.5 * div[0]:
            rate, sigma = min(0.3, rate * 1.5), min(0.1, sigma * 1.5)
        else:
            rate, sigma = max(0.1, rate * 0.9), max(0.02, sigma * 0.9)
    return dict(cur, p_mut=rate, sigma=sigma)


def evolve(sides, generations=100, sim_steps=10000, seed_genome=1, seed_ga=3, sigma_B=1.0,
           params=None, supervisor=None, empty_bias=None, log=None, precision=SR_QUERY_BF16,
           sim_params=None, start_generation=0, genomes=None, out_genomes=None, **sim):
    """Runs `generations` generations on the given grid sides; returns the
    per-generation history (parameters, fitness statistics, diversity, times).
    sim_params: a full sr_sim_params (e.g. table2_params()); else the defaults
    with the keyword overrides in **sim.
    Resuming: `genomes` ([R, 8710], host or device) replaces the seeded
    initial genomes and `start_generation` numbers the first generation run
    (the GA draws depend only on (seed_ga, generation, child)), so a run
    stopped after generation g - 1 and resumed with its genomes at g repeats
    the uninterrupted run bit for bit.  out_genomes (device [R, 8710]) receives
    the genomes the last generation bred."""
    dev = torch.device("cuda:0")
    R = len(sides)
    params = dict(elite_frac=0.3, tournament_k=4, p_cross=0.4, p_mut=0.1, sigma=0.02) if params is None else params
    B = torch.from_numpy(inputs.gaussian_B(sigma=sigma_B)).to(dev)
    if genomes is None:
        g0 = torch.from_numpy(inputs.random_genomes(R, seed=seed_genome, empty_bias=empty_bias)).to(dev)
    else:
        g0 = torch.as_tensor(genomes, dtype=torch.float32).to(dev).clone()
    G = [g0, torch.empty((R, inputs.GENOME_LEN), dtype=torch.float32, device=dev)]
    P = Population(sides, params=sim_params, **sim)
    fit = torch.empty(R, dtype=torch.float32, device=dev)
    history = []
    for i in range(generations):
        g = start_generation + i
        t0 = time.perf_counter()
        cur, nxt = G[i % 2], G[(i + 1) % 2]
        P.build_from_genomes(cur, B, precision)
        P.step(sim_steps)
        P.fitness(fit)
        f = fit.cpu().numpy()
        kept = P.voxels()[0].cpu().numpy()
        dm, dg = diversity(kept, sides, cur.cpu().numpy())
        finite = f[np.isfinite(f)]
        rec = {"generation": g, "params": dict(params),
               "fit_max": float(finite.max()) if len(finite) else float("-inf"),
               "fit_mean": float(finite.mean()) if len(finite) else float("-inf"),
               "fit_min": float(finite.min()) if len(finite) else float("-inf"),
               "diverged": int((~np.isfinite(f)).sum()), "div_morph": dm, "div_genome": dg}
        history.append(rec)
        if supervisor is not None:
            params = supervisor(history[-3:])
        ga_generation(fit, cur, nxt, GAConfig(**params), seed=seed_ga, generation=g)
        torch.cuda.synchronize()
        rec["seconds"] = time.perf_counter() - t0
        if log is not None:
            log.write(json.dumps(rec) + "\n")
            log.flush()
    if out_genomes is not None and generations > 0:
        out_genomes.copy_(G[generations % 2])
    P.close()
    return history


def sigma_sweep(sigmas, sides, repeats=1, **kw):
    """Sweep the standard deviation of the encoding matrix B (Sec. II-B states
    that it was chosen by a sweep but gives no values): runs `evolve` once per
    (sigma, repeat), the repeat changing the genome seed, and returns
    {sigma: [history, ...]}."""
    seed0 = kw.pop("seed_genome", 1)
    return {float(s): [evolve(sides, sigma_B=float(s), seed_genome=seed0 + r, **kw) for r in range(repeats)]
            for s in sigmas}


if __name__ == "__main__":
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="co-design loop: the paper's shape is 30 robots of 5^3, 100 generations")
    ap.add_argument("--robots", type=int, default=30)
    ap.add_argument("--side", type=int, default=5)
    ap.add_argument("--generations", type=int, default=100)
    ap.add_argument("--sim-steps", type=int, default=10000)
    ap.add_argument("--sigma-B", type=float, default=1.0, help="standard deviation of the encoding matrix B")
    ap.add_argument("--supervisor", action="store_true", help="use the rule-based stand-in for the LLM supervisor")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--repeats", type=int, default=1, help="independent runs (genome seeds seed, seed+1, ...)")
    ap.add_argument("--sigma-sweep", default=None, help="comma-separated values of sigma_B to sweep")
    ap.add_argument("--table2", action="store_true",
                    help="Table II material and contact model (dt 1e-5 s, weighted muscles, dashpots)")
    a = ap.parse_args()
    from ._lib import table2_params
    simp = table2_params() if a.table2 else None
    sup = rule_supervisor if a.supervisor else None
    sigmas = [float(q) for q in a.sigma_sweep.split(",")] if a.sigma_sweep else [a.sigma_B]
    for s in sigmas:
        for r in range(a.repeats):
            sys.stdout.write(json.dumps({"sigma_B": s, "repeat": r}) + "\n")
            evolve([a.side] * a.robots, a.generations, a.sim_steps, seed_genome=a.seed + r, sigma_B=s,
                   supervisor=sup, log=sys.stdout, sim_params=simp)
