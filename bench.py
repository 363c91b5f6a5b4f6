#!/usr/bin/env python3
"""Benchmark of the soft-robot co-design hot path on one MI355X.

One bench step is one generation of the co-design loop over the throughput
workload (4096 robots on 10x10x10 grids, random genomes): genome query and
mesh build, 10,000 simulation steps in the persistent LDS-resident kernel,
fitness, and the GA generation that produces the next genomes.  The metric is
spring updates per second over the whole generation.

Prints one JSON line (rank 0).  Only one GPU is supported: the population
would shard across GPUs by robots, which this benchmark does not run.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# roofline denominators (MI355X: 256 CUs at 2.4 GHz)
CU, CLK = 256, 2.4e9
LDS_PEAK_GBS = CU * 128 * CLK / 1e9          # 128 B/clk/CU LDS bandwidth
VALU_PEAK_SLOTS = CU * 64 * CLK               # FP32 lane-op issue slots/s without packed math
LDS_B_PER_SPRING = 24.0                      # both endpoint positions, FP32 xyz
LDS_B_PER_MASS = 12.0                        # each mass publishes its position
VALU_SLOTS_PER_SPRING = 18.0                 # one force evaluation applied to both ends
VALU_SLOTS_PER_MASS = 20.0                   # gravity, ground, friction, damping, integrate


def measured_traffic(kernel_cfg, sim_steps, key="hbm_bytes_per_launch"):
    """HBM bytes per launch of the step kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (scaled by a copy probe), or with
    key="lds_bytes_per_launch" the LDS bytes its instructions moved (LDS
    bandwidth counters); None when the kernel source or the launch differs from
    the one measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    h = hashlib.sha256()
    for f in d["source_files"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != d["source_sha256"] or d["launch_steps"] != sim_steps or kernel_cfg not in d["kernels"]:
        return None
    return d["kernels"][kernel_cfg].get(key)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--robots", type=int, default=4096)
    ap.add_argument("--side", type=int, default=10)
    ap.add_argument("--workload", default="uniform", choices=["uniform", "uneven"],
                    help="uniform: all robots of --side; uneven: sides drawn uniformly from 4..12 and "
                         "empty-class biases U(-0.2, 0.4), only the largest component kept")
    ap.add_argument("--sim-steps", type=int, default=10000)
    ap.add_argument("--mode", default="persistent", choices=["persistent", "plain"])
    ap.add_argument("--query", default="fp32", choices=["bf16", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=5000)
    ap.add_argument("--cpu-robots", type=int, default=64)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the per-step-launch baseline and the adjoint/forward ratio")
    ap.add_argument("--no-tune", action="store_true", help="keep the default step-kernel configuration")
    ap.add_argument("--kernel", default=None,
                    help="BLOCK,VARIANT: run the uniform workload with this step-kernel configuration (no tuning)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB device copy (HBM counter calibration under rocprofv3)")
    return ap.parse_args()


def cpu_baseline(args, genomes, B):
    """The FP64 oracle on the host cores, on a bounded sample of the workload."""
    import oracle
    from paper_2405_00698_amd import inputs  # noqa: F401
    oracle.build()
    robots = [oracle.robot_from_genome(genomes[r].astype(np.float64), B.astype(np.float64), args.side)
              for r in range(args.cpu_robots)]
    S = sum(R.S for R in robots)
    t = time.perf_counter()
    oracle.pop_step(robots, args.cpu_steps)
    dt = time.perf_counter() - t
    return {"value": S * args.cpu_steps / dt, "unit": "spring updates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%d robots of %d^3 from the same genomes, %d steps, FP64, one robot per thread (%.1f s)"
                      % (args.cpu_robots, args.side, args.cpu_steps, dt)}


def plain_baseline(api, inputs, torch, R, n, steps, prec):
    """The same workload stepped by the per-step-launch kernel (state in HBM)."""
    from paper_2405_00698_amd import SR_STEP_PLAIN
    dev = torch.device("cuda:0")
    P = api.Population([n] * R)
    P.set_step_config(SR_STEP_PLAIN)
    P.build_from_genomes(torch.from_numpy(inputs.random_genomes(R)).to(dev),
                         torch.from_numpy(inputs.gaussian_B()).to(dev), prec)
    S = sum(P.counts()[1])
    P.step(20)
    torch.cuda.synchronize()
    t = time.perf_counter()
    P.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    P.close()
    return S * steps / dt


def model_rates(api, inputs, torch, R, n, steps, prec):
    """Step-kernel throughput of the base model and of the Table II model
    (weight-scaled muscles, spring and ground dashpots, static/kinetic
    friction) on the same genomes, each with its tuned kernel."""
    from paper_2405_00698_amd import tune, _lib
    dev = torch.device("cuda:0")
    G = torch.from_numpy(inputs.random_genomes(R)).to(dev)
    B = torch.from_numpy(inputs.gaussian_B()).to(dev)
    out = {"workload": "%d robots on %d^3 grids, %d steps" % (R, n, steps)}
    for name, params in (("base", _lib.default_params()), ("table2", _lib.table2_params())):
        P = api.Population([n] * R, params=params)
        P.build_from_genomes(G, B, prec)
        cfg = tune.tune(P, steps=200, cache_path="/tmp/softrobot_tune.json")
        S = sum(P.counts()[1])
        P.step(20)
        torch.cuda.synchronize()
        t = time.perf_counter()
        P.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        out[name] = {"spring_updates_per_s": S * steps / dt, "kernel": P.kernel_config(n),
                     "tuned_s": cfg[n][2]}
        P.close()
    return out


def adjoint_ratio(api, inputs, torch):
    """64 robots of 8^3, 2000 steps, checkpoint every 100 steps: pop_backward
    (segment recompute included) over the forward pop_step(2000)."""
    from paper_2405_00698_amd import SR_QUERY_FP32
    dev = torch.device("cuda:0")
    P = api.Population([8] * 64)
    P.build_from_genomes(torch.from_numpy(inputs.random_genomes(64)).to(dev),
                         torch.from_numpy(inputs.gaussian_B()).to(dev), SR_QUERY_FP32)
    P.record(100, 2000)
    dJ = torch.ones(64, device=dev)
    tf, tb = [], []
    for _ in range(3):
        P.reset()
        torch.cuda.synchronize()
        t = time.perf_counter()
        P.step(2000)
        torch.cuda.synchronize()
        tf.append(time.perf_counter() - t)
        t = time.perf_counter()
        P.backward(dJ)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t)
    P.close()
    f, b = float(np.median(tf)), float(np.median(tb))
    return {"value": b / f, "forward_s": f, "backward_s": b,
            "workload": "64 robots of 8^3, 2000 steps, checkpoint every 100, FP32"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only; the population shards by robots across GPUs, "
              "which this build does not launch (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2405_00698_amd import inputs, api, _lib
    from paper_2405_00698_amd import SR_QUERY_BF16, SR_QUERY_FP32, SR_STEP_PLAIN, SR_STEP_AUTO

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    R, n = args.robots, args.side
    B = inputs.gaussian_B()
    if args.workload == "uneven":
        sides = [int(q) for q in inputs.grid_sides(R, 4, 12)]
        G = inputs.random_genomes(R, empty_bias=inputs.uniform(R, -0.2, 0.4, seed=2))
    else:
        sides = [n] * R
        G = inputs.random_genomes(R)
    Bt = torch.from_numpy(B).to(dev)
    Gt = [torch.from_numpy(G).to(dev), torch.empty((R, _lib.GENOME_LEN), dtype=torch.float32, device=dev)]
    fit = torch.empty(R, dtype=torch.float32, device=dev)
    P = api.Population(sides)
    P.set_step_config(SR_STEP_PLAIN if args.mode == "plain" else SR_STEP_AUTO)
    prec = SR_QUERY_BF16 if args.query == "bf16" else SR_QUERY_FP32
    has_ga = hasattr(_lib.load(), "ga_generation")
    if has_ga:
        from paper_2405_00698_amd.api import ga_generation, GAConfig
        gacfg = GAConfig()

    tuned = None
    if args.kernel:
        b, v = (int(q) for q in args.kernel.split(","))
        P.set_persist_variant(args.side, b, v)
    elif not args.no_tune:
        # pick the fastest compiled step-kernel configuration for this population (cached)
        from paper_2405_00698_amd import tune
        P.build_from_genomes(Gt[0], Bt, prec)
        tuned = {int(k): list(v) for k, v in tune.tune(P, steps=500, cache_path="/tmp/softrobot_tune.json").items()}

    stream = torch.cuda.current_stream()
    springs_per_gen = []
    sim_ms = []

    def one_generation(g, record):
        # without the GA the same genomes are rebuilt every generation
        cur = Gt[g % 2] if has_ga else Gt[0]
        P.build_from_genomes(cur, Bt, prec)
        M, S, _, _ = P.counts()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.step(args.sim_steps)
        e1.record(stream)
        P.fitness(fit)
        if has_ga:
            ga_generation(fit, cur, Gt[(g + 1) % 2], gacfg, seed=inputs.SEED_GA, generation=g)
        if record:
            springs_per_gen.append((sum(S), sum(M)))
            sim_ms.append((e0, e1))

    for g in range(args.warmup):
        one_generation(g, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(args.warmup, args.warmup + args.steps):
        one_generation(g, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    total_springs = sum(s for s, _ in springs_per_gen) * args.sim_steps
    total_masses = sum(m for _, m in springs_per_gen) * args.sim_steps
    value = total_springs / wall
    kern_s = sum(a.elapsed_time(b) for a, b in sim_ms) / 1e3 / len(sim_ms)
    su_per_launch = total_springs / len(sim_ms)
    mu_per_launch = total_masses / len(sim_ms)
    lds_bytes = su_per_launch * LDS_B_PER_SPRING + mu_per_launch * LDS_B_PER_MASS
    lds_gbs = lds_bytes / kern_s / 1e9
    valu = (su_per_launch * VALU_SLOTS_PER_SPRING + mu_per_launch * VALU_SLOTS_PER_MASS) / kern_s
    # LDS bytes the kernel's instructions actually moved per launch (counters),
    # against the algorithmic bytes above
    lds_traffic = (measured_traffic(P.kernel_config(n), args.sim_steps, "lds_bytes_per_launch")
                   if args.mode == "persistent" and args.workload == "uniform" else None)
    out = {
        "metric": "spring updates/sec at 1 GPU (% LDS roofline); adjoint/forward time ratio",
        "value": value,
        "unit": "spring updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded random genomes (W ~ N(0, 1/64), b = 0), B ~ N(0, 1)",
        "config": {"workload": ("%d robots on %d^3 voxel grids" % (R, n) if args.workload == "uniform" else
                                "%d robots with sides uniform on 4..12" % R) +
                               ", %d sim steps per generation (dt 1e-4 s), %s genome query, GA %s"
                               % (args.sim_steps, args.query, "on" if has_ga else "off"),
                   "robots": R, "grid_side": n if args.workload == "uniform" else "4..12", "sim_steps": args.sim_steps, "mode": args.mode,
                   "springs_per_generation": springs_per_gen[0][0], "masses_per_generation": springs_per_gen[0][1],
                   "step_kernel": {q: P.kernel_config(q) for q in sorted(set(sides))}, "tuned": tuned},
        "sim_kernel_s": kern_s,
        "sim_spring_updates_per_s": su_per_launch / kern_s,
        # The VALU floor (algorithmic lane-op slots at the unpacked issue rate) is
        # higher than the LDS floor (algorithmic bytes at 128 B/clk/CU), so the
        # arithmetic roofline is the one that bounds the step kernel.
        "roofline": {"bound": "alu", "achieved": valu / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                     "unit": "T lane-op slots/s", "frac": valu / VALU_PEAK_SLOTS,
                     "traffic": measured_traffic(P.kernel_config(n), args.sim_steps)
                     if args.mode == "persistent" and args.workload == "uniform" else None},
        "roofline_lds": {"bound": "lds", "achieved": lds_gbs, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                         "frac": lds_gbs / LDS_PEAK_GBS, "traffic": lds_traffic,
                         "traffic_frac": None if lds_traffic is None else lds_traffic / kern_s / 1e9 / LDS_PEAK_GBS},
        "floors_s": {"alu": (su_per_launch * VALU_SLOTS_PER_SPRING + mu_per_launch * VALU_SLOTS_PER_MASS)
                     / VALU_PEAK_SLOTS, "lds": lds_bytes / (LDS_PEAK_GBS * 1e9)},
    }
    if args.copy_probe:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 4
    if not args.no_extras and args.workload == "uniform":
        peaks = {name: api.microbench(name) for name in ("lds_read_16B", "lds_read_12B", "lds_read_4B",
                                                         "valu_fma", "valu_rsq")}
        out["measured_peaks"] = {k: (v / 1e9 if k.startswith("lds") else v / 1e12) for k, v in peaks.items()}
        out["measured_peaks"]["units"] = "LDS GB/s, VALU T lane-ops/s"
        out["roofline_lds"]["frac_of_measured_lds_16B"] = lds_gbs / out["measured_peaks"]["lds_read_16B"]
        out["roofline"]["frac_of_measured_fma"] = valu / peaks["valu_fma"]
        P.close()
        pl = plain_baseline(api, inputs, torch, R, n, 500, prec)
        out["per_step_launch_spring_updates_per_s"] = pl
        out["persistent_over_per_step_launch"] = (su_per_launch / kern_s) / pl
        out["adjoint_forward_ratio"] = adjoint_ratio(api, inputs, torch)
        out["material_models"] = [model_rates(api, inputs, torch, 4096, 5, 10000, prec),
                                  model_rates(api, inputs, torch, 1024, 8, 5000, prec)]
    if not args.no_cpu_baseline and args.workload == "uniform":
        out["cpu_baseline"] = cpu_baseline(args, G, B)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
