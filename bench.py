#!/usr/bin/env python3
"""Benchmark of the soft-robot co-design hot path on one MI355X.

One bench step is one generation of the co-design loop over the throughput
workload (4096 robots on 10x10x10 grids, random genomes): genome query and
mesh build, 10,000 simulation steps in the persistent LDS-resident kernel,
fitness, and the GA generation that produces the next genomes.  The metric is
spring updates per second over the whole generation.

Beside it the line carries the step kernel's LDS roofline (the bound the
metric names) and its VALU roofline, the other workloads of the method
(256 robots of 8^3; the uneven 1024-robot population over 20 generations;
the adjoint/forward time ratio at 64 robots of 8^3), the per-step-launch
form on the same GPU, and the FP64 oracle timed on the host cores.

Prints one JSON line.  Only one GPU is supported: the population would shard
across GPUs by robots, which this benchmark does not run.
"""
import argparse
import faulthandler
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Roofline denominators (MI355X: 256 CUs at 2.4 GHz).
CU, CLK = 256, 2.4e9
# LDS: CDNA4 reads 256 B/clk/CU with ds_read_b128 (twice CDNA3's 128 B/clk)
LDS_PEAK_GBS = CU * 256 * CLK / 1e9
# VALU: 4 SIMDs x 16 lanes per CU issue one FP32 lane-op slot per clock each;
# packed FP32 is not used by this library, so this unpacked rate is the ceiling
VALU_PEAK_SLOTS = CU * 64 * CLK
# Algorithmic work per unit (one spring update = one spring force applied to
# both ends in one step; one mass update = one node integrated in one step):
LDS_B_PER_SPRING = 24.0      # both endpoint positions, FP32 xyz
LDS_B_PER_MASS = 12.0        # each mass publishes its new position
# 3 sub (d), 3 (r^2), v_rsq_f32 (4 slots), 1 (r), 2 fma (actuated L), 1 sub,
# 2 mul (f / r), 3 mul (F), 3 add (both ends' accumulators)
VALU_SLOTS_PER_SPRING = 22.0
# gravity, ground normal, friction, damping, semi-implicit Euler
VALU_SLOTS_PER_MASS = 25.0


def measured_counters(kernel_cfg, sim_steps, key):
    """A per-launch counter figure of the step kernel from the committed
    rocprofv3 summary (profiles/hbm_traffic.json): key "hbm_bytes_per_launch"
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy probe) or "lds_bytes_per_launch"
    (LDS bandwidth counters); None when the kernel source or the launch differs
    from the one measured."""
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
    ap.add_argument("--cpu-robots", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=10000)
    ap.add_argument("--cpu-single-robots", type=int, default=8)
    ap.add_argument("--cpu-single-steps", type=int, default=2500)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads, the per-step-launch form and the adjoint ratio")
    ap.add_argument("--no-tune", action="store_true", help="keep the default step-kernel configuration")
    ap.add_argument("--kernel", default=None,
                    help="BLOCK,VARIANT: run the uniform workload with this step-kernel configuration (no tuning)")
    ap.add_argument("--only", default=None, choices=["adjoint", "uneven"],
                    help="run just the adjoint ratio (64 x 8^3) or the uneven 1024-robot generations and print "
                         "their figures (for profiling those workloads)")
    ap.add_argument("--gens", type=int, default=20, help="generations of the uneven workload with --only uneven")
    ap.add_argument("--adj-side", type=int, default=8, help="grid side of the 64 robots with --only adjoint")
    ap.add_argument("--adj-table2", action="store_true", help="the Table II model with --only adjoint")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB device copy (HBM counter calibration under rocprofv3)")
    return ap.parse_args()


def host_cpu():
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    return model


def cpu_baseline(args, genomes, B):
    """The FP64 oracle (built -O3 -march=native on this host) on the host
    cores, on bounded samples of the workload: all threads over robots, and
    one thread."""
    import oracle
    oracle.use_native()
    threads = oracle.num_threads()
    out = {"unit": "spring updates/s", "kind": "oracle", "cpu_model": host_cpu(), "nproc": os.cpu_count()}
    for label, nr, steps, th in (("all", args.cpu_robots, args.cpu_steps, threads),
                                 ("single", args.cpu_single_robots, args.cpu_single_steps, 1)):
        oracle.set_threads(th)
        robots = [oracle.robot_from_genome(genomes[r].astype(np.float64), B.astype(np.float64), args.side)
                  for r in range(nr)]
        S = sum(R.S for R in robots)
        t = time.perf_counter()
        oracle.pop_step(robots, steps)
        dt = time.perf_counter() - t
        rate = S * steps / dt
        if label == "all":
            out.update(value=rate, cores=th,
                       sample="%d robots of %d^3 from the same genomes, %d steps, FP64, one robot per thread "
                              "(%.1f s)" % (nr, args.side, steps, dt))
        else:
            out.update(single_thread_value=rate,
                       single_thread_sample="%d robots of %d^3, %d steps, one thread (%.1f s)"
                                            % (nr, args.side, steps, dt))
        del robots
    oracle.set_threads(threads)
    return out


def timed_steps(P, torch, steps):
    """Seconds of one pop_step(steps) from HIP events on the population's stream."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(P.stream)
    P.step(steps)
    e1.record(P.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3


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
    dt = timed_steps(P, torch, steps)
    P.close()
    return S * steps / dt


def uniform_workload(api, inputs, torch, R, n, steps, prec, tune_cache):
    """R robots of n^3 from random genomes: tuned persistent step rate."""
    from paper_2405_00698_amd import tune
    dev = torch.device("cuda:0")
    P = api.Population([n] * R)
    P.build_from_genomes(torch.from_numpy(inputs.random_genomes(R)).to(dev),
                         torch.from_numpy(inputs.gaussian_B()).to(dev), prec)
    tuned = tune.tune(P, steps=min(steps, 500), cache_path=tune_cache)
    S = sum(P.counts()[1])
    P.step(20)
    P.reset()
    dt = timed_steps(P, torch, steps)
    out = {"workload": "%d robots on %d^3 grids, %d steps" % (R, n, steps), "springs": S,
           "spring_updates_per_s": S * steps / dt, "seconds": dt, "kernel": P.kernel_config(n),
           "tuned": {str(k): list(v) for k, v in tuned.items()}}
    P.close()
    return out


def uneven_generations(api, inputs, torch, R, gens, steps, tune_cache):
    """The uneven population as configured: R robots with sides uniform on
    4..12 and empty fractions spread 0.1..0.5, BF16-MFMA genome query, `gens`
    generations of (build -> steps -> fitness -> GA, Table I rates)."""
    from paper_2405_00698_amd import SR_QUERY_BF16, tune
    from paper_2405_00698_amd.api import GAConfig, ga_generation
    dev = torch.device("cuda:0")
    sides = [int(q) for q in inputs.grid_sides(R, 4, 12)]
    G = [torch.from_numpy(inputs.random_genomes(R, empty_bias=inputs.uniform(R, -0.2, 0.4, seed=2))).to(dev),
         torch.empty((R, 8710), dtype=torch.float32, device=dev)]
    B = torch.from_numpy(inputs.gaussian_B()).to(dev)
    fit = torch.empty(R, dtype=torch.float32, device=dev)
    P = api.Population(sides)
    P.build_from_genomes(G[0], B, SR_QUERY_BF16)
    tuned = tune.tune(P, steps=500, cache_path=tune_cache)
    # one untimed call of the production length (captures its step graph)
    P.step(steps)
    P.reset()
    cfg = GAConfig()
    springs, sim_s = 0, 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(gens):
        P.build_from_genomes(G[g % 2], B, SR_QUERY_BF16)
        springs += sum(P.counts()[1])
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(P.stream)
        P.step(steps)
        e1.record(P.stream)
        P.fitness(fit)
        ga_generation(fit, G[g % 2], G[(g + 1) % 2], cfg, seed=inputs.SEED_GA, generation=g)
        e1.synchronize()
        sim_s += e0.elapsed_time(e1) / 1e3
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"workload": "%d robots with sides uniform on 4..12, empty fractions 0.1..0.5, BF16-MFMA query, "
                       "%d generations of %d steps, GA on (Table I rates)" % (R, gens, steps),
           "spring_updates_per_s": springs * steps / wall, "sim_spring_updates_per_s": springs * steps / sim_s,
           "seconds": wall, "sim_seconds": sim_s, "generations": gens,
           "kernels": {str(q): P.kernel_config(q) for q in sorted(set(sides))},
           "tuned": {str(k): list(v) for k, v in tuned.items()},
           "schedule": dict(zip(("sides", "lanes"), P.schedule())),
           "steps_per_launch": P.steps_per_launch or steps}
    P.close()
    return out


def model_rates(api, inputs, torch, R, n, steps, prec, tune_cache):
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
        tune.tune(P, steps=200, cache_path=tune_cache)
        S = sum(P.counts()[1])
        P.step(20)
        P.reset()
        dt = timed_steps(P, torch, steps)
        out[name] = {"spring_updates_per_s": S * steps / dt, "kernel": P.kernel_config(n)}
        P.close()
    return out


def adjoint_ratio(api, inputs, torch, n=8, table2=False):
    """64 robots of 8^3 (or side n; Table II model with table2), 2000 steps,
    checkpoint every 100 steps: pop_backward (segment recompute included) over
    the forward pop_step(2000), the forward timed both as it runs under
    recording (checkpoint copies between segment launches) and as the
    production forward (one captured graph launch)."""
    from paper_2405_00698_amd import SR_QUERY_FP32
    from paper_2405_00698_amd._lib import table2_params
    dev = torch.device("cuda:0")
    G = torch.from_numpy(inputs.random_genomes(64)).to(dev)
    B = torch.from_numpy(inputs.gaussian_B()).to(dev)
    params = table2_params() if table2 else None
    F = api.Population([n] * 64, params=params)
    F.build_from_genomes(G, B, SR_QUERY_FP32)
    F.step(2000)
    tg = []
    for _ in range(5):
        F.reset()
        tg.append(timed_steps(F, torch, 2000))
    F.close()
    P = api.Population([n] * 64, params=params)
    P.build_from_genomes(G, B, SR_QUERY_FP32)
    P.record(100, 2000)
    dJ = torch.ones(64, device=dev)
    tf, tb = [], []
    for _ in range(5):
        P.reset()
        tf.append(timed_steps(P, torch, 2000))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(P.stream)
        P.backward(dJ)
        e1.record(P.stream)
        e1.synchronize()
        tb.append(e0.elapsed_time(e1) / 1e3)
    P.close()
    f, g, b = float(np.median(tf)), float(np.median(tg)), float(np.median(tb))
    return {"value": b / g, "vs_recording_forward": b / f, "forward_graph_s": g, "forward_recording_s": f,
            "backward_s": b, "workload": "64 robots of %d^3%s, 2000 steps, checkpoint every 100, FP32; "
                                         "value = backward / forward as one graph launch"
                                         % (n, " (Table II model)" if table2 else "")}


def main():
    # a fatal signal in native code prints the Python stack instead of nothing
    faulthandler.enable()
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only; the population shards by robots across GPUs, "
              "which this build does not launch (got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2405_00698_amd import inputs, api, _lib
    from paper_2405_00698_amd import SR_QUERY_BF16, SR_QUERY_FP32, SR_STEP_PLAIN, SR_STEP_AUTO
    from paper_2405_00698_amd.api import ga_generation, GAConfig

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tune_cache = "/tmp/softrobot_tune.json"
    if args.only == "adjoint":
        print(json.dumps({"adjoint_forward_ratio": adjoint_ratio(api, inputs, torch, args.adj_side,
                                                                 args.adj_table2)}), flush=True)
        return
    if args.only == "uneven":
        print(json.dumps({"c3_uneven_1024": uneven_generations(api, inputs, torch, 1024, args.gens, 10000,
                                                               tune_cache)}), flush=True)
        return
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
    gacfg = GAConfig()

    tuned = None
    if args.kernel:
        b, v = (int(q) for q in args.kernel.split(","))
        P.set_persist_variant(args.side, b, v)
    elif not args.no_tune and args.mode == "persistent":
        # pick the fastest compiled step-kernel configuration for this population (cached)
        from paper_2405_00698_amd import tune
        P.build_from_genomes(Gt[0], Bt, prec)
        tuned = {int(k): list(v) for k, v in tune.tune(P, steps=500, cache_path=tune_cache).items()}

    stream = P.stream
    springs_per_gen = []
    sim_ms = []

    def one_generation(g, record):
        cur = Gt[g % 2]
        P.build_from_genomes(cur, Bt, prec)
        M, S, _, _ = P.counts()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P.step(args.sim_steps)
        e1.record(stream)
        P.fitness(fit)
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
    # the step kernel's average launch time, from HIP events on the stream it runs on
    kern_s = sum(a.elapsed_time(b) for a, b in sim_ms) / 1e3 / len(sim_ms)
    su_per_launch = total_springs / len(sim_ms)
    mu_per_launch = total_masses / len(sim_ms)
    lds_alg = su_per_launch * LDS_B_PER_SPRING + mu_per_launch * LDS_B_PER_MASS
    lds_gbs = lds_alg / kern_s / 1e9
    valu_alg = su_per_launch * VALU_SLOTS_PER_SPRING + mu_per_launch * VALU_SLOTS_PER_MASS
    valu = valu_alg / kern_s
    counted = args.mode == "persistent" and args.workload == "uniform"
    cfg_name = P.kernel_config(n) if counted else None
    lds_moved = measured_counters(cfg_name, args.sim_steps, "lds_bytes_per_launch") if counted else None
    hbm_moved = measured_counters(cfg_name, args.sim_steps, "hbm_bytes_per_launch") if counted else None
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
                               ", %d sim steps per generation (dt 1e-4 s), %s genome query, GA on"
                               % (args.sim_steps, args.query),
                   "robots": R, "grid_side": n if args.workload == "uniform" else "4..12",
                   "sim_steps": args.sim_steps, "mode": args.mode,
                   "springs_per_generation": springs_per_gen[0][0], "masses_per_generation": springs_per_gen[0][1],
                   "step_kernel": {q: P.kernel_config(q) for q in sorted(set(sides))}, "tuned": tuned},
        "sim_kernel_s": kern_s,
        "sim_spring_updates_per_s": su_per_launch / kern_s,
        # LDS bound: algorithmic bytes (24 B per spring update + 12 B per mass
        # update) per launch over the launch time; traffic = the LDS bytes the
        # kernel's instructions actually moved per launch (rocprofv3 counters)
        "roofline": {"bound": "lds", "achieved": lds_gbs, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                     "frac": lds_gbs / LDS_PEAK_GBS, "traffic": lds_moved,
                     "traffic_unit": "LDS bytes per launch (SQ_INSTS_LDS_LOAD/STORE_BANDWIDTH)",
                     "algorithmic_bytes_per_launch": lds_alg},
        # VALU co-bound: algorithmic FP32 lane-op slots (22 per spring update,
        # 25 per mass update) over the launch time, against the unpacked issue rate
        "roofline_valu": {"bound": "alu", "achieved": valu / 1e12, "peak": VALU_PEAK_SLOTS / 1e12,
                          "unit": "T lane-op slots/s", "frac": valu / VALU_PEAK_SLOTS,
                          "algorithmic_slots_per_launch": valu_alg},
        "hbm_traffic_per_launch": hbm_moved,
        "floors_s": {"lds": lds_alg / (LDS_PEAK_GBS * 1e9), "alu": valu_alg / VALU_PEAK_SLOTS},
    }
    if args.copy_probe:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 4
    if not args.no_extras and args.workload == "uniform":
        peaks = {name: api.microbench(name) for name in ("lds_read_16B", "lds_read_12B", "lds_read_4B",
                                                         "valu_fma", "valu_rsq", "hbm_copy")}
        out["measured_peaks"] = {k: (v / 1e12 if k.startswith("valu") else v / 1e9) for k, v in peaks.items()}
        out["measured_peaks"]["units"] = "LDS and HBM GB/s (copy: bytes read plus written), VALU T lane-ops/s"
        out["roofline"]["frac_of_measured_lds_16B"] = lds_gbs / out["measured_peaks"]["lds_read_16B"]
        if lds_moved is not None:
            out["roofline"]["moved_over_algorithmic"] = lds_moved / lds_alg
        out["roofline_valu"]["frac_of_measured_fma"] = valu / peaks["valu_fma"]
        P.close()
        pl = plain_baseline(api, inputs, torch, R, n, 500, prec)
        out["per_step_launch_spring_updates_per_s"] = pl
        out["persistent_over_per_step_launch"] = (su_per_launch / kern_s) / pl
        out["adjoint_forward_ratio"] = adjoint_ratio(api, inputs, torch)
        out["workloads"] = {
            "c2_256x8cubed": uniform_workload(api, inputs, torch, 256, 8, 10000, prec, tune_cache),
            "c3_uneven_1024": uneven_generations(api, inputs, torch, 1024, 20, 10000, tune_cache),
            "table2_model": [model_rates(api, inputs, torch, 4096, 5, 10000, prec, tune_cache),
                             model_rates(api, inputs, torch, 1024, 8, 5000, prec, tune_cache)],
        }
    if not args.no_cpu_baseline and args.workload == "uniform":
        out["cpu_baseline"] = cpu_baseline(args, G, B)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
