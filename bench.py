"""Benchmark: population TabuCol moves/s on one MI355X.

Default workload (the configuration the headline metric is quoted on):
G(500, 0.5) from seed 0, k = 49, population 8192, 100,000 tabu iterations
per individual, one wavefront per individual with everything in LDS: byte
gamma whose top bit flags the current colour and tabu pairs, and a list of
the live tabu pairs (five individuals resident per CU).  One step = random population initialisation + one full TabuCol
pass over the population (every kernel of the search path); the graph is
uploaded once, before timing.  Step s uses initial-colouring seed
1 + s so every step searches new individuals.

Prints ONE JSON line (rank 0).  value = total tabu moves / timed wall time.
roofline (primary): the LDS-bandwidth bound of the TabuCol kernel with a
fixed byte model per iteration and move (entry sizes 2 B for gamma, tabu
expiry and colour, 4 B gamma on the 18-colour G(100, 0.5) workload), summed
over the kernel's exact counters (conflicting vertices scanned, degrees of
the moved vertices, moves), divided by the kernel's average duration from
HIP events on the launch stream, against the nominal 256 CU x 128 B/clk x
2.4 GHz and against the peak a probe kernel measures in the same run.
roofline_alu, roofline_lds_tier (the table tier's own entry sizes) and
roofline_hbm are secondary views of the same launch; traffic is the HBM byte
count measured with rocprofv3 for the same launch.
cpu_baseline: the CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

GNP500_BLOCK = 64
GNP500_TABLE = "wave8"
LDS_PEAK_GBS = 256 * 128 * 2.4  # GB/s: 256 CUs x 128 B/clk x 2.4 GHz
HBM_PEAK_GBS = 8000.0
# 32-bit integer vector ops: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
METRIC = "tabu moves/sec (population, 1 GPU) + time-to-legal-k-coloring, learned vs plain"


# HBM bytes per launch of the benchmarked TabuCol launch, from two rocprofv3
# --pmc runs (FETCH_SIZE, WRITE_SIZE), each scaled by what the counter reads
# for a 1 GiB device-to-device copy.  Valid only for the kernel sources they
# were taken on (digest below) and the same table and block; otherwise null.
MEASURED_TRAFFIC = {"sources_sha256": "90f622ede0f2d30055248402ea1008c515523046e0683b22b3d379670c082e06",
                    "table": "wave8", "block": 64, "bytes": 27144576}  # profiles/tabucol_wave8_gnp500.md
KERNEL_SOURCES = ("paper_2109_05948_amd/csrc/tabu_body.h", "paper_2109_05948_amd/csrc/tabucol.hip",
                  "paper_2109_05948_amd/csrc/dlm_common.h", "paper_2109_05948_amd/csrc/tabu_wave.h")


# HBM bytes of the two distance launches of one diversity step (old x new
# block + new x new triangle), from the same counter runs
DIVERSITY_TRAFFIC = {"sources_sha256": "9f79de36c3bbbdb83d6884a3ccb01ff45ffbb8d43bbc23bc6ed9041fc722adea", "bytes": 1629448352}  # profiles/distance_diversity_gnp500.md
DIVERSITY_SOURCES = ("paper_2109_05948_amd/csrc/diversity.hip", "paper_2109_05948_amd/csrc/dlm_common.h")


def kernel_sources_digest(sources=None) -> str:
    import hashlib
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for rel in sources or KERNEL_SOURCES:
        with open(os.path.join(root, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(table: str, block: int):
    m = MEASURED_TRAFFIC
    if m["bytes"] is None or m["table"] != table or m["block"] != block:
        return None
    return m["bytes"] if kernel_sources_digest() == m["sources_sha256"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# bytes of one table entry by tier: (gamma in LDS, tabu in LDS, gamma in device memory, tabu in device memory)
TIER_BYTES = {"lds16": (2, 2, 0, 0), "lds32": (4, 4, 0, 0), "split16": (2, 0, 0, 2),
              "split8": (1, 0, 0, 2), "global16": (0, 0, 2, 2),
              # byte gamma whose top bit flags tabu pairs: no separate tabu entry
              "wave8": (1, 0, 0, 0)}
# the search kernel of each table tier (the dominant kernel of a launch)
TIER_KERNEL = {"wave8": "tabucol_w8_kernel"}


def lds_bytes(st: np.ndarray, k: int, table: str = "lds16", s_col: int = 2) -> float:
    """Algorithmic LDS bytes of a TabuCol run from its counters, with the
    entry sizes of the table tier (g, u: LDS bytes of a gamma and a tabu entry).

    per iteration: C_t (k-1) (g + u)     [candidate scan]
                 + C_t (g + s_col)       [current colour and its gamma]
    per move:      deg(v*) (4 g + s_col) [neighbour gamma updates, read + write]
                 + u + s_col             [tabu entry, colour of v*]
    st columns: 0 moves, 2 sum C_t, 3 sum deg(v*).
    """
    g, u = TIER_BYTES[table][:2]
    return lds_model_bytes(st, k, g, u, s_col)


def lds_model_bytes(st: np.ndarray, k: int, s_g: int, s_t: int, s_col: int) -> float:
    """The same byte model with given entry sizes."""
    moves, sum_c, sum_deg = float(st[:, 0].sum()), float(st[:, 2].sum()), float(st[:, 3].sum())
    return sum_c * ((k - 1) * (s_g + s_t) + s_g + s_col) + sum_deg * (4 * s_g + s_col) + moves * (s_t + s_col)


def fixed_lds_bytes(st: np.ndarray, k: int) -> float:
    """The fixed model that does not depend on the storage chosen: gamma,
    tabu and colour entries of 2 bytes each (4-byte gamma when k <= 18, the
    G(100, 0.5) workload's int32 table)."""
    return lds_model_bytes(st, k, 4 if k <= 18 else 2, 2, 2)


def alu_ops(st: np.ndarray, k: int) -> float:
    """Algorithmic 32-bit integer operations of a TabuCol run from its counters.

    Per candidate (v, c) examined: delta = gamma[v][c] - gamma[v][col v], the
    tabu test, the aspiration test, their combination and the comparison with
    the running best (5).  Per neighbour u of the moved vertex: the two gamma
    updates and the two own-colour tests (4).  Tie hashing, reductions and
    bookkeeping are not counted.
    st columns: 2 sum C_t, 3 sum deg(v*).
    """
    return float(5 * st[:, 2].sum() * (k - 1) + 4 * st[:, 3].sum())


def hbm_bytes(st: np.ndarray, k: int, table: str = "lds16") -> float:
    """Algorithmic device-memory bytes: the CSR row of v* (4 B per neighbour)
    per move, plus the table entries the tier keeps in device memory (same
    terms as the LDS model with the device-memory entry sizes)."""
    g, u = TIER_BYTES[table][2:]
    moves, sum_c, sum_deg = st[:, 0].sum(), st[:, 2].sum(), st[:, 3].sum()
    return float(4 * sum_deg + sum_c * ((k - 1) * (g + u) + g) + sum_deg * 4 * g + moves * u)


def host_cores() -> int:
    """Cores this process may run on (the affinity mask, which is what the
    oracle's OpenMP threads can use)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(g, k, T, seed, init_seed, count, threads):
    import oracle
    ids = np.arange(count, dtype=np.int32)
    starts = oracle.init_random(g.n, k, count, seed=init_seed)
    t0 = time.perf_counter()
    r = oracle.tabucol_batch(g, starts, ids, k, T, seed=seed, nthreads=threads)
    dt = time.perf_counter() - t0
    moves = int(r["stats"][:, 0].sum())
    return {"value": moves / dt, "unit": "moves/s", "cores": threads, "kind": "oracle",
            "sample": f"{count} individuals x {T} iterations of the same workload "
                      f"({moves} moves in {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gnp500",
                    choices=["gnp500", "gnp100", "uneven64", "wvcp300", "memetic1000", "scorer", "diversity",
                             "decreasing", "popsweep", "invnet", "predict", "gemm"])
    ap.add_argument("--pops", default="100,400,1600,6400,25600,51200", help="popsweep: population sizes")
    ap.add_argument("--sweep-graph", default="wvcp500", choices=["wvcp500", "wvcp300"],
                    help="popsweep: the weighted graph")
    ap.add_argument("--passes", type=int, default=3,
                    help="popsweep: budget = this many local-search passes of the largest population")
    ap.add_argument("--budget-pop", type=int, default=0,
                    help="popsweep: the population the budget's passes are counted in (default: the largest of "
                         "--pops), so that runs split over several commands share one budget")
    ap.add_argument("--cutoff", type=float, default=300.0,
                    help="memetic1000: wall-clock limit per loop (seconds)")
    ap.add_argument("--loops", default="plain,learned", help="memetic1000: which loops to run")
    ap.add_argument("--k", type=int, default=0, help="memetic1000: colours (default: the workload's 85)")
    ap.add_argument("--seeds", default="1", help="memetic1000: comma-separated loop seeds")
    ap.add_argument("--diversity", type=int, default=0,
                    help="memetic1000: K > 0 runs the loops with the paper's diversity steps (K nearest "
                         "neighbours, one child per individual, spacing update)")
    ap.add_argument("--network", default="mlp", choices=["mlp", "invariant"],
                    help="memetic1000: the learned loop's scorer (the per-class MLP, or the paper's "
                         "colour-invariant network at its k-COL depth)")
    ap.add_argument("--epochs", type=int, default=0,
                    help="memetic1000: training epochs per generation (default: the workload's)")
    ap.add_argument("--generations", type=int, default=16, help="predict: generations per loop")
    ap.add_argument("--eval-chunk", type=int, default=2048, help="invnet: colourings per evaluation pass")
    ap.add_argument("--block", type=int, default=GNP500_BLOCK)
    ap.add_argument("--table", default=GNP500_TABLE)
    ap.add_argument("--pop", type=int, default=0, help="override the population (testing only)")
    ap.add_argument("--cpu-sample", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (the reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for {args.gpus}); "
              "the population shards by individual with no communication between shards",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {n} bytes 3 times")
        return

    import paper_2109_05948_amd as dlm
    from workloads import workload

    if args.workload == "scorer":
        return bench_scorer(args, workload("memetic1000"), dlm, torch)
    if args.workload == "diversity":
        return bench_diversity(args, workload("gnp500"), dlm, torch)
    if args.workload == "invnet":
        return bench_invnet(args, workload("gnp500"), dlm, torch)
    if args.workload == "gemm":
        return bench_gemm(args, workload("gnp500"), dlm, torch)
    if args.workload == "predict":
        return bench_predict(args, workload("wvcp300"), dlm, torch)
    if args.workload == "popsweep":
        return bench_popsweep(args, workload(args.sweep_graph), workload("memetic1000"), dlm, torch)
    if args.workload == "decreasing":
        return bench_decreasing(args, workload("gnp500"), workload("memetic1000"), dlm, torch)
    w = workload(args.workload)
    if args.workload == "uneven64":
        return bench_uneven(args, w, dlm, torch)
    if args.workload == "wvcp300":
        return bench_wvcp(args, w, dlm, torch)
    if args.workload == "memetic1000":
        return bench_memetic(args, w, dlm, torch)
    g, k, T = w.graphs[0], w.k[0], w.iters[0]
    pop = args.pop or w.pop
    G = dlm.Graph.from_csr(g)
    dev = torch.device("cuda:0")
    colors = torch.empty((pop, g.n), dtype=torch.int16, device=dev)
    stream = torch.cuda.current_stream()

    def step(s, ev=None):
        dlm.init_population(G, k, pop, seed=w.init_seed + s, colors=colors)
        if ev:
            ev[0].record(stream)
        r = dlm.tabu_batch(G, colors, k, T, w.tabu_seed, block=args.block, table=args.table)
        if ev:
            ev[1].record(stream)
        return r

    for s in range(args.warmup):
        log(f"warmup step {s}")
        step(1000 + s)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    stats = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        r = step(s, evs[s])
        stats.append(r["stats"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = torch.cat(stats).cpu().numpy()
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    moves = int(st[:, 0].sum())
    log(f"timed {args.steps} steps in {dt:.3f} s; tabu kernel {kern_ms:.2f} ms/launch; "
        f"moves {moves}; no-ops {int(st[:, 1].sum())}")

    traffic = measured_traffic(args.table, args.block) if pop == w.pop else None
    sec = kern_ms * 1e-3
    per_launch = {"moves": float(st[:, 0].sum()) / args.steps, "sum_conflicting": float(st[:, 2].sum()) / args.steps,
                  "sum_deg": float(st[:, 3].sum()) / args.steps, "noops": float(st[:, 1].sum()) / args.steps}
    fixed_lds = fixed_lds_bytes(st, k) / args.steps
    tier_lds = lds_bytes(st, k, args.table) / args.steps
    per_launch_ops = alu_ops(st, k) / args.steps
    # HBM per the fixed model: the CSR row of every moved vertex
    fixed_hbm = 4.0 * per_launch["sum_deg"]
    tier_hbm = hbm_bytes(st, k, args.table) / args.steps
    lds_gbs, hbm_gbs = fixed_lds / sec / 1e9, fixed_hbm / sec / 1e9
    alu_tops = per_launch_ops / sec / 1e12
    # the LDS peak measured by the probe kernel on this device, in this run
    probe_gbs = dlm.probe_lds_bandwidth(20000) / 1e9
    log(f"LDS probe {probe_gbs:.0f} GB/s")
    out = {
        "metric": METRIC,
        "value": moves / dt,
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": f"G(n={g.n}, p=0.5) seed 0", "k": k,
                   "population": pop, "iters_per_individual": T, "block": args.block,
                   "table": args.table, "parallelism": "population (one workgroup per individual)"},
        "roofline": {"bound": "lds", "achieved": lds_gbs, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                     "frac": lds_gbs / LDS_PEAK_GBS, "traffic": traffic,
                     "peak_measured": probe_gbs, "frac_measured": lds_gbs / probe_gbs,
                     "model": "fixed entry sizes (gamma, tabu, colour) = (%d, 2, 2) B" % (4 if k <= 18 else 2),
                     "kernel": TIER_KERNEL.get(args.table, "tabucol_kernel"), "kernel_ms": kern_ms, "bytes_per_launch": fixed_lds,
                     "counters_per_launch": per_launch},
        "roofline_hbm": {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": hbm_gbs / HBM_PEAK_GBS, "bytes_per_launch": fixed_hbm, "traffic": traffic,
                         "model": "CSR row of the moved vertex, 4 B per neighbour"},
        "roofline_alu": {"bound": "alu", "achieved": alu_tops, "peak": ALU_PEAK_TOPS, "unit": "Tops/s",
                         "frac": alu_tops / ALU_PEAK_TOPS, "ops_per_launch": per_launch_ops},
        "roofline_lds_tier": {"bound": "lds", "achieved": tier_lds / sec / 1e9, "peak": LDS_PEAK_GBS,
                              "unit": "GB/s", "frac": tier_lds / sec / 1e9 / LDS_PEAK_GBS,
                              "bytes_per_launch": tier_lds, "device_bytes_per_launch": tier_hbm,
                              "model": f"entry sizes of the {args.table} table"},
        "tabu_kernel_moves_per_s": moves / args.steps / sec,
    }
    if args.workload == "gnp500" and pop == w.pop and args.table != "lds16":
        # the same search with the 16-bit LDS table the configuration names
        # (gamma and expiry packed in one LDS word): a sample of the population
        # large enough to fill every CU several times over
        ns = 4096
        cs = torch.empty((ns, g.n), dtype=torch.int16, device=dev)
        dlm.init_population(G, k, ns, seed=w.init_seed, colors=cs)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        r16 = dlm.tabu_batch(G, cs, k, T, w.tabu_seed, block=256, table="lds16")
        e1.record(stream)
        torch.cuda.synchronize()
        s16 = r16["stats"].cpu().numpy()
        ms16 = e0.elapsed_time(e1)
        out["lds16_sample"] = {"individuals": ns, "kernel_ms": ms16, "block": 256,
                               "moves_per_s": float(s16[:, 0].sum()) / (ms16 * 1e-3),
                               "lds_frac": fixed_lds_bytes(s16, k) / (ms16 * 1e-3) / 1e9 / LDS_PEAK_GBS}
        log(f"lds16 sample: {ns} individuals in {ms16:.1f} ms")
    if not args.no_cpu_baseline and args.workload == "gnp500":
        threads = host_cores()
        log(f"cpu baseline: oracle on {args.cpu_sample} individuals, {threads} threads "
            f"(affinity mask; os.cpu_count() = {os.cpu_count()})")
        out["cpu_baseline"] = cpu_baseline(g, k, T, w.tabu_seed, w.init_seed, args.cpu_sample,
                                           threads)
    print(json.dumps(out), flush=True)


def _line(metric, value, unit, args, dt, config, extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3 / max(args.steps, 1),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
           "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def bench_uneven(args, w, dlm, torch):
    """64 graphs of uneven size, 256 individuals each, one persistent hipGraph launch."""
    jobs = []
    for gi, (g, k, T) in enumerate(zip(w.graphs, w.k, w.iters)):
        G = dlm.Graph.from_csr(g)
        col, _ = dlm.init_population(G, k, w.pop, seed=w.init_seed, ind_base=gi * w.pop)
        jobs.append({"graph": G, "colors": col, "k": k, "iters": T, "seed": w.tabu_seed,
                     "ind_base": gi * w.pop})
    starts = [j["colors"].clone() for j in jobs]
    log("autotuning the persistent launch")
    (block, budget), rates = dlm.MultiBatch.autotune(jobs, calib_iters=1000)
    log(f"autotune: block {block}, LDS budget {budget}; rates {rates.tolist()}")
    mb = dlm.MultiBatch(jobs, block=block, lds_budget=budget)
    info = mb.info()
    log(f"plan {info}")

    def reset():
        for j, s0 in zip(jobs, starts):
            j["colors"].copy_(s0)

    for _ in range(args.warmup):
        reset()
        mb.launch()
    torch.cuda.synchronize()
    moves, dt = 0, 0.0
    for _ in range(args.steps):
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mb.launch()
        torch.cuda.synchronize()
        dt += time.perf_counter() - t0
        moves += sum(int(j["stats"][:, 0].sum().item()) for j in jobs)
    solved = sum(int((j["f_best"] == 0).sum().item()) for j in jobs)
    _line("tabu moves/sec, uneven 64-graph batch in one persistent hipGraph launch", moves / dt,
          "moves/s", args, dt,
          {"workload": "uneven64", "graphs": len(jobs), "population_per_graph": w.pop,
           "iters_per_individual": "128 n", "block": block, "lds_budget": budget, **info},
          {"individuals_legal": solved, "autotune_rates": rates.tolist()})


def bench_wvcp(args, w, dlm, torch):
    """Weighted colouring: greedy init, 10 rounds x 10 n iterations, population 4096."""
    g = w.graphs[0]
    G = dlm.Graph.from_csr(g)
    rounds = w.extra["rounds"]
    moves, dt, best = 0, 0.0, None
    for s in range(args.warmup + args.steps):
        col, ku = dlm.init_population(G, 0, w.pop, seed=w.init_seed + s, mode="greedy")
        k = int(ku.max().item())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = dlm.wvcp_batch(G, col, k, w.iters[0], rounds, seed=w.tabu_seed)
        torch.cuda.synchronize()
        if s >= args.warmup:
            dt += time.perf_counter() - t0
            moves += int(r["stats"][:, 0].sum().item())
            b = int(r["best_legal"].min().item())
            best = b if best is None else min(best, b)
    _line("weighted tabu moves/sec (population, 1 GPU)", moves / dt, "moves/s", args, dt,
          {"workload": "wvcp300", "graph": "G(n=300, p=0.3) seed 0, weights U{1..100}",
           "k": k, "population": w.pop, "rounds": rounds, "iters_per_round": w.iters[0]},
          {"best_legal_wscore": best})


def bench_memetic(args, w, dlm, torch):
    """Time to a legal k-colouring: learned offspring selection vs random
    selection, each loop run once per seed with the same wall-clock cutoff.
    value = the learned loop's median time over the seeds (a run that misses
    the cutoff counts as infinite; null if the median does)."""
    from paper_2109_05948_amd import memetic
    from workloads.invnet_init import col_widths, invnet_weights
    from workloads.scorer_init import scorer_weights
    g, T = w.graphs[0], w.iters[0]
    k = args.k or w.k[0]
    G = dlm.Graph.from_csr(g)
    e = w.extra
    pop = args.pop or w.pop
    seeds = [int(x) for x in args.seeds.split(",")]
    epochs = args.epochs or e["epochs"]
    if args.network == "invariant":  # the paper's network: its batch of 100
        params = invnet_weights(g.n, col_widths(g.n), seed=0)
        params["widths"] = col_widths(g.n)
        batch = 100
    else:
        params, batch = scorer_weights(g.n, seed=0), e["batch"]
    res = {}
    for name in args.loops.split(","):
        runs = []
        for sd in seeds:
            log(f"memetic {name} k={k} seed={sd}")
            r = memetic.run(G, k, pop, T, learned=(name == "learned"), seed=sd,
                            cutoff_s=args.cutoff, children_per_pair=e["children_per_pair"],
                            keep_frac=e["keep_frac"], scorer_params=params, batch=batch, epochs=epochs,
                            lr=e["lr"], log=log, diversity=args.diversity > 0,
                            neighbours=max(args.diversity, 1), network=args.network)
            runs.append({"seed": sd, "time_to_legal_s": r.time_to_legal, "best_f": r.best,
                         "generations": r.generations, "wall_s": r.wall,
                         "tabu_moves_per_s": r.tabu_moves / r.wall,
                         "history": [list(h) for h in r.history]})
        times = sorted(x["time_to_legal_s"] if x["time_to_legal_s"] is not None else float("inf")
                       for x in runs)
        med = times[len(times) // 2] if len(times) % 2 else 0.5 * (times[len(times) // 2 - 1] + times[len(times) // 2])
        res[name] = {"median_time_to_legal_s": med if med != float("inf") else None,
                     "legal_runs": sum(t != float("inf") for t in times), "runs": runs}
    out = {"metric": "time-to-legal-k-coloring, learned vs plain (seconds, lower is better)",
           "value": res.get("learned", {}).get("median_time_to_legal_s"), "unit": "s", "n_gpus": 1,
           "higher_is_better": False, "vs_baseline": None, "dtype": "int16+bf16",
           "data": "synthetic",
           "config": {"workload": "memetic1000", "graph": "G(n=1000, p=0.5) seed 0", "k": k,
                      "population": pop, "children_per_pair": e["children_per_pair"],
                      "keep_frac": e["keep_frac"], "iters_per_tabu": T, "cutoff_s": args.cutoff,
                      "seeds": seeds, "diversity_neighbours": args.diversity, "network": args.network,
                      "train_batch": batch, "epochs": epochs},
           "loops": res}
    print(json.dumps(out), flush=True)


def bench_scorer(args, w, dlm, torch):
    """The offspring scorer at the memetic shape (G(1000, 0.5), k = 85): score
    the 32,768 GPX offspring of one generation, then train on 8,192 (start,
    result) pairs for 5 epochs at batch 1024.  Inputs are random colourings
    and standardised-normal targets, resident before timing.

    Per colouring, inference gathers one FP32 W1 row (H1 = 256 floats) per
    vertex and runs kpad x 256 x 128 BF16 MFMA products (kpad = k rounded up
    to 32); training adds the two backward products (dH1, dW2) and the dW1
    scatter, so about 3x the MFMA work and 2x the gather bytes."""
    from workloads.scorer_init import scorer_weights
    g, k = w.graphs[0], w.k[0]
    n, h1, h2 = g.n, 256, 128
    kpad = (k + 31) // 32 * 32
    G = dlm.Graph.from_csr(g)
    nchild, npairs, batch, epochs = 32768, 8192, 1024, 5
    sc = dlm.Scorer(n, k, scorer_weights(n, seed=0), max_batch=batch)
    col, _ = dlm.init_population(G, k, nchild, seed=5)
    gen = torch.Generator().manual_seed(11)
    tgt = torch.randn(npairs, generator=gen).to("cuda")
    scores = torch.empty(nchild, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        sc.score(col, out=scores)
        sc.train(col[:npairs], tgt, batch, epochs)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        ev[s_][0].record(stream)
        sc.score(col, out=scores)
        ev[s_][1].record(stream)
        sc.train(col[:npairs], tgt, batch, epochs)
        ev[s_][2].record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    inf_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    tr_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    gather_b = float(nchild) * n * h1 * 4
    mfma_f = float(nchild) * 2 * kpad * h1 * h2
    inf_gbs = gather_b / (inf_ms * 1e-3) / 1e9
    tr_tflops = 3 * float(npairs * epochs) * 2 * kpad * h1 * h2 / (tr_ms * 1e-3) / 1e12
    out = {"metric": "offspring scored/s (learned selection, memetic shape)", "value": nchild / (inf_ms * 1e-3),
           "unit": "colourings/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3 / max(args.steps, 1), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16+fp32", "data": "synthetic",
           "config": {"workload": "scorer", "graph": "G(n=1000, p=0.5) seed 0", "k": k,
                      "offspring": nchild, "train_pairs": npairs, "batch": batch, "epochs": epochs},
           "inference_ms": inf_ms, "train_ms": tr_ms,
           "train_pairs_per_s": npairs * epochs / (tr_ms * 1e-3),
           "roofline": {"bound": "hbm", "achieved": inf_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": inf_gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "scorer_fwd_kernel",
                        "note": "W1 rows gathered per colouring (L2-resident, 1 MB)"},
           "roofline_mfma": {"bound": "mfma", "achieved": mfma_f / (inf_ms * 1e-3) / 1e12, "peak": 2500.0,
                             "unit": "TFLOP/s", "frac": mfma_f / (inf_ms * 1e-3) / 1e12 / 2500.0,
                             "train_achieved": tr_tflops}}
    print(json.dumps(out), flush=True)


def bench_popsweep(args, w, wm, dlm, torch):
    """Sensitivity to the population size at a fixed total number of local-
    search iterations (the study of the paper's Section 4 on the WVCP): the
    learned memetic loop on the weighted G(500, 0.5) of wvcp500 (the shape of
    the paper's DSJC500.5 study), greedy start, 10 rounds of 10 n iterations
    per local search, for each population p and each seed as many
    generations as the budget allows (budget = passes x the largest p local
    searches; the largest p gets passes - 1 generations).  Reports the best
    legal weighted score reached by each (p, seed) and its trajectory."""
    from paper_2109_05948_amd import memetic
    from workloads.scorer_init import scorer_weights
    g = w.graphs[0]
    G = dlm.Graph.from_csr(g)
    pops = [int(x) for x in args.pops.split(",")]
    seeds = [int(x) for x in args.seeds.split(",")]
    per_search = 10 * g.n * 10
    budget = args.passes * (args.budget_pop or max(pops)) * per_search
    e = wm.extra
    out_runs = []
    for p in pops:
        passes = budget // (p * per_search)
        for sd in seeds:
            log(f"popsweep p={p} seed={sd}: {passes} local-search passes ({passes - 1} generations)")
            r = memetic.run(G, 0, p, 10 * g.n, learned=True, seed=sd,
                            cutoff_s=args.cutoff, max_generations=max(passes - 1, 0),
                            children_per_pair=e["children_per_pair"], keep_frac=e["keep_frac"],
                            scorer_params=scorer_weights(g.n, seed=0), batch=min(e["batch"], p),
                            epochs=e["epochs"], lr=e["lr"], weighted=True, rounds=10, log=log,
                            diversity=args.diversity > 0, neighbours=max(args.diversity, 1),
                            slice_rows=8192)
            out_runs.append({"population": p, "seed": sd, "generations": r.generations,
                             "best_wscore": r.best, "wall_s": r.wall, "moves": r.tabu_moves,
                             "history": [[h[0], h[1], h[2]] for h in r.history]})
            log(f"popsweep p={p} seed={sd}: best {r.best} after {r.generations} generations, {r.wall:.1f} s")
    best = min(out_runs, key=lambda x: (x["best_wscore"], x["population"]))
    out = {"metric": "best legal weighted score at a fixed tabu budget vs population size (lower is better)",
           "value": best["best_wscore"], "unit": "weighted score", "n_gpus": 1, "higher_is_better": False,
           "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "popsweep", "graph": f"{w.name}: G(n={g.n}) weights U{{1..100}}",
                      "populations": pops, "seeds": seeds, "iters_per_search": per_search,
                      "budget_iters": budget, "best_population": best["population"]},
           "runs": out_runs}
    print(json.dumps(out), flush=True)


def bench_decreasing(args, w, wm, dlm, torch):
    """COL by decreasing k (Section 2.7) on G(500, 0.5), the shape of
    DSJC500.5: the memetic loop from k (default 53), k dropping by one after
    every legal colouring, population 8192, 128 n tabu iterations per
    offspring, the memetic1000 generation settings, one overall cutoff.
    value = the smallest k coloured legally; the record lists when each k
    was first solved."""
    from paper_2109_05948_amd import memetic
    from workloads.scorer_init import scorer_weights
    g = w.graphs[0]
    G = dlm.Graph.from_csr(g)
    k0 = args.k or 53
    pop, T, e = args.pop or w.pop, 128 * g.n, wm.extra
    res = {}
    for name in args.loops.split(","):
        sd = int(args.seeds.split(",")[0])
        log(f"decreasing {name} from k={k0} seed={sd}")
        r = memetic.decreasing_k(G, k0, pop, T, learned=(name == "learned"), seed=sd, cutoff_s=args.cutoff,
                                 scorer_params=scorer_weights(g.n, seed=0), log=log,
                                 children_per_pair=e["children_per_pair"], keep_frac=e["keep_frac"],
                                 batch=e["batch"], epochs=e["epochs"], lr=e["lr"],
                                 diversity=args.diversity > 0, neighbours=max(args.diversity, 1))
        res[name] = {"best_k": r.best_k, "found": [[k, t] for k, t in r.found], "wall_s": r.wall,
                     "generations": [x.generations for x in r.runs]}
    best = [v["best_k"] for v in res.values() if v["best_k"] is not None]
    out = {"metric": "smallest k coloured legally by decreasing-k COL within the cutoff (lower is better)",
           "value": min(best) if best else None, "unit": "colours", "n_gpus": 1, "higher_is_better": False,
           "vs_baseline": None, "dtype": "int16+bf16", "data": "synthetic",
           "config": {"workload": "decreasing", "graph": "G(n=500, p=0.5) seed 0", "k_start": k0,
                      "population": pop, "iters_per_tabu": T, "cutoff_s": args.cutoff,
                      "diversity_neighbours": args.diversity},
           "loops": res}
    print(json.dumps(out), flush=True)


def bench_diversity(args, w, dlm, torch):
    """One generation's diversity step at the G(500, 0.5), k = 49 shape with
    8192 individuals: the old x new and new x new partition distances
    written into the pool matrix (100.6 M pairs), the spacing update of the
    16,384-member pool (spacing |V| / 10), the gather of the survivors'
    distances and rows, and the 16 nearest neighbours of every survivor.
    Inputs are two Philox-random populations and their conflict counts,
    resident before timing.

    The distance kernel is bound by issue (integer ALU): per pair, the
    algorithmic work is n overlap increments plus two greedy passes of at
    most k steps over k classes, n + 2 k^2 operations."""
    g, k = w.graphs[0], w.k[0]
    n, p = g.n, args.pop or w.pop
    G = dlm.Graph.from_csr(g)
    old, _ = dlm.init_population(G, k, p, seed=21)
    new, _ = dlm.init_population(G, k, p, seed=22)
    f_old, _ = dlm.evaluate(G, old, k)
    f_new, _ = dlm.evaluate(G, new, k)
    pools = [torch.zeros((2 * p, 2 * p), dtype=torch.int32, device="cuda") for _ in range(2)]
    dlm.partition_distance(old, k, out=pools[0][:p, :p])  # the carried old x old block
    stream = torch.cuda.current_stream()
    spacing, K = n // 10, 16
    pairs = p * p + p * (p - 1) // 2

    def step(ev=None):
        pool, nxt = pools[0], pools[1]
        if ev:
            ev[0].record(stream)
        dlm.partition_distance(old, k, new, out=pool[:p, p:])
        dlm.partition_distance(new, k, out=pool[p:, p:], upper_only=True)
        if ev:
            ev[1].record(stream)
        pick, nsp = dlm.spacing_update(f_old, f_new, pool, p, spacing)
        if ev:
            ev[2].record(stream)
        dlm.gather_distances(pool, pick, out=nxt[:p, :p])
        rows, fs = dlm.gather_pool(old, f_old, new, f_new, pick)
        nn = dlm.nearest(nxt, K, p=p)
        if ev:
            ev[3].record(stream)
        return nsp, nn

    for s_ in range(args.warmup):
        log(f"warmup step {s_}")
        step()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        nsp, _ = step(ev[s_])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dist_ms = float(np.mean([a.elapsed_time(b) for a, b, _, _ in ev]))
    upd_ms = float(np.mean([b.elapsed_time(c) for _, b, c, _ in ev]))
    rest_ms = float(np.mean([c.elapsed_time(d) for _, _, c, d in ev]))
    ops = float(pairs) * (n + 2 * k * k)
    tops = ops / (dist_ms * 1e-3) / 1e12
    log(f"timed {args.steps} steps in {dt:.3f} s; distances {dist_ms:.1f} ms, spacing update {upd_ms:.1f} ms, "
        f"gathers + nearest {rest_ms:.1f} ms; {int(nsp.item())} of {p} taken under the spacing")
    out = {"metric": "partition distances/s (population diversity step)", "value": pairs / (dist_ms * 1e-3),
           "unit": "pairs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": dt * 1e3 / max(args.steps, 1), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "diversity", "graph": "G(n=500, p=0.5) seed 0", "k": k, "population": p,
                      "pairs": pairs, "spacing": spacing, "nearest": K},
           "distance_ms": dist_ms, "spacing_update_ms": upd_ms, "gather_nearest_ms": rest_ms,
           "n_spaced": int(nsp.item()),
           "roofline": {"bound": "alu", "achieved": tops, "peak": ALU_PEAK_TOPS, "unit": "Tops/s",
                        "frac": tops / ALU_PEAK_TOPS, "kernel": "distance_kernel",
                        "traffic": (DIVERSITY_TRAFFIC["bytes"] if p == 8192 and
                                    kernel_sources_digest(DIVERSITY_SOURCES) == DIVERSITY_TRAFFIC["sources_sha256"]
                                    else None),
                        "ops_per_pair": n + 2 * k * k}}
    print(json.dumps(out), flush=True)


def invnet_flops(n, k, widths, b, train):
    """GEMM flops of one pass over b colourings: per layer the class rows
    (b k x l_in x l_out) and the class means (b x l_in x l_out); training adds
    the weight gradients of both and, above the first layer, the input
    gradients of both."""
    f, l_in = 0.0, n
    for j, l_out in enumerate(widths):
        per = 2.0 * (b * k + b) * l_in * l_out
        f += per
        if train:
            f += per * (2 if j > 0 else 1)
        l_in = l_out
    return f


def bench_invnet(args, w, dlm, torch):
    """The paper's colour-invariant network for k-COL at the G(500, 0.5),
    k = 49 shape (hidden widths 10n, 5n, 2n x 5, n, n // 2; 44.3 M
    trainables): one generation's scoring of 8192 colourings (evaluation, in
    chunks of --eval-chunk, 2048 by default) and one training epoch over 8192 (colouring, score) pairs
    at the paper's batch of 100 (82 Adam steps).  Inputs are Philox-random
    colourings and standard-normal targets, resident before timing; weights
    from the seeded fully connected initialisation.

    Every product is a BF16 GEMM with FP32 accumulation (the library's MFMA
    kernel, dlm_gemm_bf16); the rest
    (one-hot input, class means, normalisation, activation, loss, Adam) runs
    on the library's kernels.  The roofline is the dense BF16 MFMA peak."""
    from workloads.invnet_init import col_widths, invnet_weights
    g, k = w.graphs[0], w.k[0]
    n, p = g.n, args.pop or w.pop
    widths = col_widths(n)
    batch, chunk = 100, args.eval_chunk
    G = dlm.Graph.from_csr(g)
    net = dlm.InvNet(n, k, widths, invnet_weights(n, widths, seed=0), max_batch=chunk)
    col, _ = dlm.init_population(G, k, p, seed=31)
    gen = torch.Generator().manual_seed(12)
    tgt = torch.randn(p, generator=gen).to("cuda")
    scores = torch.empty(p, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    for s_ in range(args.warmup):
        log(f"warmup step {s_}")
        net.forward(col, out=scores)
        net.train(col, tgt, batch, 1)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        ev[s_][0].record(stream)
        net.forward(col, out=scores)
        ev[s_][1].record(stream)
        losses = net.train(col, tgt, batch, 1)
        ev[s_][2].record(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    inf_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    tr_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    inf_f = invnet_flops(n, k, widths, p, False)
    tr_f = invnet_flops(n, k, widths, p, True)
    inf_tf = inf_f / (inf_ms * 1e-3) / 1e12
    tr_tf = tr_f / (tr_ms * 1e-3) / 1e12
    log(f"timed {args.steps} steps in {dt:.3f} s; scoring {inf_ms:.1f} ms ({inf_tf:.0f} TFLOP/s), "
        f"training epoch {tr_ms:.1f} ms ({tr_tf:.0f} TFLOP/s); last loss {float(losses[-1].item()):.4f}")
    out = {"metric": "colourings scored/s (colour-invariant network, k-COL depth)",
           "value": p / (inf_ms * 1e-3), "unit": "colourings/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3 / max(args.steps, 1), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16+fp32", "data": "synthetic",
           "config": {"workload": "invnet", "graph": "G(n=500, p=0.5) seed 0", "k": k, "widths": widths,
                      "colourings": p, "batch": batch, "eval_chunk": chunk, "epochs": 1},
           "inference_ms": inf_ms, "train_epoch_ms": tr_ms,
           "train_pairs_per_s": p / (tr_ms * 1e-3),
           "roofline": {"bound": "mfma", "achieved": inf_tf, "peak": 2500.0, "unit": "TFLOP/s",
                        "frac": inf_tf / 2500.0, "traffic": None, "kernel": "whole evaluation pass",
                        "flops_per_colouring": inf_f / p, "train_achieved": tr_tf,
                        "train_frac": tr_tf / 2500.0, "train_flops_per_pair": tr_f / p}}
    print(json.dumps(out), flush=True)

def gemm_shapes(n, k, widths, chunk, batch):
    """Every product of the network's scoring chunk and training step:
    (name, a_kcontig, b_kcontig, M, N, K, calls per chunk or step)."""
    out, l_in = [], n
    for j, l_out in enumerate(widths[:-1]):
        # forward products read Lambda^T / Gamma^T: both operands K-contiguous
        out.append((f"score rows L{j}", True, True, chunk * k, l_out, l_in, 1))
        out.append((f"score mean L{j}", True, True, chunk, l_out, l_in, 1))
        out.append((f"train rows L{j}", True, True, batch * k, l_out, l_in, 1))
        out.append((f"train mean L{j}", True, True, batch, l_out, l_in, 1))
        out.append((f"train at L{j}", False, False, l_in, l_out, batch * k, 1))
        out.append((f"train at-mean L{j}", False, False, l_in, l_out, batch, 1))
        if j > 0:
            out.append((f"train wt L{j}", True, True, batch * k, l_in, l_out, 1))
            out.append((f"train wt-mean L{j}", True, True, batch, l_in, l_out, 1))
        l_in = l_out
    return out


def bench_gemm(args, w, dlm, torch):
    """The network's products alone (the paper-depth k-COL network for
    G(500, 0.5), k = 49: scoring chunks of --eval-chunk colourings, training
    batches of 100), each timed with dlm_gemm_bf16 (FP32 output) and, for
    context, with torch.mm on the same BF16 operands (the vendor BLAS, BF16
    output).  Reports TFLOP/s per product and flop-weighted totals for a
    scoring chunk and a training step."""
    g, k = w.graphs[0], w.k[0]
    from workloads.invnet_init import col_widths
    widths = col_widths(g.n)
    shapes = gemm_shapes(g.n, k, widths, args.eval_chunk, 100)
    gen = torch.Generator(device="cuda").manual_seed(5)
    reps = max(args.steps, 1)
    ws = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")  # split-K partials
    rows = []
    tot = {"score": [0.0, 0.0, 0.0], "train": [0.0, 0.0, 0.0]}
    for name, ak, bk, M, N, K, calls in shapes:
        A = torch.randn((M, K) if ak else (K, M), device="cuda", generator=gen).to(torch.bfloat16)
        B = torch.randn((N, K) if bk else (K, N), device="cuda", generator=gen).to(torch.bfloat16)
        C = torch.empty((M, N), dtype=torch.float32, device="cuda")
        At = A if ak else A.t()
        Bt = B.t() if bk else B
        def ours():
            dlm.gemm_bf16(A, B, M, N, K, ak, bk, out=C, workspace=ws)
        def lib():
            torch.mm(At, Bt)
        res = []
        for fn in (ours, lib):
            for _ in range(max(args.warmup, 1)):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            res.append(e0.elapsed_time(e1) / reps)
        fl = 2.0 * M * N * K * calls
        part = tot["score" if name.startswith("score") else "train"]
        part[0] += fl
        part[1] += res[0] * 1e-3
        part[2] += res[1] * 1e-3
        rows.append({"product": name, "M": M, "N": N, "K": K, "ms": res[0], "tflops": fl / res[0] / 1e9,
                     "torch_mm_ms": res[1], "torch_mm_tflops": fl / res[1] / 1e9})
        log(f"{name:>18s} {M:>6d} x {N:>5d} x {K:>6d}: {res[0]:8.3f} ms {fl / res[0] / 1e9:6.0f} TFLOP/s"
            f" | torch.mm {res[1]:8.3f} ms {fl / res[1] / 1e9:6.0f} TFLOP/s")
        del A, B, C
    summary = {kk: {"tflops": v[0] / v[1] / 1e12, "ms": v[1] * 1e3, "torch_mm_tflops": v[0] / v[2] / 1e12,
                    "torch_mm_ms": v[2] * 1e3} for kk, v in tot.items()}
    for kk, v in summary.items():
        log(f"{kk}: {v['ms']:.2f} ms, {v['tflops']:.0f} TFLOP/s (torch.mm {v['torch_mm_ms']:.2f} ms, "
            f"{v['torch_mm_tflops']:.0f} TFLOP/s)")
    tf = summary["train"]["tflops"]
    print(json.dumps({"metric": "BF16 MFMA product throughput (paper-depth network, training step)",
                      "value": tf, "unit": "TFLOP/s", "n_gpus": 1, "steps": reps, "warmup": args.warmup,
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+fp32",
                      "data": "synthetic",
                      "config": {"workload": "gemm", "widths": widths, "k": k, "eval_chunk": args.eval_chunk,
                                 "batch": 100},
                      "roofline": {"bound": "mfma", "achieved": tf, "peak": 2500.0, "unit": "TFLOP/s",
                                   "frac": tf / 2500.0, "traffic": None, "kernel": "gemm_bf16_kernel"},
                      "summary": summary, "products": rows}), flush=True)


def bench_predict(args, w, dlm, torch):
    """The paper's analysis of its network (Section 4.2) on the weighted
    G(300, 0.3) stand-in: the WVCP loop with the diversity steps (K = 32
    nearest neighbours, as the paper's WVCP setting), population 4096, 5
    training epochs per generation, run for a fixed number of generations
    with the per-class MLP, with the paper's colour-invariant network at its
    WVCP depth (hidden 5n, 2n, n, n // 2, batch 100), and plain (the second
    parent's child drawn at random among the K nearest: the ablation).  Each
    learned generation records the Pearson correlation between the kept
    offsprings' predicted and actual post-search scores and the median
    relative error of the predictions; every loop records its best legal
    weighted score per generation."""
    from paper_2109_05948_amd import memetic
    from workloads.invnet_init import invnet_weights, wvcp_widths
    from workloads.scorer_init import scorer_weights
    g = w.graphs[0]
    G = dlm.Graph.from_csr(g)
    pop = args.pop or w.pop
    seeds = [int(x) for x in args.seeds.split(",")]
    out = {}
    for net in ("mlp", "invariant", "plain"):
        if net == "invariant":
            params = invnet_weights(g.n, wvcp_widths(g.n), seed=0)
            params["widths"] = wvcp_widths(g.n)
            batch = 100
        else:
            params, batch = scorer_weights(g.n, seed=0), 1024
        runs = []
        for sd in seeds:
            log(f"predict: WVCP loop, {net}, seed {sd}")
            r = memetic.run(G, 0, pop, w.iters[0], learned=net != "plain", seed=sd, cutoff_s=args.cutoff,
                            max_generations=args.generations, scorer_params=params, batch=batch, epochs=5,
                            lr=1e-3, diversity=True, neighbours=32, weighted=True, rounds=w.extra["rounds"],
                            network="invariant" if net == "invariant" else "mlp")
            runs.append({"seed": sd, "generations": r.generations, "wall_s": r.wall,
                         "best_per_generation": [h[2] for h in r.history],
                         "predictions": [{"gen": gg, "pearson": pr, "median_rel_err_pct": re}
                                         for gg, pr, re in r.predictions]})
            log(f"  best per generation: {runs[-1]['best_per_generation']}")
            for gg, pr, re in r.predictions:
                log(f"  {net} seed {sd} gen {gg}: pearson {pr:.3f}, median relative error {re:.2f} %")
        out[net] = runs
    last = [x["predictions"][-1]["pearson"] for x in out["invariant"] if x["predictions"]]
    line = {"metric": "Pearson correlation of predicted and actual post-search scores (paper's network, "
                      "last generation, median over seeds)",
            "value": float(np.median(last)) if last else None, "unit": "r", "n_gpus": 1,
            "higher_is_better": True, "vs_baseline": None, "dtype": "bf16+fp32", "data": "synthetic",
            "config": {"workload": "predict", "graph": "G(n=300, p=0.3) seed 0, weights U{1..100}",
                       "population": pop, "neighbours": 32, "epochs": 5, "generations": args.generations,
                       "seeds": seeds},
            "loops": out}
    print(json.dumps(line), flush=True)

if __name__ == "__main__":
    main()
