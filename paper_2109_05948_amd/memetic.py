"""Memetic loop (Algorithm 1) on the device, plain and learned.

One generation:
  1. pair every individual i with a uniform other member (it is the first
     parent, the crossover being asymmetric, Section 2.6);
  2. GPX: ``children_per_pair`` children per pair;
  3. selection (eq. select_cross, population-wide): learned = the offspring
     with the smallest predicted post-search score; plain = a random subset
     of the same size;
  4. TabuCol on the selected offspring (their start colourings S^O kept);
  5. learned only: train the scorer on (S^O, standardised f(S')) (Section 2.3);
  6. (mu + lambda) update: the best ``pop`` of parents and improved offspring.
With ``diversity=True`` steps 1, 3 and 6 follow Sections 2.4 to 2.6 instead:
  1. every individual is paired with its ``neighbours`` nearest members by
     the approximate partition distance, one GPX child per pair;
  3. one child per individual: learned = the smallest predicted score of
     its group (eq. select_cross), plain = a random one of the group;
  6. the distances of the new offspring to the population and to each
     other go into the pool matrix, and the spacing update (quality order,
     distance > |V| / 10) builds the next population and its distances.
The loop stops at the first legal colouring (f = 0) or at the time limit.
Every step is a call into libdlmcol; only the best score crosses to the host
each generation.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

from . import _abi as A

SEED_TABU = 0x7ab0
SEED_PAIR = 0x9a17
SEED_GPX = 0x69c5
SEED_SEL = 0x5e1e


@dataclass
class MemeticResult:
    learned: bool
    best: int
    generations: int
    time_to_legal: float | None
    wall: float
    history: list = field(default_factory=list)  # (seconds, generation, best f, mean f)
    tabu_moves: int = 0
    scorer_loss: list = field(default_factory=list)
    colors: object = None  # final population (device int16 [pop, n]) and its scores
    f: object = None


def run(graph: A.Graph, k: int, pop: int, iters: int, learned: bool, seed: int = 0,
        cutoff_s: float = 600.0, max_generations: int = 1 << 30, children_per_pair: int = 4,
        keep_frac: float = 0.25, scorer_params: dict | None = None, batch: int = 1024,
        epochs: int = 5, lr: float = 1e-3, block: int = 0, table: str = "auto",
        log=None, diversity: bool = False, neighbours: int = 16) -> MemeticResult:
    dev = torch.device("cuda", torch.cuda.current_device())
    if diversity:
        children_per_pair, keep_frac = neighbours, 1.0 / neighbours
        if not 1 <= neighbours < pop:
            raise ValueError("neighbours must lie in [1, pop)")
    nchild = pop * children_per_pair
    nsel = int(round(nchild * keep_frac))
    if nsel != pop:
        raise ValueError("this loop keeps the population size: children_per_pair * keep_frac must be 1")
    if learned and scorer_params is None:
        raise ValueError("the learned loop needs initial scorer parameters")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cols, _ = A.init_population(graph, k, pop, seed=seed)
    r = A.tabu_batch(graph, cols, k, iters, seed ^ SEED_TABU, ind_base=0, block=block, table=table)
    f = r["f_best"].clone()
    moves = int(r["stats"][:, 0].sum().item())
    best = int(f.min().item())
    res = MemeticResult(learned, best, 0, None, 0.0)
    now = time.perf_counter() - t0
    res.history.append((now, 0, best, float(f.float().mean().item())))
    if best == 0:
        res.time_to_legal = now
    sc = A.Scorer(graph.n, k, scorer_params, max_batch=batch) if learned else None
    off = torch.empty((nsel, graph.n), dtype=torch.int16, device=dev)
    start = torch.empty_like(off)
    if diversity:
        # pool distances: old members 0..pop-1, offspring pop..2pop-1 (upper triangle used)
        pools = [torch.zeros((2 * pop, 2 * pop), dtype=torch.int32, device=dev) for _ in range(2)]
        A.partition_distance(cols, k, out=pools[0][:pop, :pop])
        first = torch.arange(pop, dtype=torch.int32, device=dev).repeat_interleave(neighbours)
    ind_next = pop
    gen = 0
    while best > 0 and gen < max_generations and time.perf_counter() - t0 < cutoff_s:
        gen += 1
        if diversity:
            nn = A.nearest(pools[0], neighbours, p=pop)
            pairs = torch.stack((first, nn.reshape(-1)), 1).contiguous()
        else:
            pairs = A.random_pairs(pop, seed ^ SEED_PAIR, gen)
        children = A.gpx_batch(graph, k, cols, pairs, 1 if diversity else children_per_pair, seed ^ SEED_GPX,
                               child_base=gen * nchild)
        if diversity and learned:
            idx = A.select_groups(sc.score(children), pop, neighbours, "top")
        elif diversity:
            idx = A.select_groups(None, pop, neighbours, "random", seed=seed ^ SEED_SEL, gen=gen)
        elif learned:
            scores = sc.score(children)
            idx = A.select(scores, nchild, nsel, "top")
        else:
            idx = A.select(None, nchild, nsel, "random", seed=seed ^ SEED_SEL, gen=gen)
        A.gather_rows(children, idx, out=off)
        A.gather_rows(children, idx, out=start)
        r = A.tabu_batch(graph, off, k, iters, seed ^ SEED_TABU, ind_base=ind_next, block=block,
                         table=table)
        ind_next += nsel
        if learned:
            tgt = A.standardize(r["f_best"])
            loss = sc.train(start, tgt, batch=batch, epochs=epochs, lr=lr)
            res.scorer_loss.append(float(loss[-1].item()))
        if diversity:
            pool, nxt = pools
            A.partition_distance(cols, k, off, out=pool[:pop, pop:])
            A.partition_distance(off, k, out=pool[pop:, pop:], upper_only=True)
            pick, _ = A.spacing_update(f, r["f_best"], pool, pop, graph.n // 10)
            A.gather_distances(pool, pick, out=nxt[:pop, :pop])
            cols, f = A.gather_pool(cols, f, off, r["f_best"], pick)
            pools = [nxt, pool]
        else:
            cols, f = A.pop_update(cols, f, off, r["f_best"])
        moves += int(r["stats"][:, 0].sum().item())
        best = int(f.min().item())
        now = time.perf_counter() - t0
        res.history.append((now, gen, best, float(f.float().mean().item())))
        if log:
            log(f"[{'learned' if learned else 'plain'}] gen {gen} t={now:.1f}s best={best} "
                f"mean={res.history[-1][3]:.2f}")
        if best == 0:
            res.time_to_legal = now
    torch.cuda.synchronize()
    res.best, res.generations, res.tabu_moves = best, gen, moves
    res.colors, res.f = cols, f
    res.wall = time.perf_counter() - t0
    return res
