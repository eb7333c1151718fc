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
    scorer_params: dict | None = None  # the learned loop's scorer at the end
    # learned loop, per generation: (generation, Pearson r, median relative
    # error in %) of the kept offsprings' predicted against actual scores
    predictions: list = field(default_factory=list)


def prediction_quality(pred: torch.Tensor, actual: torch.Tensor, mean: float, sd: float) -> tuple:
    """The quality measures of the paper's analysis of its network: the
    Pearson correlation between the predictions and the scores the local
    search then reached, and the median relative error of the predictions
    in score units (the network predicts standardised scores; ``mean`` and
    ``sd`` are those of its last training targets).  Individuals without a
    finite score (WVCP: no legal colouring) are left out."""
    a = actual.double()
    p = pred.double()
    ok = a < 0x7FFFFFFF
    a, p = a[ok], p[ok]
    if a.numel() < 2 or float(a.std()) == 0.0 or float(p.std()) == 0.0:
        return float("nan"), float("nan")
    r = float(torch.corrcoef(torch.stack((p, a)))[0, 1])
    rel = float(((mean + sd * p - a).abs() / a.clamp(min=1.0)).median()) * 100.0
    return r, rel


def wvcp_targets(f: torch.Tensor):
    """Training scores of a WVCP generation (dlm_wvcp_targets): a search that
    met no legal colouring (score 0x7fffffff) gets the generation's worst
    legal score; None when no search met one."""
    t, any_legal = A.wvcp_targets(f)
    return t if int(any_legal.item()) else None


def _score_scale(f: torch.Tensor) -> tuple:
    """Mean and population standard deviation, as dlm_standardize takes them."""
    d = f.double()
    return float(d.mean()), float(d.std(unbiased=False))


def run(graph: A.Graph, k: int, pop: int, iters: int, learned: bool, seed: int = 0,
        cutoff_s: float = 600.0, max_generations: int = 1 << 30, children_per_pair: int = 4,
        keep_frac: float = 0.25, scorer_params: dict | None = None, batch: int = 1024,
        epochs: int = 5, lr: float = 1e-3, block: int = 0, table: str = "auto",
        log=None, diversity: bool = False, neighbours: int = 16,
        init_colors: torch.Tensor | None = None, weighted: bool = False, rounds: int = 10,
        target: int | None = None, network: str = "mlp", eval_chunk: int = 1024,
        slice_rows: int = 0) -> MemeticResult:
    """One loop of Algorithm 1.  With ``weighted`` it solves the WVCP
    (Section 2.2): the start is the greedy colouring (k = 0 takes the largest
    number of colours it uses), the local search is Algorithm 2 with
    ``iters`` iterations per round over ``rounds`` rounds, and an
    individual's score is its best legal weighted score.  The loop stops when
    the best score reaches ``target`` (default 0 for k-COL, none for WVCP),
    at ``max_generations`` or at the cutoff; ``time_to_legal`` is then the
    time the target was reached.

    ``network`` picks the learned loop's scorer: "mlp" is the per-class MLP
    with sum pooling (dlm_scorer, ``scorer_params`` its packed weights);
    "invariant" is the paper's colour-invariant network of Section 2.3
    (dlm_invnet, ``scorer_params`` its weights with a "widths" entry),
    trained at ``batch`` colourings per step and evaluated in chunks of
    ``eval_chunk``.

    ``slice_rows`` > 0 runs each local-search pass in launches of at most
    that many individuals, logging each; every individual keeps its own
    random stream (``ind_base``), so the results do not change."""
    dev = torch.device("cuda", torch.cuda.current_device())
    if target is None:
        target = -1 if weighted else 0
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
    if network not in ("mlp", "invariant"):
        raise ValueError(f"unknown network {network!r}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if init_colors is not None:
        if tuple(init_colors.shape) != (pop, graph.n):
            raise ValueError(f"init_colors must be [{pop}, {graph.n}]")
        cols = init_colors.clone()
    elif weighted:
        cols, k_used = A.init_population(graph, k, pop, seed=seed, mode="greedy")
        k = k or int(k_used.max().item())
    else:
        cols, _ = A.init_population(graph, k, pop, seed=seed)

    def search(colors, ind_base):  # the local search, in place; returns (scores, moves)
        rows = colors.shape[0]
        step = slice_rows if 0 < slice_rows < rows else max(rows, 1)
        scores, moves = [], 0
        for r0 in range(0, rows, step):
            part = colors[r0:r0 + step]
            if weighted:
                o = A.wvcp_batch(graph, part, k, iters, rounds, seed ^ SEED_TABU, ind_base=ind_base + r0,
                                 block=block)
                scores.append(o["best_legal"])
            else:
                o = A.tabu_batch(graph, part, k, iters, seed ^ SEED_TABU, ind_base=ind_base + r0, block=block,
                                 table=table)
                scores.append(o["f_best"])
            moves += int(o["stats"][:, 0].sum().item())
            if step < rows and log:
                log(f"  local search of individuals {ind_base + r0}..{ind_base + r0 + part.shape[0] - 1} done")
        return (scores[0] if len(scores) == 1 else torch.cat(scores)), moves

    f, moves = search(cols, 0)
    f = f.clone()
    best = int(f.min().item())
    res = MemeticResult(learned, best, 0, None, 0.0)
    now = time.perf_counter() - t0
    res.history.append((now, 0, best, float(f.float().mean().item())))
    if best <= target:
        res.time_to_legal = now
    sc = None
    if learned and network == "mlp":
        sc = A.Scorer(graph.n, k, scorer_params, max_batch=batch)
    elif learned:
        sc = A.InvNet(graph.n, k, scorer_params["widths"], scorer_params, max_batch=max(batch, eval_chunk))
    off = torch.empty((nsel, graph.n), dtype=torch.int16, device=dev)
    start = torch.empty_like(off)
    if diversity:
        # pool distances: old members 0..pop-1, offspring pop..2pop-1 (upper triangle used)
        pools = [torch.zeros((2 * pop, 2 * pop), dtype=torch.int32, device=dev) for _ in range(2)]
        A.partition_distance(cols, k, out=pools[0][:pop, :pop])
        first = torch.arange(pop, dtype=torch.int32, device=dev).repeat_interleave(neighbours)
    ind_next = pop
    gen = 0
    scale = _score_scale(f)  # what the untrained network's outputs are read against
    while best > target and gen < max_generations and time.perf_counter() - t0 < cutoff_s:
        gen += 1
        if diversity:
            nn = A.nearest(pools[0], neighbours, p=pop)
            pairs = torch.stack((first, nn.reshape(-1)), 1).contiguous()
        else:
            pairs = A.random_pairs(pop, seed ^ SEED_PAIR, gen)
        children = A.gpx_batch(graph, k, cols, pairs, 1 if diversity else children_per_pair, seed ^ SEED_GPX,
                               child_base=gen * nchild)
        if diversity and learned:
            scores = sc.score(children)
            idx = A.select_groups(scores, pop, neighbours, "top")
        elif diversity:
            idx = A.select_groups(None, pop, neighbours, "random", seed=seed ^ SEED_SEL, gen=gen)
        elif learned:
            scores = sc.score(children)
            idx = A.select(scores, nchild, nsel, "top")
        else:
            idx = A.select(None, nchild, nsel, "random", seed=seed ^ SEED_SEL, gen=gen)
        A.gather_rows(children, idx, out=off)
        A.gather_rows(children, idx, out=start)
        f_off, gen_moves = search(off, ind_next)
        ind_next += nsel
        if learned:
            res.predictions.append((gen,) + prediction_quality(scores[idx.long()], f_off, *scale))
            f_t = wvcp_targets(f_off) if weighted else f_off
            if f_t is not None:
                scale = _score_scale(f_t)
                loss = sc.train(start, A.standardize(f_t), batch=batch, epochs=epochs, lr=lr)
                res.scorer_loss.append(float(loss[-1].item()))
            else:
                res.scorer_loss.append(float("nan"))
        if diversity:
            pool, nxt = pools
            A.partition_distance(cols, k, off, out=pool[:pop, pop:])
            A.partition_distance(off, k, out=pool[pop:, pop:], upper_only=True)
            pick, _ = A.spacing_update(f, f_off, pool, pop, graph.n // 10)
            A.gather_distances(pool, pick, out=nxt[:pop, :pop])
            cols, f = A.gather_pool(cols, f, off, f_off, pick)
            pools = [nxt, pool]
        else:
            cols, f = A.pop_update(cols, f, off, f_off)
        moves += gen_moves
        best = int(f.min().item())
        now = time.perf_counter() - t0
        res.history.append((now, gen, best, float(f.float().mean().item())))
        if log:
            log(f"[{'learned' if learned else 'plain'}] gen {gen} t={now:.1f}s best={best} "
                f"mean={res.history[-1][3]:.2f}")
        if best <= target:
            res.time_to_legal = now
    torch.cuda.synchronize()
    res.best, res.generations, res.tabu_moves = best, gen, moves
    res.colors, res.f = cols, f
    if sc is not None:
        res.scorer_params = sc.params()
        if network == "invariant":
            res.scorer_params["widths"] = list(scorer_params["widths"])
    res.wall = time.perf_counter() - t0
    return res


@dataclass
class DecreasingResult:
    best_k: int | None
    found: list  # (k, seconds from the start) of every legal k-colouring, in order
    legal: dict  # k -> a legal k-colouring (host int16 [n])
    wall: float
    runs: list = field(default_factory=list)  # the MemeticResult of each k


def decreasing_k(graph: A.Graph, k: int, pop: int, iters: int, learned: bool, seed: int = 0,
                 cutoff_s: float = 600.0, scorer_params: dict | None = None, log=None,
                 **kw) -> DecreasingResult:
    """COL as a series of k-COL problems (Section 2.7): once a legal
    k-colouring is found, k drops by one and the search continues from the
    same population, moved to k - 1 colours by dissolving each individual's
    smallest class (dlm_reduce_colours); the learned loop keeps its scorer
    (fresh Adam moments).  Stops when a k is not solved within the overall
    cutoff; the last k solved bounds the chromatic number from above."""
    t0 = time.perf_counter()
    res = DecreasingResult(None, [], {}, 0.0)
    cols, params, step = None, scorer_params, 0
    while k >= 2:
        start = time.perf_counter() - t0
        left = cutoff_s - start
        if left <= 0:
            break
        r = run(graph, k, pop, iters, learned, seed=seed + step, cutoff_s=left, scorer_params=params,
                init_colors=cols, log=log, **kw)
        res.runs.append(r)
        if r.time_to_legal is None:
            break
        res.found.append((k, start + r.time_to_legal))
        i = int(torch.argmin(r.f).item())
        res.legal[k] = r.colors[i].cpu().numpy()
        res.best_k = k
        if log:
            log(f"[decreasing] legal {k}-colouring at {res.found[-1][1]:.1f} s")
        cols = A.reduce_colours(r.colors, k, seed, step=k - 1)
        params = r.scorer_params if learned else params
        k -= 1
        step += 1
    torch.cuda.synchronize()
    res.wall = time.perf_counter() - t0
    return res
