"""The five named workload shapes (synthetic stand-ins for the paper's
DIMACS/COLOR instances), with every seed fixed.

* ``gnp100``   : plain TabuCol, G(100, 0.5), k=18, population 64, 10,000
  iterations, 32-bit gamma table.  Small enough for the oracle to run in
  full.
* ``gnp500``   : batched plain TabuCol at scale, G(500, 0.5), k=49,
  population 8192, 100,000 iterations, 16-bit gamma table in LDS.  Shape of
  DSJC500.5 (best known 47 colors in the paper's COL table).
* ``uneven64`` : 64 graphs of uneven size and density in one launch, half
  of them with a planted coloring; population 256 per graph.
* ``memetic1000`` : the memetic loop with the learned offspring scorer on
  G(1000, 0.5), k=85, population 8192.  Shape of DSJC1000.5.
* ``wvcp300``  : weighted coloring, G(300, 0.3), weights uniform on
  [1, 100], population 4096, 10 rounds of 10*n tabu iterations.
* ``wvcp500``  : weighted coloring, G(500, 0.5), weights uniform on
  [1, 100]: the graph of the population-size study.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .graphs import Graph, dsatur_colors, gnp, planted_partite, uniform_weights


@dataclass
class Workload:
    name: str
    graphs: list            # list[Graph]
    k: list                 # colors per graph
    pop: int                # individuals per graph
    iters: list             # tabu iterations per individual (per round for WVCP)
    init_seed: int = 1
    tabu_seed: int = 2
    ten_num: int = 6
    ten_den: int = 10
    ten_rand: int = 10
    extra: dict = field(default_factory=dict)


def _gnp100() -> Workload:
    g = gnp(100, 0.5, seed=0)
    return Workload("gnp100", [g], [18], 64, [10_000], extra={"wide_gamma": True})


def _gnp500() -> Workload:
    g = gnp(500, 0.5, seed=0)
    return Workload("gnp500", [g], [49], 8192, [100_000],
                    extra={"sample_stride": 128})


def _uneven64(seed: int = 0) -> Workload:
    rng = np.random.default_rng(seed)
    graphs, ks, iters, hidden = [], [], [], []
    for gi in range(64):
        n = int(rng.integers(100, 1001))
        p = float(rng.uniform(0.1, 0.9))
        gseed = int(rng.integers(0, 2**31 - 1))
        if gi % 2 == 0:
            g = gnp(n, p, seed=gseed)
            k = max(2, int(dsatur_colors(g).max()) + 1 - 2)
            hidden.append(None)
        else:
            hk = int(rng.integers(5, 61))
            g, _ = planted_partite(n, hk, 0.5, seed=gseed)
            k = hk
            hidden.append(hk)
        graphs.append(g)
        ks.append(k)
        iters.append(128 * n)
    return Workload("uneven64", graphs, ks, 256, iters, extra={"hidden_k": hidden})


def _memetic1000() -> Workload:
    g = gnp(1000, 0.5, seed=0)
    return Workload("memetic1000", [g], [85], 8192, [128 * 1000],
                    extra={"children_per_pair": 4, "keep_frac": 0.25,
                           "h1": 256, "h2": 128, "h3": 64, "lr": 1e-3,
                           "batch": 1024, "epochs": 5})


def _wvcp300() -> Workload:
    g = gnp(300, 0.3, seed=0)
    w = uniform_weights(300, 1, 100, seed=7)
    g = g.with_weights(w)
    return Workload("wvcp300", [g], [60], 4096, [10 * 300],
                    ten_num=2, ten_den=10, extra={"rounds": 10, "k_cap": 60})


def _wvcp500() -> Workload:
    # stand-in for the paper's DSJC500.5 weighted-colouring study of the
    # population size: G(500, 0.5), weights uniform on [1, 100]
    g = gnp(500, 0.5, seed=0)
    w = uniform_weights(500, 1, 100, seed=7)
    g = g.with_weights(w)
    return Workload("wvcp500", [g], [0], 4096, [10 * 500],
                    ten_num=2, ten_den=10, extra={"rounds": 10})


WORKLOADS = {
    "gnp100": _gnp100,
    "gnp500": _gnp500,
    "uneven64": _uneven64,
    "memetic1000": _memetic1000,
    "wvcp300": _wvcp300,
    "wvcp500": _wvcp500,
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]()
