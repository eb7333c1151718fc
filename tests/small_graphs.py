"""Small named graphs with known colouring facts, for pins."""
from __future__ import annotations

import itertools

import numpy as np

from workloads.graphs import from_edges, gnp


def complete(n):
    return from_edges(n, np.array(list(itertools.combinations(range(n), 2)) or
                                  np.zeros((0, 2), int)), name=f"K{n}")


def cycle(n):
    return from_edges(n, np.array([(i, (i + 1) % n) for i in range(n)]), name=f"C{n}")


def grid(a, b):
    e = []
    for i in range(a):
        for j in range(b):
            v = i * b + j
            if j + 1 < b:
                e.append((v, v + 1))
            if i + 1 < a:
                e.append((v, v + b))
    return from_edges(a * b, np.array(e), name=f"grid{a}x{b}")


def complete_bipartite(a, b):
    return from_edges(a + b, np.array([(i, a + j) for i in range(a) for j in range(b)]),
                      name=f"K{a},{b}")


def edgeless(n):
    return from_edges(n, np.zeros((0, 2), dtype=np.int64), name=f"E{n}")


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return from_edges(10, np.array(outer + spokes + inner), name="petersen")


def random_tiny(seed, n=None, p=None):
    rng = np.random.default_rng(seed)
    n = n or int(rng.integers(4, 11))
    p = p if p is not None else float(rng.uniform(0.2, 0.8))
    return gnp(n, p, seed=int(rng.integers(0, 2**31)))


def kn_min_conflicts(n, k):
    """Closed form: balanced split of K_n into k classes; n = q k + r."""
    q, r = divmod(n, k)
    return r * (q + 1) * q // 2 + (k - r) * q * (q - 1) // 2
