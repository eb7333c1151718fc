"""Seeded graph and weight generators, stored as CSR.

The instances the paper measures on (DIMACS/COLOR files) are not
available, so every workload is synthetic:

* ``gnp``: Erdos-Renyi G(n, p), the shape of the DSJCn.p family used in
  the paper's vertex-coloring experiments (Section 3, tables of difficult
  and easy DIMACS instances).
* ``planted_partite``: a graph with a hidden legal k-coloring (edges only
  between different hidden parts), the shape of the flat/le450 families
  whose chromatic number is known by construction.
* ``uniform_weights``: integer vertex weights for the weighted problem
  (WVCP), uniform on [lo, hi].

Randomness comes from numpy's PCG64 seeded generator, so a (seed, shape)
pair always gives the same graph.  Nothing here depends on the coloring
method.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Graph:
    """Undirected simple graph in CSR form (both directions stored).

    ``row_ptr``: int32[n+1]; ``col_idx``: int32[2m], each row sorted
    ascending, no self loops, symmetric.  ``weights`` is int32[n] or None.
    """

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    weights: np.ndarray | None = None
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col_idx.shape[0] // 2)

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int32)

    @property
    def max_deg(self) -> int:
        return int(self.degrees.max()) if self.n else 0

    def neighbors(self, v: int) -> np.ndarray:
        return self.col_idx[self.row_ptr[v]:self.row_ptr[v + 1]]

    def edges(self) -> np.ndarray:
        """int32[m, 2] array of (u, v) with u < v."""
        src = np.repeat(np.arange(self.n, dtype=np.int32), self.degrees)
        keep = src < self.col_idx
        return np.stack([src[keep], self.col_idx[keep]], axis=1)

    def with_weights(self, weights: np.ndarray) -> "Graph":
        w = np.ascontiguousarray(weights, dtype=np.int32)
        assert w.shape == (self.n,)
        return Graph(self.n, self.row_ptr, self.col_idx, w, self.name)


def from_edges(n: int, edges: np.ndarray, name: str = "") -> Graph:
    """Build a CSR graph from an (m, 2) array of undirected edges."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size:
        if (e < 0).any() or (e >= n).any():
            raise ValueError("edge endpoint out of range")
        e = e[e[:, 0] != e[:, 1]]
        lo = np.minimum(e[:, 0], e[:, 1])
        hi = np.maximum(e[:, 0], e[:, 1])
        key = np.unique(lo * n + hi)
        lo, hi = key // n, key % n
        src = np.concatenate([lo, hi])
        dst = np.concatenate([hi, lo])
    else:
        src = dst = np.zeros(0, dtype=np.int64)
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return Graph(n, row_ptr.astype(np.int32), dst.astype(np.int32), None, name)


def gnp(n: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi G(n, p): each of the n(n-1)/2 pairs is an edge with prob. p."""
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.shape[0]) < p
    return from_edges(n, np.stack([iu[keep], ju[keep]], axis=1),
                      name=f"gnp(n={n},p={p},seed={seed})")


def planted_partite(n: int, hidden_k: int, p_cross: float, seed: int) -> tuple[Graph, np.ndarray]:
    """Random graph with a planted legal ``hidden_k``-coloring.

    Each vertex gets a uniform hidden part in [0, hidden_k); each pair in
    different parts is an edge with probability ``p_cross``; pairs in the
    same part never are.  Returns (graph, parts).
    """
    rng = np.random.default_rng(seed)
    parts = rng.integers(0, hidden_k, size=n).astype(np.int32)
    iu, ju = np.triu_indices(n, k=1)
    keep = (rng.random(iu.shape[0]) < p_cross) & (parts[iu] != parts[ju])
    g = from_edges(n, np.stack([iu[keep], ju[keep]], axis=1),
                   name=f"planted(n={n},hk={hidden_k},p={p_cross},seed={seed})")
    return g, parts


def uniform_weights(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """int32 weights uniform on the integers [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=n).astype(np.int32)


def is_valid_csr(g: Graph) -> bool:
    """Symmetric, per-row strictly ascending, in range, no self loops."""
    n = g.n
    rp, ci = g.row_ptr, g.col_idx
    if rp.shape != (n + 1,) or rp[0] != 0 or rp[-1] != ci.shape[0]:
        return False
    if (np.diff(rp) < 0).any():
        return False
    if ci.size and ((ci < 0).any() or (ci >= n).any()):
        return False
    src = np.repeat(np.arange(n), np.diff(rp))
    if (src == ci).any():
        return False
    for v in range(n):
        row = ci[rp[v]:rp[v + 1]]
        if row.size > 1 and (np.diff(row) <= 0).any():
            return False
    fwd = set(zip(src.tolist(), ci.tolist()))
    return all((b, a) in fwd for a, b in fwd)


def dsatur_colors(g: Graph) -> np.ndarray:
    """Brelaz DSATUR greedy coloring, used only to pick a color budget k.

    Next vertex: max saturation, then max degree, then lowest index; it
    takes the smallest color not used by its colored neighbours.
    """
    n = g.n
    deg = g.degrees.astype(np.int64)
    color = np.full(n, -1, dtype=np.int64)
    # seen[v, c] = 1 if some coloured neighbour of v has colour c
    seen = np.zeros((n, n + 1), dtype=bool)
    sat = np.zeros(n, dtype=np.int64)
    for _ in range(n):
        cand = np.where(color < 0)[0]
        key = sat[cand] * (n + 1) * 2 + deg[cand]
        best = cand[key == key.max()].min()
        c = int(np.argmin(seen[best]))
        color[best] = c
        nb = g.neighbors(best)
        newly = nb[~seen[nb, c]]
        seen[newly, c] = True
        sat[newly] += 1
    return color.astype(np.int32)
