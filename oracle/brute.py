"""Exhaustive solvers for tiny graphs, used only as pins for the oracle.

TEST INFRASTRUCTURE ONLY.

* ``chromatic_number``: smallest k admitting a legal k-colouring
  (backtracking), the quantity the COL problem minimises (Section 1).
* ``min_conflicts``: min over all k^n colourings of eq. (f) (Section 2.7).
* ``wvcp_opt``: min over all legal colourings of eq. (score_WVCP)
  (Section 1), by enumerating set partitions as restricted growth strings.
"""
from __future__ import annotations

import itertools

import numpy as np


def _adj(g) -> list[set]:
    return [set(g.neighbors(v).tolist()) for v in range(g.n)]


def _colorable(adj, n, k) -> bool:
    col = [-1] * n
    order = sorted(range(n), key=lambda v: -len(adj[v]))

    def rec(i):
        if i == n:
            return True
        v = order[i]
        used = {col[u] for u in adj[v] if col[u] >= 0}
        top = max(col) + 1  # symmetry breaking: at most one fresh colour
        for c in range(min(k, top + 1)):
            if c in used:
                continue
            col[v] = c
            if rec(i + 1):
                return True
            col[v] = -1
        return False

    return rec(0)


def chromatic_number(g) -> int:
    if g.n == 0:
        return 0
    adj = _adj(g)
    for k in range(1, g.n + 1):
        if _colorable(adj, g.n, k):
            return k
    return g.n


def min_conflicts(g, k: int) -> int:
    """Minimum number of monochromatic edges over all k-colourings (n <= 10)."""
    n = g.n
    assert n <= 10 and k ** n <= 2 ** 22
    e = g.edges()
    if e.shape[0] == 0:
        return 0
    # all colourings as rows of base-k digits
    idx = np.arange(k ** n, dtype=np.int64)
    digits = np.stack([(idx // k ** i) % k for i in range(n)], axis=1)
    f = (digits[:, e[:, 0]] == digits[:, e[:, 1]]).sum(axis=1)
    return int(f.min())


def _partitions(n):
    """Restricted growth strings: every set partition of range(n) once."""
    if n == 0:
        yield []
        return
    a = [0] * n

    def rec(i, mx):
        if i == n:
            yield list(a)
            return
        for c in range(mx + 2):
            a[i] = c
            yield from rec(i + 1, max(mx, c))

    a[0] = 0
    yield from rec(1, 0)


def wvcp_opt(g, weights) -> int:
    """Minimum of sum over classes of max weight, over legal colourings (n <= 8)."""
    n = g.n
    assert n <= 9
    w = list(int(x) for x in weights)
    e = g.edges().tolist()
    best = None
    for p in _partitions(n):
        if any(p[u] == p[v] for u, v in e):
            continue
        mx = {}
        for v, c in enumerate(p):
            mx[c] = max(mx.get(c, 0), w[v])
        s = sum(mx.values())
        if best is None or s < best:
            best = s
    return int(best)


def all_colorings(n: int, k: int):
    return itertools.product(range(k), repeat=n)
