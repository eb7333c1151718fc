"""Plain reference of the population's diversity machinery.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may import this module; the product path never
does.  It shares no code with the HIP kernels.

Three steps of a memetic generation (Sections 2.4 to 2.6 of the paper):

* the set-theoretic partition distance D(A, B) between two k-colourings: the
  fewest vertices to move between the classes of A to obtain the partition
  of B (Section 2.4).  Its exact value is n minus a maximum-weight matching
  on the k x k class-overlap matrix; the paper uses an approximation of
  linear cost instead, which is taken here as follows (the paper does not
  spell it out):
    M[i][j] = |A_i & B_j|;
    one greedy pass takes the classes of A by decreasing size (ties by
    class index) and gives each the free class j of B with the largest
    M[i][j] (ties by smaller j), leaving it unmatched when that overlap is
    0; a second pass does the same with the roles of A and B swapped;
    D~(A, B) = n - (the larger of the two matched totals).
  Both passes build matchings, so D~ >= D, and D~ is symmetric.  D~ = D
  for close partitions: when every non-empty class of A shares more than
  half of itself with a class of B that shares more than half of itself
  with it, those pairs are the row maxima of M, they form a matching (so
  it is a maximum one), and the pass over A takes exactly them.
* the distance-and-quality population update (Section 2.5): the pool of
  old and new individuals, best score first (ties by pool index), is taken
  greedily; an individual joins when its distance to every one already
  taken exceeds the spacing |V| / 10.  When the pool runs out before the
  population is full (the paper does not say what happens then), the best
  of the individuals left out fill the remaining places.
* K-nearest-neighbour parent matching (Section 2.6): the K individuals
  closest to each one (ties by index), itself excluded; each individual's K
  GPX children (one per neighbour) then yield one offspring: the child with
  the smallest predicted score (eq. select_cross), or for the plain loop a
  uniformly drawn one.
"""
from __future__ import annotations

import numpy as np

from . import philox, uniform

D_SELGROUP = 0x8000000A  # Philox domain of the plain loop's draw within a group


def overlap(a: np.ndarray, b: np.ndarray, k: int) -> np.ndarray:
    """M[i][j] = number of vertices with colour i in a and colour j in b."""
    m = np.zeros((k, k), dtype=np.int64)
    np.add.at(m, (np.asarray(a, np.int64), np.asarray(b, np.int64)), 1)
    return m


def class_order(a: np.ndarray, k: int) -> list[int]:
    """Classes of a by decreasing size, ties by class index."""
    sizes = np.bincount(np.asarray(a, np.int64), minlength=k)
    return sorted(range(k), key=lambda c: (-int(sizes[c]), c))


def greedy_match(m: np.ndarray, order: list[int]) -> int:
    """Rows of m in the given order each take their largest free column
    (ties by smaller column); a row whose largest free entry is 0 takes
    none.  Returns the matched total."""
    k = m.shape[1]
    taken = [False] * k
    total = 0
    for i in order:
        best, bj = 0, -1
        for j in range(k):
            if not taken[j] and m[i][j] > best:
                best, bj = int(m[i][j]), j
        if bj >= 0:
            taken[bj] = True
            total += best
    return total


def approx_distance(a: np.ndarray, b: np.ndarray, k: int) -> int:
    """D~(a, b) of Section 2.4, in the reading stated in the module header."""
    a = np.asarray(a)
    b = np.asarray(b)
    m = overlap(a, b, k)
    s_ab = greedy_match(m, class_order(a, k))
    s_ba = greedy_match(m.T, class_order(b, k))
    return int(a.shape[0]) - max(s_ab, s_ba)


def distance_matrix(rows_a: np.ndarray, rows_b: np.ndarray, k: int) -> np.ndarray:
    """D~ of every pair (row of rows_a, row of rows_b)."""
    out = np.zeros((rows_a.shape[0], rows_b.shape[0]), dtype=np.int32)
    for i in range(rows_a.shape[0]):
        for j in range(rows_b.shape[0]):
            out[i, j] = approx_distance(rows_a[i], rows_b[j], k)
    return out


def spacing_update(f: np.ndarray, dist: np.ndarray, keep: int, min_spacing: int) -> tuple[list[int], int]:
    """Section 2.5.  f: the scores of the pool (lower is better), dist: its
    pairwise distances.  Returns the indices taken, in the order taken, and
    how many of them were taken under the spacing rule (the rest fill)."""
    order = sorted(range(len(f)), key=lambda i: (int(f[i]), i))
    taken: list[int] = []
    for c in order:
        if len(taken) == keep:
            break
        if all(int(dist[c][s]) > min_spacing for s in taken):
            taken.append(c)
    spaced = len(taken)
    chosen = set(taken)
    for c in order:
        if len(taken) == keep:
            break
        if c not in chosen:
            taken.append(c)
            chosen.add(c)
    return taken, spaced


def nearest(dist: np.ndarray, K: int) -> np.ndarray:
    """Section 2.6: for every i, the K indices j != i with the smallest
    dist[i][j], nearest first, ties by smaller j."""
    p = dist.shape[0]
    out = np.zeros((p, K), dtype=np.int32)
    for i in range(p):
        cand = sorted((int(dist[i][j]), j) for j in range(p) if j != i)
        out[i] = [j for _, j in cand[:K]]
    return out


def select_groups(scores: np.ndarray | None, groups: int, K: int, mode: str, seed: int = 0,
                  gen: int = 0) -> np.ndarray:
    """One child per group of K consecutive children (group g = children
    gK .. gK + K - 1).  "top": the smallest FP32 score, ties by smaller
    index.  "random": child gK + floor(w0 K / 2^32), w0 = word 0 of
    Philox(seed; g, gen, 0, D_SELGROUP)."""
    out = np.zeros(groups, dtype=np.int32)
    for g in range(groups):
        if mode == "top":
            s = np.asarray(scores[g * K:(g + 1) * K], dtype=np.float32)
            best = 0
            for j in range(1, K):
                if s[j] < s[best]:
                    best = j
            out[g] = g * K + best
        else:
            out[g] = g * K + uniform(philox(g, gen, 0, D_SELGROUP, seed)[0], K)
    return out
