"""Pins for oracle parts that other tests used only one-sidedly: the random
parent pairing of the simplified generation, the brute-force minimum
conflict count (checked against closed forms), and the vertex order of the
randomized greedy WVCP start (Section 2.1), on hand-made graphs whose
colourings are forced once the order is fixed."""
import numpy as np
import pytest

import oracle
from oracle import brute
from small_graphs import complete, complete_bipartite, cycle, edgeless, kn_min_conflicts, petersen
from workloads.graphs import from_edges

D_PAIRS = 0x80000009


# ---------------------------------------------------------------------------
# random parent pairing: (i, j), j uniform over the other members
def test_random_pairs_structure_and_uniformity():
    pop = 9
    pairs = oracle.random_pairs(pop, seed=11, gen=2)
    assert pairs.shape == (pop, 2)
    assert (pairs[:, 0] == np.arange(pop)).all()
    assert (pairs[:, 1] != pairs[:, 0]).all()
    assert ((pairs[:, 1] >= 0) & (pairs[:, 1] < pop)).all()
    # every other member is drawn about equally often over many generations
    counts = np.zeros((pop, pop), dtype=np.int64)
    for gen in range(2000):
        p = oracle.random_pairs(pop, seed=11, gen=gen)
        counts[np.arange(pop), p[:, 1]] += 1
    assert (np.diag(counts) == 0).all()
    off = counts[~np.eye(pop, dtype=bool)]
    assert off.min() > 0.75 * 2000 / (pop - 1) and off.max() < 1.25 * 2000 / (pop - 1)
    # a new generation or seed gives a new pairing
    assert (oracle.random_pairs(pop, 11, 3)[:, 1] != pairs[:, 1]).any()
    assert (oracle.random_pairs(pop, 12, 2)[:, 1] != pairs[:, 1]).any()


@pytest.mark.parametrize("i,gen,pop", [(0, 0, 5), (4, 7, 5), (13, 1, 100), (99, 250, 100)])
def test_random_pairs_published_philox_draw(i, gen, pop):
    # the draw is word 0 of the published Philox4x32-10 at (i, gen, 0, domain),
    # scaled to the pop - 1 other members, skipping i itself
    w0 = oracle.philox(i, gen, 0, D_PAIRS, 5)[0]
    j = (w0 * (pop - 1)) >> 32
    j += j >= i
    assert oracle.random_pairs(pop, seed=5, gen=gen)[i, 1] == j


def test_random_pairs_degenerate():
    assert oracle.random_pairs(1, 3, 0).tolist() == [[0, 0]]
    assert oracle.random_pairs(2, 3, 0).tolist() == [[0, 1], [1, 0]]
    assert oracle.random_pairs(0, 3, 0).shape == (0, 2)


# ---------------------------------------------------------------------------
# brute-force minimum conflicts against closed forms
@pytest.mark.parametrize("n", range(1, 9))
@pytest.mark.parametrize("k", range(1, 5))
def test_min_conflicts_complete_graph(n, k):
    # K_n split as evenly as possible: r classes of q + 1 and k - r of q
    assert brute.min_conflicts(complete(n), k) == kn_min_conflicts(n, k)


@pytest.mark.parametrize("m", range(1, 5))
def test_min_conflicts_cycles(m):
    odd, even = cycle(2 * m + 1), cycle(2 * m + 2)
    assert brute.min_conflicts(odd, 2) == 1  # an odd cycle is not bipartite; one edge suffices
    assert brute.min_conflicts(odd, 3) == 0
    assert brute.min_conflicts(even, 2) == 0
    assert brute.min_conflicts(odd, 1) == 2 * m + 1  # one colour: every edge conflicts


def test_min_conflicts_other_closed_forms():
    # Petersen graph: chromatic number 3, maximum cut 12 of its 15 edges
    assert brute.min_conflicts(petersen(), 3) == 0
    assert brute.min_conflicts(petersen(), 2) == 15 - 12
    assert brute.min_conflicts(complete_bipartite(3, 4), 2) == 0
    assert brute.min_conflicts(complete_bipartite(3, 4), 1) == 12
    assert brute.min_conflicts(edgeless(7), 1) == 0


# ---------------------------------------------------------------------------
# greedy WVCP start: order by weight desc, degree desc, index asc (Section 2.1)
def _path4(weights):
    return from_edges(4, np.array([(0, 1), (1, 2), (2, 3)])).with_weights(np.asarray(weights, np.int32))


def test_greedy_order_degree_breaks_weight_ties():
    # equal weights: order 1, 2 (degree 2, by index), then 0, 3 (degree 1).
    # 1 opens colour 0, 2 opens 1, 0 can only take 1, 3 can only take 0.
    # Degree ascending would give [0, 1, 2, 0]; index descending [0, 1, 0, 1].
    col, used = oracle.greedy_init(_path4([4, 4, 4, 4]), seed=1, ind=0)
    assert col.tolist() == [1, 0, 1, 0] and used == 2


def test_greedy_order_weight_first():
    # weights 5, 1, 1, 5: order 0, 3 (weight 5, equal degree, by index), then 1, 2.
    # 0 opens 0, 3 takes 0, 1 opens 1, 2 (next to colours 1 and 0) opens 2.
    # Ordering by degree first would give [1, 0, 1, 0] with two colours.
    col, used = oracle.greedy_init(_path4([5, 1, 1, 5]), seed=1, ind=0)
    assert col.tolist() == [0, 1, 2, 0] and used == 3


def test_greedy_order_index_breaks_full_ties():
    # a triangle 0-1-2 plus vertex 3 joined to 2 only, weights 2, 2, 2, 2:
    # degrees 2, 2, 3, 1 -> order 2, 0, 1, 3.  2 opens 0, 0 opens 1, 1 opens 2,
    # 3 (next to colour 0 only) picks among {1, 2} by the Philox draw.
    g = from_edges(4, np.array([(0, 1), (0, 2), (1, 2), (2, 3)])).with_weights(np.full(4, 2, np.int32))
    for seed in range(6):
        col, used = oracle.greedy_init(g, seed=seed, ind=3)
        assert col[:3].tolist() == [1, 2, 0] and used == 3
        w0 = oracle.philox(3, 0, 3, 0x80000008, seed)[0]
        assert col[3] == [1, 2][(w0 * 2) >> 32]
