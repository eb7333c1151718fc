"""Input generators: CSR validity, determinism, planted structure, DSATUR."""
import numpy as np
import pytest

from oracle import brute
import oracle
from small_graphs import random_tiny
from workloads.graphs import (dsatur_colors, from_edges, gnp, is_valid_csr, planted_partite,
                              uniform_weights)


@pytest.mark.parametrize("n,p", [(50, 0.1), (100, 0.5), (120, 0.9)])
def test_gnp_valid_and_dense_enough(n, p):
    g = gnp(n, p, seed=0)
    assert is_valid_csr(g)
    dens = g.m / (n * (n - 1) / 2)
    assert abs(dens - p) < 5 * np.sqrt(p * (1 - p) / (n * (n - 1) / 2)) + 1e-9
    g2 = gnp(n, p, seed=0)
    assert (g.col_idx == g2.col_idx).all() and (g.row_ptr == g2.row_ptr).all()
    assert g.col_idx.dtype == np.int32 and g.row_ptr.dtype == np.int32


def test_planted_has_hidden_legal_coloring():
    g, parts = planted_partite(200, 7, 0.5, seed=3)
    assert is_valid_csr(g)
    assert oracle.conflicts(g, parts.astype(np.int16)) == 0
    e = g.edges()
    assert (parts[e[:, 0]] != parts[e[:, 1]]).all()


def test_from_edges_dedups_and_drops_loops():
    g = from_edges(4, np.array([[0, 1], [1, 0], [2, 2], [3, 1], [0, 1]]))
    assert is_valid_csr(g) and g.m == 2


def test_weights():
    w = uniform_weights(1000, 1, 100, seed=1)
    assert w.min() >= 1 and w.max() <= 100 and w.dtype == np.int32
    assert len(np.unique(w)) == 100


@pytest.mark.parametrize("case", range(8))
def test_dsatur_legal_and_bounded(case):
    g = random_tiny(400 + case)
    c = dsatur_colors(g)
    assert oracle.conflicts(g, c.astype(np.int16)) == 0
    assert c.max() + 1 >= brute.chromatic_number(g)


def test_dsatur_vs_networkx():
    nx = pytest.importorskip("networkx")
    g = gnp(80, 0.3, seed=2)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from(g.edges().tolist())
    ref = max(nx.greedy_color(G, strategy="saturation_largest_first").values()) + 1
    ours = int(dsatur_colors(g).max()) + 1
    assert abs(ours - ref) <= 2   # same heuristic, different tie rules
