"""Pins for the oracle's GPX crossover (Sections 1 and 2.6) and offspring
selection (eq. select_cross): partition invariants, relabelling invariance,
the greedy largest-class property, and agreement with numpy's stable sort."""
import numpy as np
import pytest

import oracle


def _partition(col):
    """canonical form of a colouring: the set of its classes"""
    col = np.asarray(col)
    return frozenset(frozenset(np.where(col == c)[0].tolist()) for c in np.unique(col))


@pytest.mark.parametrize("case", range(8))
def test_gpx_greedy_property(case):
    rng = np.random.default_rng(case)
    n, k = int(rng.integers(10, 60)), int(rng.integers(2, 9))
    A = rng.integers(0, k, n).astype(np.int16)
    B = rng.integers(0, k, n).astype(np.int16)
    ch = oracle.gpx(k, A, B, child=case, seed=3)
    assert ch.min() >= 0 and ch.max() < k
    # replay: step l takes a largest remaining class of the alternating parent
    left = np.ones(n, bool)
    for l in range(k):
        P = A if l % 2 == 0 else B
        sizes = np.bincount(P[left], minlength=k) if left.any() else np.zeros(k, int)
        if sizes.max() == 0:
            break
        # the class taken at step l: a largest remaining class of P, all of
        # whose remaining vertices got colour l (leftovers may also hold l)
        taken = [c for c in range(k) if sizes[c] == sizes.max()
                 and (ch[left & (P == c)] == l).all()]
        assert taken, f"step {l}: no largest class of the parent became colour {l}"
        left &= ~(P == taken[0])
    # whatever is left got a colour in range (random fill)
    assert (ch[left] >= 0).all() and (ch[left] < k).all()


@pytest.mark.parametrize("case", range(6))
def test_gpx_relabelling_invariance(case):
    rng = np.random.default_rng(50 + case)
    n, k = 40, 6
    A = rng.integers(0, k, n).astype(np.int16)
    B = rng.integers(0, k, n).astype(np.int16)
    perm = rng.permutation(k).astype(np.int16)
    c1 = oracle.gpx(k, A, B, child=7, seed=1)
    c2 = oracle.gpx(k, perm[A], B, child=7, seed=1)
    c3 = oracle.gpx(k, A, perm[B], child=7, seed=1)
    assert _partition(c1) == _partition(c2) == _partition(c3)
    # crossing a colouring with a relabelled copy of itself returns its partition
    c4 = oracle.gpx(k, A, perm[A], child=2, seed=1)
    assert _partition(c4) == _partition(A)


def test_gpx_batch_matches_single():
    rng = np.random.default_rng(3)
    par = rng.integers(0, 5, (6, 30)).astype(np.int16)
    pairs = np.array([[0, 1], [2, 5], [4, 4]], np.int32)
    out = oracle.gpx_batch(5, par, pairs, per_pair=4, child_base=100, seed=9)
    for p, (a, b) in enumerate(pairs):
        for j in range(4):
            ref = oracle.gpx(5, par[a], par[b], child=100 + 4 * p + j, seed=9)
            assert (out[4 * p + j] == ref).all()


@pytest.mark.parametrize("case", range(5))
def test_select_top_matches_stable_sort(case):
    rng = np.random.default_rng(case)
    s = rng.normal(size=500).astype(np.float32)
    s[::7] = s[3]                       # plenty of exact ties
    keep = 125
    got = oracle.select(s, keep, mode=0)
    ref = np.argsort(s, kind="stable")[:keep]
    assert (got == ref).all()


def test_select_random_is_a_subset_and_deterministic():
    s = np.zeros(1000, np.float32)
    a = oracle.select(s, 250, mode=1, seed=4, gen=2)
    b = oracle.select(s, 250, mode=1, seed=4, gen=2)
    c = oracle.select(s, 250, mode=1, seed=4, gen=3)
    assert (a == b).all() and len(set(a.tolist())) == 250
    assert set(a.tolist()) != set(c.tolist())
    assert a.min() >= 0 and a.max() < 1000
