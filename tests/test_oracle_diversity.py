"""Pins of the diversity reference (Sections 2.4 to 2.6): the approximate
partition distance against the partition distance's definition (brute force
over class bijections), the assignment bound, relabelling and symmetry, and
hand-worked cases; the spacing update and the nearest-neighbour lists
against hand-worked cases and their defining invariants."""
import itertools

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

from oracle import diversity as dv


def exact_by_bijection(a, b, k):
    """Fewest vertices to move so that a's partition becomes b's: the
    smallest number of disagreements over all relabellings of a."""
    best = len(a)
    for perm in itertools.permutations(range(k)):
        best = min(best, int(sum(perm[x] != y for x, y in zip(a, b))))
    return best


def test_two_passes_hand_case():
    # M = [[3,0,0],[2,2,0],[0,0,1]]: the pass over A (classes by size 1, 0, 2)
    # matches only 2 + 1; the pass over B (0, 1, 2) matches 3 + 2 + 1
    a = [0, 0, 0, 1, 1, 1, 1, 2]
    b = [0, 0, 0, 0, 0, 1, 1, 2]
    m = dv.overlap(np.array(a), np.array(b), 3)
    assert m.tolist() == [[3, 0, 0], [2, 2, 0], [0, 0, 1]]
    assert dv.class_order(np.array(a), 3) == [1, 0, 2]
    assert dv.greedy_match(m, [1, 0, 2]) == 3
    assert dv.greedy_match(m.T, [0, 1, 2]) == 6
    assert dv.approx_distance(a, b, 3) == 2
    assert exact_by_bijection(a, b, 3) == 2


def test_greedy_overestimates_hand_case():
    # M = [[2,1],[2,0]]: both greedy passes match 2, the best matching is
    # 1 + 2, so D~ = 3 > D = 2
    a = [0, 0, 0, 1, 1]
    b = [0, 0, 1, 0, 0]
    assert dv.overlap(np.array(a), np.array(b), 2).tolist() == [[2, 1], [2, 0]]
    assert dv.approx_distance(a, b, 2) == 3
    assert exact_by_bijection(a, b, 2) == 2


def test_relabelling_is_distance_zero():
    rng = np.random.default_rng(1)
    for _ in range(50):
        k = int(rng.integers(1, 9))
        a = rng.integers(0, k, size=40)
        perm = rng.permutation(k)
        assert dv.approx_distance(a, perm[a], k) == 0


def test_upper_bound_and_exact_when_close_brute_force():
    rng = np.random.default_rng(2)
    for _ in range(300):
        k = int(rng.integers(1, 5))
        n = int(rng.integers(1, 9))
        a = rng.integers(0, k, size=n)
        b = rng.integers(0, k, size=n)
        d = exact_by_bijection(a, b, k)
        e = dv.approx_distance(a, b, k)
        assert d <= e <= n
        assert e == dv.approx_distance(b, a, k)


def test_close_partitions_are_exact():
    """A relabelled copy with a few vertices moved: every class keeps a
    strict majority partner, so D~ equals the assignment optimum."""
    rng = np.random.default_rng(3)
    for _ in range(100):
        k = int(rng.integers(2, 12))
        n = 20 * k
        a = np.repeat(np.arange(k), 20)
        rng.shuffle(a)
        b = rng.permutation(k)[a]
        moved = rng.choice(n, size=int(rng.integers(0, 6)), replace=False)
        b[moved] = rng.integers(0, k, size=moved.size)
        m = dv.overlap(a, b, k)
        r, c = linear_sum_assignment(m, maximize=True)
        assert dv.approx_distance(a, b, k) == n - int(m[r, c].sum())


def test_assignment_bound_random():
    rng = np.random.default_rng(4)
    for _ in range(100):
        k = int(rng.integers(2, 30))
        n = int(rng.integers(k, 400))
        a = rng.integers(0, k, size=n)
        b = rng.integers(0, k, size=n)
        m = dv.overlap(a, b, k)
        r, c = linear_sum_assignment(m, maximize=True)
        assert dv.approx_distance(a, b, k) >= n - int(m[r, c].sum())


def test_spacing_update_hand_case():
    # quality order: 1 (f=1), 2 (f=1), 3 (f=3), 0 (f=5); spacing 2
    f = [5, 1, 1, 3]
    d = np.array([[0, 9, 9, 9],
                  [9, 0, 2, 3],
                  [9, 2, 0, 9],
                  [9, 3, 9, 0]])
    # 1 joins; 2 is at distance 2 of 1 (not > 2); 3 joins; 0 joins
    assert dv.spacing_update(f, d, 4, 2) == ([1, 3, 0, 2], 3)
    assert dv.spacing_update(f, d, 2, 2) == ([1, 3], 2)
    # spacing 3 also rejects 3 (distance 3 of 1); then 0 joins, 2 and 3 fill
    assert dv.spacing_update(f, d, 4, 3) == ([1, 0, 2, 3], 2)


@pytest.mark.parametrize("spacing", [-1, 10**6])
def test_spacing_update_degenerate_is_top_by_quality(spacing):
    rng = np.random.default_rng(5)
    f = rng.integers(0, 6, size=30)
    d = rng.integers(0, 50, size=(30, 30))
    d = np.minimum(d, d.T)
    taken, spaced = dv.spacing_update(f, d, 12, spacing)
    top = sorted(range(30), key=lambda i: (int(f[i]), i))[:12]
    assert taken == top
    assert spaced == (12 if spacing < 0 else 1)


def test_spacing_update_invariants():
    rng = np.random.default_rng(6)
    for _ in range(20):
        total, keep, sp = 40, int(rng.integers(1, 20)), int(rng.integers(0, 30))
        f = rng.integers(0, 8, size=total)
        d = rng.integers(0, 40, size=(total, total))
        d = np.minimum(d, d.T)
        np.fill_diagonal(d, 0)
        taken, spaced = dv.spacing_update(f, d, keep, sp)
        assert len(taken) == keep and len(set(taken)) == keep
        head = taken[:spaced]
        for x, y in itertools.combinations(head, 2):
            assert d[x][y] > sp
        order = sorted(range(total), key=lambda i: (int(f[i]), i))
        for c in order[:order.index(head[-1])]:
            if c not in head:  # rejected: too close to one taken before it
                assert any(d[c][s] <= sp for s in head[:sum(order.index(h) < order.index(c) for h in head)])


def test_nearest_hand_case():
    d = np.array([[0, 4, 2, 2],
                  [4, 0, 1, 7],
                  [2, 1, 0, 5],
                  [2, 7, 5, 0]])
    assert dv.nearest(d, 2).tolist() == [[2, 3], [2, 0], [1, 0], [0, 2]]
    assert dv.nearest(d, 3).tolist() == [[2, 3, 1], [2, 0, 3], [1, 0, 3], [0, 2, 1]]


def test_select_groups_top_hand_case():
    s = np.array([3.0, 1.0, 1.0, 2.0, 0.5, -1.0, 7.0, -1.0], np.float32)
    assert dv.select_groups(s, 2, 4, "top").tolist() == [1, 5]
    assert dv.select_groups(s, 4, 2, "top").tolist() == [1, 2, 5, 7]
    assert dv.select_groups(s, 8, 1, "top").tolist() == list(range(8))


def test_select_groups_random_is_uniform_and_seeded():
    import oracle
    K, groups = 5, 4000
    a = dv.select_groups(None, groups, K, "random", seed=9, gen=3)
    assert ((a // K) == np.arange(groups)).all()
    counts = np.bincount(a % K, minlength=K)
    assert counts.min() > 0.8 * groups / K  # each position drawn about equally often
    b = dv.select_groups(None, groups, K, "random", seed=9, gen=4)
    assert (a != b).any()
    # the draw is word 0 of the published Philox4x32-10 scaled to [0, K)
    w0 = oracle.philox(17, 3, 0, dv.D_SELGROUP, 9)[0]
    assert a[17] == 17 * K + (w0 * K >> 32)
