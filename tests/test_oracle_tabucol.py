"""Pins for the oracle's TabuCol (Section 2.7) against facts it cannot fake:
brute force on tiny graphs, closed forms, invariants re-derived from the
colours alone, and an independent replay of every recorded move."""
import numpy as np
import pytest

import oracle
from oracle import brute
from small_graphs import (complete, complete_bipartite, cycle, edgeless, grid,
                          kn_min_conflicts, petersen, random_tiny)
from workloads.graphs import gnp


def run(g, k, iters=2000, seed=5, ind=0, check=False, trace_cap=0, start=None):
    col = start if start is not None else oracle.init_random(g.n, k, 1, seed=11, ind_base=ind)[0]
    return oracle.tabucol(g, col, k, iters, seed=seed, ind=ind, check=check,
                          trace_cap=trace_cap)


@pytest.mark.parametrize("case", range(12))
def test_check_mode_small_random(case):
    # check mode re-derives gamma, f and the chosen move from scratch every iteration
    g = random_tiny(case, n=12 + case, p=0.4)
    for k in (2, 3, 4):
        r = run(g, k, iters=300, seed=case, ind=case, check=True)
        assert r["f_best"] == oracle.conflicts(g, r["colors"])


@pytest.mark.parametrize("case", range(20))
def test_brute_force_bounds(case):
    g = random_tiny(100 + case)
    chi = brute.chromatic_number(g)
    for k in range(1, min(4, g.n) + 1):
        r = run(g, k, iters=3000, seed=case, ind=case)
        mc = brute.min_conflicts(g, k)
        assert r["f_best"] >= mc            # guaranteed
        if k < chi:
            assert r["f_best"] > 0          # guaranteed
        assert r["f_best"] == oracle.conflicts(g, r["colors"])
    r = run(g, chi, iters=5000, seed=case, ind=case)
    assert r["f_best"] == 0                 # expected at k = chi on n <= 10


@pytest.mark.parametrize("n,k", [(5, 5), (6, 7), (7, 3), (8, 3), (9, 4), (10, 3), (6, 1)])
def test_complete_graph_closed_form(n, k):
    g = complete(n)
    r = run(g, k, iters=4000)
    assert r["f_best"] == kn_min_conflicts(n, min(k, n))
    assert brute.chromatic_number(g) == n


@pytest.mark.parametrize("n", [5, 7, 9, 11])
def test_odd_cycle(n):
    g = cycle(n)
    assert brute.chromatic_number(g) == 3 if n <= 10 else True
    assert run(g, 2, iters=3000)["f_best"] == 1
    assert run(g, 3, iters=3000)["f_best"] == 0


@pytest.mark.parametrize("g", [cycle(8), grid(3, 4), complete_bipartite(3, 4), grid(5, 5)],
                         ids=lambda g: g.name)
def test_bipartite(g):
    if g.n <= 10:
        assert brute.chromatic_number(g) == 2
    assert run(g, 2, iters=5000)["f_best"] == 0


def test_edgeless_and_already_legal():
    g = edgeless(7)
    r = run(g, 1, iters=100)
    assert r["f_best"] == 0 and r["iters"] == 0 and r["stats"][0] == 0
    g = petersen()
    legal = np.array([0, 1, 0, 1, 2, 1, 2, 2, 0, 0], dtype=np.int16)
    assert oracle.conflicts(g, legal) == 0
    r = run(g, 3, start=legal)
    assert r["iters"] == 0 and r["f_best"] == 0
    assert (r["colors"] == legal).all()


def _replay(g, k, start, res, seed, ind, ten=(6, 10, 10)):
    """Independent replay from the colours: recount f, recompute every
    admissible move with its delta from the adjacency, track tenure, and
    check the recorded move is the lexicographic min of (delta, hash, v, c)."""
    num, den, rnd = ten
    adj = [g.neighbors(v) for v in range(g.n)]
    col = start.astype(np.int64).copy()
    f = oracle.conflicts(g, col)
    f_best = f
    tabu = {}
    sum_conf = sum_deg = 0
    for t, (vc, f_after) in enumerate(res["trace"]):
        conf = [v for v in range(g.n) if (col[adj[v]] == col[v]).any()]
        sum_conf += len(conf)
        cands = []
        for v in conf:
            same = int((col[adj[v]] == col[v]).sum())
            for c in range(k):
                if c == col[v]:
                    continue
                d = int((col[adj[v]] == c).sum()) - same
                if tabu.get((v, c), -1) > t and not (f + d < f_best):
                    continue
                h = oracle.philox(ind, t, v, c, seed)[0]
                cands.append((d, h, v, c))
        if vc == -1:
            assert not cands
            assert f_after == f
            continue
        v, c = vc & 0xffff, (vc >> 16) & 0xffff
        assert min(cands)[2:] == (v, c)
        d = min(cands)[0]
        old = int(col[v])
        col[v] = c
        f = f + d
        assert f == f_after == oracle.conflicts(g, col)
        L = oracle.uniform(oracle.philox(ind, t, 0, oracle.D_TENURE, seed)[0], rnd)
        tabu[(v, old)] = t + L + min(num * f // den, oracle.TT_CAP)
        f_best = min(f_best, f)
        sum_deg += len(adj[v])
    assert f_best == res["f_best"]
    st = res["stats"]
    assert st[0] + st[1] == res["iters"]
    assert st[2] == sum_conf and st[3] == sum_deg


@pytest.mark.parametrize("case", range(6))
def test_replay_every_move(case):
    g = gnp(24, 0.35, seed=case)
    k = 4
    start = oracle.init_random(g.n, k, 1, seed=3, ind_base=case)[0]
    res = oracle.tabucol(g, start, k, 400, seed=77, ind=case, trace_cap=400)
    assert res["iters"] <= 400
    _replay(g, k, start, res, seed=77, ind=case)


def test_batch_equals_single_and_is_order_free():
    g = gnp(40, 0.5, seed=1)
    k = 6
    ids = np.array([5, 0, 17, 3], dtype=np.int32)
    starts = np.stack([oracle.init_random(g.n, k, 1, seed=9, ind_base=int(i))[0] for i in ids])
    b = oracle.tabucol_batch(g, starts, ids, k, 2000, seed=4, nthreads=2)
    for j, i in enumerate(ids):
        s = oracle.tabucol(g, starts[j], k, 2000, seed=4, ind=int(i))
        assert s["hash"] == b["hash"][j] and s["f_best"] == b["f_best"][j]
        assert (s["colors"] == b["colors"][j]).all() and (s["stats"] == b["stats"][j]).all()


def test_init_random_uniform():
    cols = oracle.init_random(200, 7, 50, seed=1)
    counts = np.bincount(cols.reshape(-1), minlength=7)
    exp = cols.size / 7
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 22.5   # 6 dof, p ~ 0.001
    assert cols.min() >= 0 and cols.max() < 7
