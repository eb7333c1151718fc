"""Pins for the oracle's weighted colouring path (Sections 1, 2.1, 2.2 and
Algorithm 2): exact optimum by enumeration on tiny graphs, closed forms for
the weighted score, and invariants re-derived from the colours each move."""
import numpy as np
import pytest

import oracle
from oracle import brute
from small_graphs import complete, cycle, edgeless, random_tiny
from workloads.graphs import gnp, uniform_weights


def _wgraph(g, seed, lo=1, hi=20):
    return g.with_weights(uniform_weights(g.n, lo, hi, seed))


def test_wscore_closed_forms():
    g = complete(6)
    w = np.array([3, 9, 1, 4, 4, 7], dtype=np.int32)
    # K_n: every vertex alone, so the score is the sum of the weights
    assert oracle.wscore(w, 6, np.arange(6)) == w.sum()
    # one class: the score is the largest weight
    assert oracle.wscore(w, 3, np.zeros(6)) == 9
    # unit weights: the score counts the non-empty classes (COL as WVCP)
    cols = np.array([0, 2, 2, 4, 0, 4])
    assert oracle.wscore(np.ones(6, np.int32), 5, cols) == 3
    assert brute.wvcp_opt(g, w) == w.sum()
    assert brute.wvcp_opt(edgeless(5), [2, 8, 3, 8, 1]) == 8


@pytest.mark.parametrize("case", range(10))
def test_greedy_init_legal(case):
    g = _wgraph(random_tiny(200 + case, n=9), case)
    col, used = oracle.greedy_init(g, seed=3, ind=case)
    assert oracle.conflicts(g, col) == 0
    assert col.min() == 0 and col.max() == used - 1
    assert used >= brute.chromatic_number(g)
    # the heaviest vertex is placed first, so it opens colour 0
    order = sorted(range(g.n), key=lambda v: (-g.weights[v], -len(g.neighbors(v)), v))
    assert col[order[0]] == 0


@pytest.mark.parametrize("case", range(6))
def test_check_mode(case):
    g = _wgraph(gnp(14, 0.4, seed=case), case)
    col, used = oracle.greedy_init(g, seed=1, ind=case)
    k = used + 2
    r = oracle.wvcp_tabu(g, col, k, iters_per_round=60, rounds=4, seed=case, ind=case,
                         check=True)
    if r["best_legal"] != 2**31 - 1:
        assert oracle.conflicts(g, r["colors"]) == 0
        assert oracle.wscore(g.weights, k, r["colors"]) == r["best_legal"]


@pytest.mark.parametrize("case", range(12))
def test_optimum_bound_tiny(case):
    g = _wgraph(random_tiny(300 + case, n=8), case, 1, 30)
    opt = brute.wvcp_opt(g, g.weights)
    col, used = oracle.greedy_init(g, seed=2, ind=case)
    r = oracle.wvcp_tabu(g, col, used, iters_per_round=10 * g.n, rounds=10, seed=case,
                         ind=case)
    assert r["best_legal"] >= opt          # guaranteed
    assert r["best_legal"] == opt          # expected on n = 8
    assert oracle.conflicts(g, r["colors"]) == 0


def test_odd_cycle_weighted():
    g = cycle(5).with_weights(np.array([5, 1, 1, 1, 1], np.int32))
    # vertex 0 alone in its class (5); the path 1-2-3-4 needs 2 classes of max 1
    assert brute.wvcp_opt(g, g.weights) == 7
    col, used = oracle.greedy_init(g, seed=0, ind=0)
    r = oracle.wvcp_tabu(g, col, max(used, 3), 50, 10, seed=1, ind=0)
    assert r["best_legal"] == 7


def test_batch_equals_single():
    g = _wgraph(gnp(30, 0.3, seed=4), 4, 1, 100)
    ids = np.array([2, 9, 0], np.int32)
    starts, ks = [], []
    for i in ids:
        c, u = oracle.greedy_init(g, seed=5, ind=int(i))
        starts.append(c)
        ks.append(u)
    k = max(ks)
    b = oracle.wvcp_batch(g, np.stack(starts), ids, k, 90, 3, seed=8, nthreads=2)
    for j, i in enumerate(ids):
        s = oracle.wvcp_tabu(g, starts[j], k, 90, 3, seed=8, ind=int(i))
        assert s["hash"] == b["hash"][j] and s["best_legal"] == b["best_legal"][j]
        assert (s["colors"] == b["colors"][j]).all()


def _g_of(g, w, k, col, phi, S):
    """eq. (AFISA_score) in fixed point: (f_w << S) + phi * c, from the colours"""
    return (oracle.wscore(w, k, col) << S) + phi * oracle.conflicts(g, col)


@pytest.mark.parametrize("case", range(4))
def test_replay_rounds_and_moves(case):
    """Independent replay of Algorithm 2: the phi schedule, every move's delta
    recounted from the colours, vertex freezing and aspiration."""
    g = _wgraph(gnp(10, 0.45, seed=case), case, 1, 12)
    w = g.weights
    n, S, R, T = g.n, 10, 5, 30
    col0, used = oracle.greedy_init(g, seed=4, ind=case)
    k = used + 1
    res = oracle.wvcp_tabu(g, col0, k, T, R, seed=21, ind=case, trace_cap=R * T)
    maxw = int(w.max())
    rl = res["rounds"]
    # phi schedule of Algorithm 2; the last round uses 2 * max w
    phi = (k * maxw << S) // (2 * n)
    for r in range(R):
        if r == R - 1:
            phi = (2 * maxw) << S
        assert rl[r][0] == phi, (r, rl[r][0], phi)
        if r < R - 1:
            phi = phi >> 1 if rl[r][1] else min(phi << 1, 1 << 30)
    col = col0.astype(np.int64).copy()
    best_legal = None
    frz = 2 * n // 10
    t = 0
    for r in range(R):
        phi = int(rl[r][0])
        G = _g_of(g, w, k, col, phi, S)
        G_best, best_state = G, col.copy()
        if oracle.conflicts(g, col) == 0:
            fw = oracle.wscore(w, k, col)
            best_legal = fw if best_legal is None else min(best_legal, fw)
        frozen = np.zeros(n, np.int64)
        for _ in range(T):
            cands = []
            for v in range(n):
                for c in range(k):
                    if c == col[v]:
                        continue
                    trial = col.copy()
                    trial[v] = c
                    d = _g_of(g, w, k, trial, phi, S) - G
                    if frozen[v] > t and not (G + d < G_best):
                        continue
                    cands.append((d, oracle.philox(case, t, v, c, 21)[0], v, c))
            vc, g_after = res["trace"][t]
            if vc == 0xffffffff:
                assert not cands
            else:
                v, c = int(vc) & 0xffff, (int(vc) >> 16) & 0xffff
                assert min(cands)[2:] == (v, c), (t, min(cands), (v, c))
                G += min(cands)[0]
                col[v] = c
                assert G == g_after == _g_of(g, w, k, col, phi, S)
                L = oracle.uniform(oracle.philox(case, t, 0, oracle.D_TENURE, 21)[0], 10)
                frozen[v] = t + L + frz
                if G < G_best:
                    G_best, best_state = G, col.copy()
                if oracle.conflicts(g, col) == 0:
                    fw = oracle.wscore(w, k, col)
                    best_legal = fw if best_legal is None else min(best_legal, fw)
            t += 1
        col = best_state
        assert rl[r][1] == (oracle.conflicts(g, col) == 0)
        assert rl[r][2] == oracle.wscore(w, k, col)
    assert res["best_legal"] == (best_legal if best_legal is not None else 2**31 - 1)
