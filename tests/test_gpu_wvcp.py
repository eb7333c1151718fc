"""GPU parity of the weighted tabu search (Section 2.2, Algorithm 2) and the
greedy initialisation (Section 2.1) against the CPU oracle: bit-exact best
legal colouring, score, counters and fingerprint."""
import sys

import numpy as np
import pytest
import torch

import oracle
from workloads import workload
from workloads.graphs import gnp, uniform_weights

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    return dlm


def test_greedy_init_parity(dlm, dev):
    g = gnp(200, 0.3, seed=2).with_weights(uniform_weights(200, 1, 100, seed=3))
    G = dlm.Graph.from_csr(g)
    say("greedy init n=200 pop=37")
    col, ku = dlm.init_population(G, 0, 37, seed=4, ind_base=3, mode="greedy")
    col, ku = col.cpu().numpy(), ku.cpu().numpy()
    for i in range(37):
        ref, used = oracle.greedy_init(g, seed=4, ind=3 + i)
        assert (col[i] == ref).all() and ku[i] == used


@pytest.mark.parametrize("n,p,T,R,block", [(40, 0.3, 200, 4, 64), (120, 0.5, 600, 3, 256),
                                           (90, 0.2, 300, 10, 128)])
def test_wvcp_parity(dlm, dev, n, p, T, R, block):
    g = gnp(n, p, seed=n).with_weights(uniform_weights(n, 1, 100, seed=n + 1))
    pop = 5
    starts, ks = [], []
    for i in range(pop):
        c, u = oracle.greedy_init(g, seed=2, ind=i)
        starts.append(c)
        ks.append(u)
    k = max(ks) + 2
    starts = np.stack(starts)
    ref = oracle.wvcp_batch(g, starts, np.arange(pop), k, T, R, seed=6)
    G = dlm.Graph.from_csr(g)
    say(f"wvcp n={n} k={k} T={T} R={R} block={block}")
    r = dlm.wvcp_batch(G, torch.from_numpy(starts).cuda(), k, T, R, seed=6, block=block)
    torch.cuda.synchronize()
    assert (r["best_legal"].cpu().numpy() == ref["best_legal"]).all()
    assert (r["stats"].cpu().numpy()[:, :6] == ref["stats"][:, :6]).all()
    assert (r["hash"].cpu().numpy().view(np.uint64) == ref["hash"]).all()
    assert (r["colors"].cpu().numpy() == ref["colors"]).all()


def test_wvcp300_sampled(dlm, dev):
    """The G(300, 0.3) weighted workload: greedy init, k = max colours used,
    10 rounds of 10 n iterations, population 4096 in one launch; 16 sampled
    individuals replayed by the oracle."""
    w = workload("wvcp300")
    g = w.graphs[0]
    G = dlm.Graph.from_csr(g)
    say("wvcp300: greedy init 4096")
    col, ku = dlm.init_population(G, 0, w.pop, seed=w.init_seed, mode="greedy")
    k = int(ku.max().item())
    assert k <= w.extra["k_cap"]
    starts = col.cpu().numpy()
    say(f"wvcp300: tabu 4096 x {w.extra['rounds']} x {w.iters[0]} k={k}")
    r = dlm.wvcp_batch(G, col, k, w.iters[0], w.extra["rounds"], seed=w.tabu_seed)
    torch.cuda.synchronize()
    ids = np.arange(0, w.pop, 256)
    ref = oracle.wvcp_batch(g, starts[ids], ids, k, w.iters[0], w.extra["rounds"],
                            seed=w.tabu_seed)
    assert (r["best_legal"].cpu().numpy()[ids] == ref["best_legal"]).all()
    assert (r["hash"].cpu().numpy().view(np.uint64)[ids] == ref["hash"]).all()
    assert (r["colors"].cpu().numpy()[ids] == ref["colors"]).all()
    # every legal result scores what it reports
    conf, ws = dlm.evaluate(G, r["colors"], k, weighted=True)
    bl = r["best_legal"].cpu().numpy()
    legal = bl != 2**31 - 1
    assert (conf.cpu().numpy()[legal] == 0).all()
    assert (ws.cpu().numpy()[legal] == bl[legal]).all()


def test_wvcp_wide_keys(dlm, dev):
    """Heavy weights with 16 fractional bits of phi: phi * max degree passes
    2^31, so the search keys its moves in 64 bits; results still equal the
    oracle's."""
    n, shift = 60, 16
    g = gnp(n, 0.5, seed=8).with_weights(uniform_weights(n, 1000, 8000, seed=9))
    max_deg = int(np.diff(g.row_ptr).max())
    pop, T, R = 4, 300, 6
    starts, ks = [], []
    for i in range(pop):
        c, u = oracle.greedy_init(g, seed=1, ind=i)
        starts.append(c)
        ks.append(u)
    k = max(ks) + 1
    max_w = int(g.weights.max())
    phi0 = (k * max_w << shift) // (2 * n)
    assert (max_w << shift) + phi0 * max_deg > 2**31  # the 64-bit path from the first round
    assert (2 * max_w) << shift <= 2**30             # within the supported weight range
    starts = np.stack(starts)
    ref = oracle.wvcp_batch(g, starts, np.arange(pop), k, T, R, seed=3, shift=shift)
    G = dlm.Graph.from_csr(g)
    say(f"wvcp wide keys n={n} k={k} shift={shift}")
    r = dlm.wvcp_batch(G, torch.from_numpy(starts).cuda(), k, T, R, seed=3, shift=shift, block=128)
    torch.cuda.synchronize()
    assert (r["best_legal"].cpu().numpy() == ref["best_legal"]).all()
    assert (r["stats"].cpu().numpy()[:, :6] == ref["stats"][:, :6]).all()
    assert (r["hash"].cpu().numpy().view(np.uint64) == ref["hash"]).all()
    assert (r["colors"].cpu().numpy() == ref["colors"]).all()
