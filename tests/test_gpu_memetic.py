"""GPU tests of the memetic generation steps (Algorithm 1, simplified form):
pairing against the oracle's Philox draw, gather / standardise / (mu+lambda)
update against numpy definitions, and a short learned and plain loop whose
reported scores are re-derived from the colourings."""
import sys

import numpy as np
import pytest
import torch

import oracle
from workloads.graphs import gnp, planted_partite
from workloads.scorer_init import scorer_weights

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    return dlm


def test_random_pairs(dlm, dev):
    for pop in (1, 2, 7, 8192):
        say(f"pairs pop={pop}")
        got = dlm.random_pairs(pop, seed=11, gen=3).cpu().numpy()
        assert (got == oracle.random_pairs(pop, 11, 3)).all()
        if pop > 1:
            assert (got[:, 0] != got[:, 1]).all()


def test_gather_standardize_update(dlm, dev):
    rng = np.random.default_rng(0)
    src = rng.integers(0, 9, (50, 33)).astype(np.int16)
    idx = np.array([3, 49, 0, 3, -1, 50], np.int32)
    say("gather_rows")
    got = dlm.gather_rows(torch.from_numpy(src).cuda(), torch.from_numpy(idx).cuda()).cpu().numpy()
    assert (got[:4] == src[idx[:4]]).all() and (got[4:] == -1).all()
    f = rng.integers(0, 40, 1000).astype(np.int32)
    say("standardize")
    s = dlm.standardize(torch.from_numpy(f).cuda()).cpu().numpy()
    assert np.allclose(s, (f - f.mean()) / f.std(), rtol=1e-5, atol=1e-6)
    assert (dlm.standardize(torch.full((5,), 7, dtype=torch.int32, device="cuda")).cpu().numpy() == 0).all()
    pop, n = 300, 20
    par = rng.integers(0, 5, (pop, n)).astype(np.int16)
    off = rng.integers(0, 5, (pop, n)).astype(np.int16)
    fp = rng.integers(0, 30, pop).astype(np.int32)
    fo = rng.integers(0, 30, pop).astype(np.int32)
    say("pop_update")
    out, fout = dlm.pop_update(*(torch.from_numpy(x).cuda() for x in (par, fp, off, fo)))
    order = np.argsort(np.concatenate([fp, fo]), kind="stable")[:pop]
    pool = np.concatenate([par, off])
    assert (fout.cpu().numpy() == np.concatenate([fp, fo])[order]).all()
    assert (out.cpu().numpy() == pool[order]).all()


@pytest.mark.parametrize("learned", [False, True])
def test_short_memetic_loop(dlm, dev, learned):
    from paper_2109_05948_amd import memetic
    g = gnp(120, 0.5, seed=3)
    k, pop = 16, 64
    G = dlm.Graph.from_csr(g)
    say(f"memetic learned={learned}")
    res = memetic.run(G, k, pop, 600, learned=learned, seed=1, cutoff_s=60, max_generations=4,
                      scorer_params=scorer_weights(g.n, seed=0), batch=64, epochs=2)
    bests = [h[2] for h in res.history]
    assert all(b2 <= b1 for b1, b2 in zip(bests, bests[1:]))   # the (mu+lambda) update keeps the best
    assert res.best == bests[-1]
    assert res.tabu_moves > 0
    if learned and res.generations:
        assert len(res.scorer_loss) == res.generations and np.isfinite(res.scorer_loss).all()


def test_select_groups(dlm, dev):
    from oracle import diversity as dv
    rng = np.random.default_rng(3)
    for groups, K in ((1, 1), (7, 3), (500, 16)):
        s = rng.integers(0, 6, groups * K).astype(np.float32) * 0.25  # many ties
        say(f"select_groups {groups}x{K}")
        got = dlm.select_groups(torch.from_numpy(s).cuda(), groups, K, "top").cpu().numpy()
        assert (got == dv.select_groups(s, groups, K, "top")).all()
        got = dlm.select_groups(None, groups, K, "random", seed=21, gen=5).cpu().numpy()
        assert (got == dv.select_groups(None, groups, K, "random", seed=21, gen=5)).all()


def test_diversity_generation_replay(dlm, dev):
    """One generation of the loop with the diversity steps (plain selection),
    replayed step by step with the oracle: initial search, distances,
    nearest neighbours, GPX, group draw, search of the offspring, pool
    distances, spacing update.  The resulting population must be identical."""
    from oracle import diversity as dv
    from paper_2109_05948_amd import memetic
    g = gnp(100, 0.5, seed=5)
    k, pop, T, K, seed = 11, 24, 500, 5, 3
    G = dlm.Graph.from_csr(g)
    say("memetic diversity replay")
    res = memetic.run(G, k, pop, T, learned=False, seed=seed, cutoff_s=60, max_generations=1,
                      diversity=True, neighbours=K)
    assert res.generations == 1
    r0 = oracle.tabucol_batch(g, oracle.init_random(g.n, k, pop, seed=seed), np.arange(pop), k, T,
                              seed ^ memetic.SEED_TABU)
    cols, f = r0["colors"], r0["f_best"]
    nn = dv.nearest(dv.distance_matrix(cols, cols, k), K)
    pairs = np.stack([np.repeat(np.arange(pop), K), nn.reshape(-1)], 1).astype(np.int32)
    children = oracle.gpx_batch(k, cols, pairs, 1, pop * K, seed ^ memetic.SEED_GPX)
    off = children[dv.select_groups(None, pop, K, "random", seed=seed ^ memetic.SEED_SEL, gen=1)]
    r1 = oracle.tabucol_batch(g, off, np.arange(pop, 2 * pop), k, T, seed ^ memetic.SEED_TABU)
    rows = np.concatenate([cols, r1["colors"]])
    fs = np.concatenate([f, r1["f_best"]])
    pick, _ = dv.spacing_update(fs, dv.distance_matrix(rows, rows, k), pop, g.n // 10)
    assert (res.colors.cpu().numpy() == rows[pick]).all()
    assert (res.f.cpu().numpy() == fs[pick]).all()


@pytest.mark.parametrize("learned", [False, True])
def test_short_memetic_loop_diversity(dlm, dev, learned):
    from paper_2109_05948_amd import memetic
    g = gnp(120, 0.5, seed=3)
    k, pop = 16, 64
    G = dlm.Graph.from_csr(g)
    say(f"memetic diversity learned={learned}")
    res = memetic.run(G, k, pop, 600, learned=learned, seed=1, cutoff_s=60, max_generations=4,
                      scorer_params=scorer_weights(g.n, seed=0), batch=64, epochs=2, diversity=True,
                      neighbours=8)
    bests = [h[2] for h in res.history]
    assert all(b2 <= b1 for b1, b2 in zip(bests, bests[1:]))  # the spacing update takes the best first
    assert res.best == bests[-1] == int(res.f.min().item())
    conf, _ = dlm.evaluate(G, res.colors, k)
    assert (conf == res.f).all()
    if learned and res.generations:
        assert len(res.scorer_loss) == res.generations and np.isfinite(res.scorer_loss).all()


def test_memetic_loop_invariant_network(dlm, dev):
    """The learned loop with the paper's colour-invariant network as scorer
    (k-COL widths for 120 vertices), with the diversity steps: the loop runs,
    its scores are the conflicts of its population, the network's losses are
    finite, and its parameters (with the widths) come back for the next k."""
    from paper_2109_05948_amd import memetic
    from workloads.invnet_init import col_widths, invnet_weights
    g = gnp(120, 0.5, seed=3)
    k, pop = 16, 64
    G = dlm.Graph.from_csr(g)
    params = invnet_weights(g.n, col_widths(g.n), seed=0)
    params["widths"] = col_widths(g.n)
    say("memetic invariant network")
    res = memetic.run(G, k, pop, 600, learned=True, seed=1, cutoff_s=60, max_generations=3, scorer_params=params,
                      batch=32, epochs=2, diversity=True, neighbours=8, network="invariant", eval_chunk=96)
    conf, _ = dlm.evaluate(G, res.colors, k)
    assert (conf == res.f).all() and res.best == int(res.f.min().item())
    if res.generations:
        assert len(res.scorer_loss) == res.generations and np.isfinite(res.scorer_loss).all()
    assert res.scorer_params["widths"] == col_widths(g.n)
    assert res.scorer_params["L1"].shape == (10 * g.n, 5 * g.n)


def test_reduce_colours(dlm, dev):
    from oracle import reduce as rd
    rng = np.random.default_rng(8)
    for pop, n, k in ((1, 1, 2), (9, 57, 5), (300, 500, 49), (4, 900, 300)):
        rows = rng.integers(0, k, size=(pop, n)).astype(np.int16)
        if pop > 3:
            rows[3, 5] = k  # an invalid row
        say(f"reduce_colours pop={pop} n={n} k={k}")
        got = dlm.reduce_colours(torch.from_numpy(rows).cuda(), k, seed=31, step=k - 1).cpu().numpy()
        assert (got == rd.reduce_colours(rows, k, seed=31, step=k - 1)).all()


@pytest.mark.parametrize("learned", [False, True])
def test_decreasing_k(dlm, dev, learned):
    """Section 2.7 on a planted 6-partite graph from k = 9: every k found
    legal is one below the last, each reported colouring is legal with k
    colours, and k = 6 (the planted partition) is reached."""
    from paper_2109_05948_amd import memetic
    g, _ = planted_partite(150, 6, 0.5, seed=2)
    G = dlm.Graph.from_csr(g)
    say(f"decreasing k learned={learned}")
    res = memetic.decreasing_k(G, 9, 32, 3000, learned, seed=4, cutoff_s=90, max_generations=30,
                               scorer_params=scorer_weights(g.n, seed=0), batch=32, epochs=1)
    ks = [k for k, _ in res.found]
    assert ks[:4] == [9, 8, 7, 6] and ks == list(range(9, 9 - len(ks), -1))
    assert all(t2 >= t1 for (_, t1), (_, t2) in zip(res.found, res.found[1:]))
    for k, col in res.legal.items():
        assert col.min() >= 0 and col.max() < k
        conf, _ = dlm.evaluate(G, torch.from_numpy(col[None, :]).cuda(), k)
        assert int(conf.item()) == 0
    assert res.best_k == ks[-1] <= 6


@pytest.mark.parametrize("learned", [False, True])
def test_weighted_memetic_loop(dlm, dev, learned):
    """The loop on the WVCP (Section 2.2): greedy start, Algorithm 2 as the
    local search; the best legal weighted score never rises, and every
    reported score is the weighted score of a legal colouring in the
    population."""
    from paper_2109_05948_amd import memetic
    from workloads.graphs import uniform_weights
    g = gnp(90, 0.3, seed=4)
    g = g.with_weights(uniform_weights(90, 1, 100, seed=5))
    G = dlm.Graph.from_csr(g)
    say(f"weighted memetic learned={learned}")
    res = memetic.run(G, 0, 32, 10 * g.n, learned=learned, seed=2, cutoff_s=60, max_generations=3,
                      scorer_params=scorer_weights(g.n, seed=0), batch=32, epochs=1, weighted=True, rounds=3)
    bests = [h[2] for h in res.history]
    assert all(b2 <= b1 for b1, b2 in zip(bests, bests[1:]))
    assert res.generations == 3 and res.time_to_legal is None
    k = int(res.colors.max().item()) + 1
    conf, ws = dlm.evaluate(G, res.colors, k, weighted=True)
    legal = (res.f != 0x7fffffff)
    assert legal.any() and (conf[legal] == 0).all()
    assert (ws[legal] == res.f[legal]).all()


def test_sliced_search_is_identical(dlm, dev):
    """A local-search pass split into launches of fewer individuals
    (slice_rows) gives the same loop: every individual keeps its own random
    stream."""
    from paper_2109_05948_amd import memetic
    from workloads.graphs import uniform_weights
    g = gnp(90, 0.3, seed=4)
    g = g.with_weights(uniform_weights(90, 1, 100, seed=5))
    G = dlm.Graph.from_csr(g)
    say("weighted memetic sliced search")
    runs = [memetic.run(G, 0, 32, 10 * g.n, learned=True, seed=3, cutoff_s=60, max_generations=2,
                        scorer_params=scorer_weights(g.n, seed=0), batch=32, epochs=1, weighted=True, rounds=3,
                        slice_rows=sr) for sr in (0, 12)]
    assert [h[2] for h in runs[0].history] == [h[2] for h in runs[1].history]
    assert torch.equal(runs[0].colors, runs[1].colors) and torch.equal(runs[0].f, runs[1].f)


def test_weighted_memetic_loop_invariant_network(dlm, dev):
    """The WVCP loop learning with the paper's network at its WVCP depth
    (hidden widths 5n, 2n, n, n // 2): scores stay the weighted scores of
    legal colourings and the network's losses are finite."""
    from paper_2109_05948_amd import memetic
    from workloads.graphs import uniform_weights
    from workloads.invnet_init import invnet_weights, wvcp_widths
    g = gnp(90, 0.3, seed=4)
    g = g.with_weights(uniform_weights(90, 1, 100, seed=5))
    G = dlm.Graph.from_csr(g)
    params = invnet_weights(g.n, wvcp_widths(g.n), seed=1)
    params["widths"] = wvcp_widths(g.n)
    say("weighted memetic invariant network")
    res = memetic.run(G, 0, 32, 10 * g.n, learned=True, seed=2, cutoff_s=60, max_generations=3,
                      scorer_params=params, batch=16, epochs=2, weighted=True, rounds=3, network="invariant",
                      eval_chunk=64)
    assert res.generations == 3 and len(res.scorer_loss) == 3 and np.isfinite(res.scorer_loss).all()
    k = int(res.colors.max().item()) + 1
    conf, ws = dlm.evaluate(G, res.colors, k, weighted=True)
    legal = (res.f != 0x7fffffff)
    assert legal.any() and (conf[legal] == 0).all()
    assert (ws[legal] == res.f[legal]).all()


def _weighted_replay_start(g, pop, iters, rounds, seed):
    """The oracle's side of the WVCP loop's start: greedy colourings
    (Section 2.1), k = the most colours any uses, then Algorithm 2."""
    from paper_2109_05948_amd import memetic
    starts, used = zip(*(oracle.greedy_init(g, seed=seed, ind=i) for i in range(pop)))
    k = max(used)
    r0 = oracle.wvcp_batch(g, np.stack(starts), np.arange(pop), k, iters, rounds, seed ^ memetic.SEED_TABU)
    return k, r0["colors"], r0["best_legal"]


def test_weighted_generation_replay(dlm, dev):
    """One generation of the WVCP loop (simplified form, plain selection)
    replayed step by step with the oracle: greedy start, Algorithm 2 on the
    population, random pairing, GPX (4 children per pair), random 25 %,
    Algorithm 2 on the kept offspring, (mu + lambda) update by best legal
    weighted score.  The resulting population and scores must be identical."""
    from paper_2109_05948_amd import memetic
    from workloads.graphs import uniform_weights
    g = gnp(70, 0.3, seed=6).with_weights(uniform_weights(70, 1, 100, seed=8))
    pop, iters, rounds, seed = 16, 300, 3, 5
    G = dlm.Graph.from_csr(g)
    say("weighted generation replay")
    res = memetic.run(G, 0, pop, iters, learned=False, seed=seed, cutoff_s=60, max_generations=1,
                      weighted=True, rounds=rounds)
    assert res.generations == 1
    k, cols, f = _weighted_replay_start(g, pop, iters, rounds, seed)
    nchild = 4 * pop
    pairs = oracle.random_pairs(pop, seed ^ memetic.SEED_PAIR, 1)
    children = oracle.gpx_batch(k, cols, pairs, 4, nchild, seed ^ memetic.SEED_GPX)
    idx = oracle.select(np.zeros(nchild, np.float32), pop, 1, seed=seed ^ memetic.SEED_SEL, gen=1)
    r1 = oracle.wvcp_batch(g, children[idx], np.arange(pop, 2 * pop), k, iters, rounds, seed ^ memetic.SEED_TABU)
    rows = np.concatenate([cols, r1["colors"]])
    fs = np.concatenate([f, r1["best_legal"]])
    order = np.argsort(fs, kind="stable")[:pop]
    assert (fs < 0x7FFFFFFF).any()
    assert (res.f.cpu().numpy() == fs[order]).all()
    assert (res.colors.cpu().numpy() == rows[order]).all()


def test_weighted_diversity_generation_replay(dlm, dev):
    """The same with the paper's diversity steps (Sections 2.4 to 2.6):
    nearest neighbours by partition distance, one GPX child per pair, one
    random child per group, spacing update of the pool."""
    from oracle import diversity as dv
    from paper_2109_05948_amd import memetic
    from workloads.graphs import uniform_weights
    g = gnp(80, 0.3, seed=7).with_weights(uniform_weights(80, 1, 100, seed=9))
    pop, iters, rounds, seed, K = 20, 300, 3, 4, 5
    G = dlm.Graph.from_csr(g)
    say("weighted diversity generation replay")
    res = memetic.run(G, 0, pop, iters, learned=False, seed=seed, cutoff_s=60, max_generations=1,
                      weighted=True, rounds=rounds, diversity=True, neighbours=K)
    assert res.generations == 1
    k, cols, f = _weighted_replay_start(g, pop, iters, rounds, seed)
    nn = dv.nearest(dv.distance_matrix(cols, cols, k), K)
    pairs = np.stack([np.repeat(np.arange(pop), K), nn.reshape(-1)], 1).astype(np.int32)
    children = oracle.gpx_batch(k, cols, pairs, 1, pop * K, seed ^ memetic.SEED_GPX)
    off = children[dv.select_groups(None, pop, K, "random", seed=seed ^ memetic.SEED_SEL, gen=1)]
    r1 = oracle.wvcp_batch(g, off, np.arange(pop, 2 * pop), k, iters, rounds, seed ^ memetic.SEED_TABU)
    rows = np.concatenate([cols, r1["colors"]])
    fs = np.concatenate([f, r1["best_legal"]])
    pick, _ = dv.spacing_update(fs, dv.distance_matrix(rows, rows, k), pop, g.n // 10)
    assert (res.f.cpu().numpy() == fs[pick]).all()
    assert (res.colors.cpu().numpy() == rows[pick]).all()


@pytest.mark.gpu
@pytest.mark.parametrize("count,frac,seed", [(1, 0.0, 1), (1, 1.0, 2), (37, 0.3, 3), (5000, 0.05, 4), (700, 1.0, 5),
                                             (700, 0.0, 6)])
def test_wvcp_targets_parity(dev, count, frac, seed):
    """dlm_wvcp_targets against the oracle's rule: random legal scores with a
    fraction frac of searches that met no legal colouring (all, none, one)."""
    import paper_2109_05948_amd as dlm
    from oracle.scorer import wvcp_targets
    rng = np.random.default_rng(seed)
    f = rng.integers(1, 1 << 30, size=count).astype(np.int32)
    f[rng.random(count) < frac] = 0x7FFFFFFF
    print(f"wvcp targets count={count} frac={frac}", flush=True)
    got, flag = dlm.wvcp_targets(torch.from_numpy(f).cuda())
    want = wvcp_targets(f)
    if want is None:
        assert int(flag.item()) == 0
    else:
        assert int(flag.item()) == 1
        assert np.array_equal(got.cpu().numpy().astype(np.int64), want)
