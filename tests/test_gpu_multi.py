"""Uneven batch in one persistent hipGraph launch: every individual of every
graph must equal its single-graph dlm_tabu_batch result (and the oracle on
samples), for several launch shapes, over repeated graph replays."""
import sys

import numpy as np
import pytest
import torch

import oracle
from workloads.graphs import gnp, planted_partite

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    return dlm


def make_jobs(dlm, specs, seed=5):
    jobs, starts = [], []
    for gi, (kind, n, p, k, pop, T) in enumerate(specs):
        g = gnp(n, p, seed=gi) if kind == "gnp" else planted_partite(n, k, p, seed=gi)[0]
        G = dlm.Graph.from_csr(g)
        col = oracle.init_random(n, k, pop, seed=seed, ind_base=1000 * gi)
        starts.append(col)
        jobs.append({"graph": G, "g": g, "colors": torch.from_numpy(col).cuda(), "k": k, "iters": T,
                     "seed": 77 + gi, "ind_base": 1000 * gi})
    return jobs, starts


SPECS = [("gnp", 120, 0.5, 14, 9, 1500), ("planted", 300, 0.5, 9, 5, 2500),
         ("gnp", 60, 0.3, 5, 13, 800), ("gnp", 600, 0.5, 90, 3, 1200),   # 600 x 90: split or device table
         ("planted", 200, 0.6, 20, 6, 2000),
         ("gnp", 740, 0.012, 3, 4, 800)]   # k = 3: classes near 255, byte-table reruns


@pytest.mark.parametrize("block,budget", [(256, 0), (64, 40000), (512, 80000), (128, 20000)])
def test_multi_equals_single(dlm, dev, block, budget):
    jobs, starts = make_jobs(dlm, SPECS)
    say(f"multi plan block={block} budget={budget}")
    mb = dlm.MultiBatch(jobs, block=block, lds_budget=budget)
    info = mb.info()
    assert info["items"] == sum(s[4] for s in SPECS)
    assert info["graphs_on_device_table"] >= 1
    for rep in range(3):   # replays of the captured graph, eager work between them
        for j, st in zip(jobs, starts):
            j["colors"].copy_(torch.from_numpy(st))
        torch.cuda.synchronize()
        mb.launch()
        torch.cuda.synchronize()
        for gi, (j, st) in enumerate(zip(jobs, starts)):
            single = dlm.tabu_batch(j["graph"], torch.from_numpy(st).cuda(), j["k"], j["iters"],
                                    j["seed"], ind_base=j["ind_base"])
            torch.cuda.synchronize()
            assert (j["f_best"].cpu() == single["f_best"].cpu()).all(), (rep, gi)
            assert (j["iters_out"].cpu() == single["iters"].cpu()).all(), (rep, gi)
            assert (j["hash"].cpu() == single["hash"].cpu()).all(), (rep, gi)
            assert (j["colors"].cpu() == single["colors"].cpu()).all(), (rep, gi)
    # and the oracle on the first individual of every graph
    for j, st in zip(jobs, starts):
        ref = oracle.tabucol(j["g"], st[0], j["k"], j["iters"], seed=j["seed"], ind=j["ind_base"])
        assert ref["f_best"] == int(j["f_best"][0]) and ref["hash"] == int(j["hash"][0].cpu().numpy().view(np.uint64))


def test_autotune_picks_a_valid_config(dlm, dev):
    jobs, _ = make_jobs(dlm, SPECS[:3])
    before = [j["colors"].clone() for j in jobs]
    say("multi autotune")
    (block, budget), rates = dlm.MultiBatch.autotune(jobs, calib_iters=300)
    assert block in (64, 128, 256, 512) and budget > 0
    assert (rates > 0).any() and np.isfinite(rates).all()
    for j, b in zip(jobs, before):   # the items' own colourings are untouched
        assert (j["colors"] == b).all()


def test_uneven64_full_plan_sampled(dlm, dev):
    """The uneven batch at its full size (64 graphs, n in [100, 1000], 256
    individuals each = 16,384 items, 128 n iterations) as the benchmark runs
    it: autotuned, one persistent launch.  Four individuals of every graph
    (0, 85, 170, 255) are replayed by the oracle; the rest must be legal
    results (f_best equal to a recount of the returned colouring)."""
    from workloads import workload
    w = workload("uneven64")
    jobs, starts = [], []
    for gi, (g, k, T) in enumerate(zip(w.graphs, w.k, w.iters)):
        G = dlm.Graph.from_csr(g)
        st = oracle.init_random(g.n, k, w.pop, seed=w.init_seed, ind_base=gi * w.pop)
        starts.append(st)
        jobs.append({"graph": G, "g": g, "colors": torch.from_numpy(st).cuda(), "k": k, "iters": T,
                     "seed": w.tabu_seed, "ind_base": gi * w.pop})
    say("uneven64: autotune")
    (block, budget), _ = dlm.MultiBatch.autotune(jobs, calib_iters=1000)
    say(f"uneven64: plan block={block} budget={budget}, one launch of {64 * w.pop} items")
    mb = dlm.MultiBatch(jobs, block=block, lds_budget=budget)
    assert mb.info()["items"] == 64 * w.pop
    mb.launch()
    torch.cuda.synchronize()
    idx = np.array([0, 85, 170, 255])
    for gi, (j, st) in enumerate(zip(jobs, starts)):
        ref = oracle.tabucol_batch(j["g"], st[idx], j["ind_base"] + idx, j["k"], j["iters"], seed=j["seed"])
        fb = j["f_best"].cpu().numpy()
        it = j["iters_out"].cpu().numpy()
        hs = j["hash"].cpu().numpy().view(np.uint64)
        col = j["colors"].cpu().numpy()
        stats = j["stats"].cpu().numpy()
        for r, i in enumerate(idx):
            msg = f"graph {gi} (n={j['g'].n}, k={j['k']}) individual {i}"
            assert fb[i] == ref["f_best"][r], msg
            assert it[i] == ref["iters"][r], msg
            assert hs[i] == ref["hash"][r], msg
            assert (col[i] == ref["colors"][r]).all(), msg
            assert (stats[i][:6] == ref["stats"][r][:6]).all(), msg
        conf, _ = dlm.evaluate(j["graph"], j["colors"], j["k"])
        assert (conf.cpu().numpy() == fb).all(), f"graph {gi}: f_best differs from the recount"
