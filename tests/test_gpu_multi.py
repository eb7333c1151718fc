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
