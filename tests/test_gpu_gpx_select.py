"""GPU parity of GPX crossover (Sections 1 and 2.6) and offspring selection
(eq. select_cross) against the CPU oracle: bit-exact children and indices."""
import sys

import numpy as np
import pytest
import torch

import oracle
from workloads.graphs import gnp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    return dlm


@pytest.mark.parametrize("n,k,pop,npairs,per", [(50, 5, 6, 7, 4), (300, 33, 20, 40, 4),
                                                (1000, 85, 16, 24, 4), (77, 2, 3, 5, 3)])
def test_gpx_parity(dlm, dev, n, k, pop, npairs, per):
    rng = np.random.default_rng(n)
    parents = rng.integers(0, k, (pop, n)).astype(np.int16)
    pairs = rng.integers(0, pop, (npairs, 2)).astype(np.int32)
    ref = oracle.gpx_batch(k, parents, pairs, per, child_base=1000, seed=12)
    G = dlm.Graph.from_csr(gnp(n, 0.1, seed=1))
    say(f"gpx n={n} k={k} children={npairs * per}")
    got = dlm.gpx_batch(G, k, torch.from_numpy(parents).cuda(), torch.from_numpy(pairs).cuda(),
                        per, seed=12, child_base=1000)
    assert (got.cpu().numpy() == ref).all()


def test_gpx_structured_parents(dlm, dev):
    # parents that share classes exercise long runs of exact size ties
    n, k = 240, 12
    base = (np.arange(n) % k).astype(np.int16)
    perm = np.random.default_rng(0).permutation(k).astype(np.int16)
    parents = np.stack([base, perm[base], base[::-1].copy()])
    pairs = np.array([[0, 1], [1, 2], [2, 0], [0, 0]], np.int32)
    ref = oracle.gpx_batch(k, parents, pairs, 4, child_base=0, seed=3)
    G = dlm.Graph.from_csr(gnp(n, 0.1, seed=1))
    say("gpx structured")
    got = dlm.gpx_batch(G, k, torch.from_numpy(parents).cuda(), torch.from_numpy(pairs).cuda(), 4, seed=3)
    assert (got.cpu().numpy() == ref).all()


def test_gpx_bad_pair_marked(dlm, dev):
    G = dlm.Graph.from_csr(gnp(30, 0.1, seed=1))
    parents = torch.zeros((2, 30), dtype=torch.int16, device="cuda")
    pairs = torch.tensor([[0, 1], [0, 5]], dtype=torch.int32, device="cuda")
    say("gpx bad pair")
    got = dlm.gpx_batch(G, 3, parents, pairs, 2, seed=1).cpu().numpy()
    assert (got[2:] == -1).all() and (got[:2] >= 0).all()


@pytest.mark.parametrize("count,keep", [(1, 1), (1000, 250), (32768, 8192), (777, 777)])
def test_select_top_and_random(dlm, dev, count, keep):
    rng = np.random.default_rng(count)
    s = rng.normal(size=count).astype(np.float32)
    s[::5] = s[0]
    if count > 10:
        s[3] = np.nan
    say(f"select count={count} keep={keep}")
    got = dlm.select(torch.from_numpy(s).cuda(), count, keep, "top").cpu().numpy()
    assert (got == oracle.select(s, keep, 0)).all()
    got = dlm.select(None, count, keep, "random", seed=5, gen=9).cpu().numpy()
    assert (got == oracle.select(s, keep, 1, seed=5, gen=9)).all()
