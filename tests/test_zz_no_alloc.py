"""The allocation-free TabuCol entry point (dlm_tabu_batch_static, the
library's fixed device scratch as workspace) against dlm_tabu_batch with a
caller-owned workspace: bit-identical outputs on two calls in a row, the
second on a smaller input, so the scratch holds the first call's contents
when the second starts; and a call whose workspace would pass the scratch
size is refused before anything is launched."""
import sys

import numpy as np
import pytest
import torch

from workloads.graphs import gnp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    return dlm


def outputs(pop, dev):
    return {"f_best": torch.empty(pop, dtype=torch.int32, device=dev),
            "iters": torch.empty(pop, dtype=torch.int32, device=dev),
            "stats": torch.empty((pop, 8), dtype=torch.int64, device=dev),
            "hash": torch.empty(pop, dtype=torch.int64, device=dev)}


def both(dlm, g, k, pop, T, seed, table, dev):
    G = dlm.Graph.from_csr(g)
    start, _ = dlm.init_population(G, k, pop, seed=seed + 100)
    a = start.clone()
    b = start.clone()
    need = dlm.tabu_workspace_bytes(G, pop, k, T, seed, table=table)
    assert 0 < need <= dlm._abi.STATIC_SCRATCH_BYTES, need
    ref = dlm.tabu_batch(G, a, k, T, seed, table=table)
    out = dlm.tabu_batch_static(G, b, k, T, seed, outputs(pop, dev), table=table)
    torch.cuda.synchronize()
    for key in ("f_best", "iters", "stats", "hash", "colors"):
        assert torch.equal(ref[key], out[key]), key
    return ref


@pytest.mark.parametrize("table", ["split8", "global16"])
def test_static_matches_workspace_twice(dlm, dev, table):
    say(f"static scratch {table}: G(100, 0.5) k=18 pop=64 T=4000, then G(60, 0.5) k=9 pop=16 T=2500")
    r1 = both(dlm, gnp(100, 0.5, seed=0), 18, 64, 4000, 7, table, dev)
    assert int(r1["stats"][:, 0].sum()) > 0
    r2 = both(dlm, gnp(60, 0.5, seed=3), 9, 16, 2500, 11, table, dev)
    assert int(r2["stats"][:, 0].sum()) > 0


def test_static_refuses_oversized(dlm, dev):
    g = gnp(500, 0.5, seed=0)
    G = dlm.Graph.from_csr(g)
    pop, k = 8192, 49
    need = dlm.tabu_workspace_bytes(G, pop, k, 100, 1, table="split8")
    assert need > dlm._abi.STATIC_SCRATCH_BYTES
    say(f"static scratch: refuses {need} bytes")
    col = torch.zeros((pop, g.n), dtype=torch.int16, device=dev)
    with pytest.raises(dlm.DlmError) as e:
        dlm.tabu_batch_static(G, col, k, 100, 1, outputs(pop, dev), table="split8")
    assert e.value.code == -4  # DLM_E_UNSUPPORTED
    # the scratch is still usable afterwards
    both(dlm, gnp(80, 0.5, seed=5), 14, 8, 1500, 2, "split8", dev)
