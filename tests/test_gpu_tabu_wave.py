"""GPU parity of the one-wavefront-per-individual TabuCol tier (table
"wave8": byte gamma with a tabu flag in LDS, live tabu pairs in an LDS list)
against the CPU oracle (Section 2.7): every individual's best colouring,
f_best, iteration count, counters and trajectory fingerprint bit-identical.
Covers every row-width bucket of the scan (k up to 256), runs past the
2^15 wrap of the stored expiries, moves with more than 64 ties, scans of
several rounds, both give-up paths (a colour class passing 127 vertices,
the tabu list overflowing) with their 16-bit reruns, and the full
8192 x 100,000 run on G(500, 0.5) with 64 individuals replayed."""
import sys

import numpy as np
import pytest
import torch

import oracle
from small_graphs import complete, cycle, edgeless
from workloads import workload
from workloads.graphs import from_edges, gnp, planted_partite

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    return dlm


def gpu_run(dlm, g, starts, k, T, seed, ind_base=0, **kw):
    G = dlm.Graph.from_csr(g)
    col = torch.from_numpy(np.ascontiguousarray(starts, np.int16)).cuda()
    r = dlm.tabu_batch(G, col, k, T, seed, ind_base=ind_base, table="wave8", **kw)
    torch.cuda.synchronize()
    out = {kk: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for kk, v in r.items()}
    if out.get("hash") is not None:
        out["hash"] = out["hash"].view(np.uint64)
    return out


def compare(gpu, ref, ids, label):
    for j, i in enumerate(ids):
        msg = f"{label} individual {i}"
        assert gpu["f_best"][j] == ref["f_best"][j], (msg, gpu["f_best"][j], ref["f_best"][j])
        assert gpu["iters"][j] == ref["iters"][j], (msg, gpu["iters"][j], ref["iters"][j])
        assert (gpu["stats"][j][:6] == ref["stats"][j][:6]).all(), (msg, gpu["stats"][j], ref["stats"][j])
        assert gpu["hash"][j] == ref["hash"][j], msg
        assert (gpu["colors"][j] == ref["colors"][j]).all(), msg


SHAPES = [  # (n, p, k, T, pop): row buckets of 8, 16, 24, 32 and 64 dwords, exact widths 9 to 15 and 17 to 23
    (37, 0.3, 4, 800, 7),
    (150, 0.5, 16, 3000, 9),
    (200, 0.1, 5, 3000, 5),
    (120, 0.9, 40, 2000, 6),
    (300, 0.5, 33, 2500, 4),
    (260, 0.8, 70, 2000, 4),
    (330, 0.9, 100, 1500, 3),
    (420, 0.95, 210, 800, 3),
    (160, 0.5, 44, 1500, 3),  # 11 dwords
    (140, 0.6, 47, 1500, 3),  # 12
    (180, 0.5, 55, 1500, 3),  # 14
    (200, 0.5, 58, 1200, 3),  # 15
    (220, 0.6, 67, 1000, 3),  # 17
    (240, 0.5, 75, 1000, 3),  # 19
    (200, 0.7, 79, 1000, 3),  # 20
    (260, 0.5, 83, 1000, 3),  # 21
    (250, 0.6, 90, 1000, 3),  # 23
    (300, 0.5, 96, 1000, 3),  # 24: the bucket at its own width
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_p%g_k%d" % s[:3])
def test_wave_parity_shapes(dlm, dev, shape):
    n, p, k, T, pop = shape
    g = gnp(n, p, seed=n)
    starts = oracle.init_random(n, k, pop, seed=3, ind_base=11)
    ids = np.arange(11, 11 + pop)
    ref = oracle.tabucol_batch(g, starts, ids, k, T, seed=17)
    say(f"wave8 n={n} p={p} k={k} T={T} pop={pop}")
    gpu = gpu_run(dlm, g, starts, k, T, 17, ind_base=11)
    compare(gpu, ref, ids, f"wave8 n{n} k{k}")


def test_wave_long_run_past_expiry_wrap(dlm, dev):
    """40,000 iterations: the stored expiries (modulo 2^15) wrap."""
    g = gnp(120, 0.5, seed=7)
    k, T, pop = 13, 40000, 4
    starts = oracle.init_random(g.n, k, pop, seed=5)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=8)
    assert (ref["iters"] == T).all()  # no individual stops early
    say(f"wave8 long run n=120 k={k} T={T}")
    gpu = gpu_run(dlm, g, starts, k, T, 8)
    compare(gpu, ref, range(pop), "wave8 long")


def test_wave_trace(dlm, dev):
    g = gnp(90, 0.5, seed=2)
    k, T = 11, 600
    starts = oracle.init_random(90, k, 3, seed=1)
    say("wave8 trace n=90 k=11")
    gpu = gpu_run(dlm, g, starts, k, T, 4, trace_cap=T)
    for i in range(3):
        ref = oracle.tabucol(g, starts[i], k, T, seed=4, ind=i, trace_cap=T)
        it = ref["iters"]
        assert (gpu["trace"][i][:it] == ref["trace"][:it]).all()


def test_wave_edge_cases(dlm, dev):
    cases = [
        ("edgeless", edgeless(40), 1, 50),
        ("K9 k=3", complete(9), 3, 400),
        ("K9 k=9", complete(9), 9, 400),
        ("C7 k=2", cycle(7), 2, 300),
        ("k=1", gnp(30, 0.2, seed=1), 1, 50),
        ("T=0", gnp(30, 0.2, seed=1), 3, 0),
        ("planted", planted_partite(200, 8, 0.5, seed=4)[0], 8, 4000),
    ]
    for name, g, k, T in cases:
        starts = oracle.init_random(g.n, k, 3, seed=2)
        ref = oracle.tabucol_batch(g, starts, np.arange(3), k, T, seed=6)
        say(f"wave8 edge case {name}")
        gpu = gpu_run(dlm, g, starts, k, T, 6)
        compare(gpu, ref, range(3), name)
    # an out-of-range start colour is refused per individual
    g = gnp(30, 0.3, seed=0)
    starts = oracle.init_random(g.n, 4, 2, seed=1)
    starts[1, 5] = 4
    gpu = gpu_run(dlm, g, starts, 4, 100, 1)
    assert gpu["f_best"][1] == -1 and gpu["iters"][1] == -1 and gpu["iters"][0] >= 0


def test_wave_many_ties(dlm, dev):
    """A perfect matching on 1000 vertices with k = 120: each conflicting
    vertex ties at delta -1 with every free colour, about 2,000 tied moves
    per iteration, so the ties are hashed 64 at a time."""
    n, k, T, pop = 1000, 120, 40, 3
    g = from_edges(n, np.array([(2 * i, 2 * i + 1) for i in range(n // 2)], np.int64), "matching1000")
    starts = oracle.init_random(n, k, pop, seed=9)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=5)
    assert (ref["stats"][:, 4] > 0).all()
    say(f"wave8 matching1000 k={k}")
    gpu = gpu_run(dlm, g, starts, k, T, 5)
    compare(gpu, ref, range(pop), "wave8 matching")


def _class_sizes_over_run(start, k, trace, iters):
    col = start.astype(np.int64).copy()
    size = np.bincount(col, minlength=k)
    worst = [int(size.max())]
    for t in range(iters):
        rec = int(trace[t][0])
        if rec < 0:
            continue
        v, c = rec & 0xffff, rec >> 16
        size[col[v]] -= 1
        size[c] += 1
        col[v] = c
        worst.append(int(size.max()))
    return worst


def test_wave_reruns_when_a_class_passes_127(dlm, dev):
    """k = 3 on 370 vertices: classes of about 123.  Individuals whose start
    has a class above 127 and individuals whose class grows past 127 during
    the search both give up and are rerun with 16-bit gamma."""
    g = gnp(370, 0.02, seed=11)
    k, T, pop = 3, 1500, 16
    starts = oracle.init_random(g.n, k, pop, seed=21)
    ids = np.arange(pop)
    ref = oracle.tabucol_batch(g, starts, ids, k, T, seed=5)
    at_start, mid_run = 0, 0
    for i in range(pop):
        tr = oracle.tabucol(g, starts[i], k, T, seed=5, ind=i, trace_cap=T)
        worst = _class_sizes_over_run(starts[i], k, tr["trace"], tr["iters"])
        at_start += worst[0] > 127
        mid_run += worst[0] <= 127 and max(worst) > 127
    assert at_start > 0 and mid_run > 0, (at_start, mid_run)
    say(f"wave8 rerun n=370 k=3 ({at_start} at start, {mid_run} mid-run)")
    gpu = gpu_run(dlm, g, starts, k, T, 5)
    compare(gpu, ref, ids, "wave8 class rerun")


def test_wave_reruns_when_the_tabu_list_overflows(dlm, dev):
    """G(2000, 0.9) with k = 64: f stays above 20,000, so every tenure
    exceeds 12,000 iterations and each of the 8,000 moves leaves a live tabu
    pair.  The table fills 139 KB of the 160 KB LDS, leaving room for about
    6,000 pairs: the list overflows, the individual gives up and its 16-bit
    rerun must still equal the oracle."""
    g = gnp(2000, 0.9, seed=3)
    k, T, pop = 64, 8000, 2
    starts = oracle.init_random(g.n, k, pop, seed=4)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=6)
    assert (ref["f_best"] > 20000).all() and (ref["stats"][:, 0] > 7800).all()
    say("wave8 tabu-list overflow n=2000 k=64")
    gpu = gpu_run(dlm, g, starts, k, T, 6)
    compare(gpu, ref, range(pop), "wave8 list overflow")


def test_wave_gnp1000_k85(dlm, dev):
    """G(1000, 0.5), k = 85 (the memetic shape): scans of several rounds."""
    g = gnp(1000, 0.5, seed=0)
    k, T, pop = 85, 4000, 6
    starts = oracle.init_random(g.n, k, pop, seed=3)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=9)
    say("wave8 gnp1000 k=85")
    gpu = gpu_run(dlm, g, starts, k, T, 9)
    compare(gpu, ref, range(pop), "wave8 gnp1000")


def test_wave_gnp500_full_size_sampled(dlm, dev):
    """G(500, 0.5), k = 49, 8192 individuals x 100,000 iterations in one
    wave8 launch; individuals i = 128 j replayed by the oracle, and for
    every individual f_best = conflicts of the returned colouring."""
    w = workload("gnp500")
    g, k, T = w.graphs[0], w.k[0], w.iters[0]
    G = dlm.Graph.from_csr(g)
    col, _ = dlm.init_population(G, k, w.pop, seed=w.init_seed)
    starts = col.cpu().numpy()
    say("wave8 gnp500 full size: 8192 x 100000")
    r = dlm.tabu_batch(G, col, k, T, w.tabu_seed, table="wave8")
    torch.cuda.synchronize()
    ids = np.arange(0, w.pop, w.extra["sample_stride"])
    ref = oracle.tabucol_batch(g, starts[ids], ids, k, T, seed=w.tabu_seed)
    gpu = {kk: v.cpu().numpy()[ids] for kk, v in r.items() if isinstance(v, torch.Tensor)}
    gpu["hash"] = gpu["hash"].view(np.uint64)
    compare(gpu, ref, ids, "wave8 gnp500")
    fb = r["f_best"].cpu().numpy()
    conf, _ = dlm.evaluate(G, r["colors"], k)
    assert (conf.cpu().numpy() == fb).all()
    st = r["stats"].cpu().numpy()
    assert (st[:, 0] + st[:, 1] == r["iters"].cpu().numpy()).all()


def test_wave_static_entry_point(dlm, dev):
    """The allocation-free entry point runs the wave tier too."""
    g = gnp(150, 0.5, seed=3)
    k, T, pop = 16, 3000, 9
    G = dlm.Graph.from_csr(g)
    starts = oracle.init_random(g.n, k, pop, seed=2)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=5)
    col = torch.from_numpy(starts.copy()).cuda()
    out = {"f_best": torch.empty(pop, dtype=torch.int32, device="cuda"),
           "iters": torch.empty(pop, dtype=torch.int32, device="cuda"),
           "stats": torch.empty((pop, 8), dtype=torch.int64, device="cuda"),
           "hash": torch.empty(pop, dtype=torch.int64, device="cuda")}
    say("wave8 static entry point")
    r = dlm.tabu_batch_static(G, col, k, T, 5, out, table="wave8")
    torch.cuda.synchronize()
    gpu = {kk: v.cpu().numpy() for kk, v in r.items()}
    gpu["hash"] = gpu["hash"].view(np.uint64)
    compare(gpu, ref, range(pop), "wave8 static")
