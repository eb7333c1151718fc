"""GPU parity of population TabuCol (Section 2.7) against the CPU oracle:
every individual's best colouring, f_best, iteration count, counters and
trajectory fingerprint must be bit-identical, for every table storage and
workgroup size, from tiny ragged shapes up to the full 8192 x 100,000 run on
G(500, 0.5) (64 sampled individuals, the launch configuration the benchmark
times)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from small_graphs import complete, cycle, edgeless
from workloads import workload
from workloads.graphs import gnp, planted_partite

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    assert dlm.abi_version() == 2
    return dlm


def gpu_run(dlm, g, starts, k, T, seed, ind_base=0, **kw):
    G = dlm.Graph.from_csr(g)
    col = torch.from_numpy(np.ascontiguousarray(starts, np.int16)).cuda()
    r = dlm.tabu_batch(G, col, k, T, seed, ind_base=ind_base, **kw)
    torch.cuda.synchronize()
    out = {kk: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for kk, v in r.items()}
    if out.get("hash") is not None:
        out["hash"] = out["hash"].view(np.uint64)
    return out


def compare(gpu, ref, ids, label):
    for j, i in enumerate(ids):
        msg = f"{label} individual {i}"
        assert gpu["f_best"][j] == ref["f_best"][j], msg
        assert gpu["iters"][j] == ref["iters"][j], msg
        assert (gpu["stats"][j][:6] == ref["stats"][j][:6]).all(), (msg, gpu["stats"][j], ref["stats"][j])
        assert gpu["hash"][j] == ref["hash"][j], msg
        assert (gpu["colors"][j] == ref["colors"][j]).all(), msg


def test_init_random_bit_exact(dlm, dev):
    g = gnp(300, 0.3, seed=1)
    G = dlm.Graph.from_csr(g)
    say("init_random n=300 k=37 pop=129")
    col, ku = dlm.init_population(G, 37, 129, seed=99, ind_base=5)
    ref = oracle.init_random(300, 37, 129, seed=99, ind_base=5)
    assert (col.cpu().numpy() == ref).all()
    assert (ku.cpu().numpy() == 37).all()


def test_evaluate(dlm, dev):
    g = gnp(257, 0.4, seed=3).with_weights(np.random.default_rng(0).integers(1, 50, 257).astype(np.int32))
    G = dlm.Graph.from_csr(g)
    rng = np.random.default_rng(1)
    cols = rng.integers(0, 11, (33, 257)).astype(np.int16)
    say("evaluate n=257 count=33")
    conf, ws = dlm.evaluate(G, torch.from_numpy(cols).cuda(), 11, weighted=True)
    conf, ws = conf.cpu().numpy(), ws.cpu().numpy()
    for i in range(33):
        assert conf[i] == oracle.conflicts(g, cols[i])
        assert ws[i] == oracle.wscore(g.weights, 11, cols[i])


SHAPES = [  # (n, p, k, T, pop)
    (37, 0.3, 4, 800, 7),
    (150, 0.5, 16, 3000, 9),
    (200, 0.1, 5, 3000, 5),
    (120, 0.9, 40, 2000, 6),
    (300, 0.5, 33, 2500, 4),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_p%g_k%d" % s[:3])
@pytest.mark.parametrize("block", [64, 256, 1024])
def test_parity_shapes(dlm, dev, shape, block):
    n, p, k, T, pop = shape
    g = gnp(n, p, seed=n)
    starts = oracle.init_random(n, k, pop, seed=3, ind_base=11)
    ids = np.arange(11, 11 + pop)
    ref = oracle.tabucol_batch(g, starts, ids, k, T, seed=17)
    say(f"tabu n={n} p={p} k={k} T={T} pop={pop} block={block}")
    gpu = gpu_run(dlm, g, starts, k, T, 17, ind_base=11, block=block)
    compare(gpu, ref, ids, f"n{n} k{k} block{block}")


@pytest.mark.parametrize("table", ["lds16", "lds32", "global16", "split16", "split8"])
def test_parity_tables(dlm, dev, table):
    g = gnp(180, 0.5, seed=7)
    k, T, pop = 19, 20000, 6   # long enough to cross the 16-bit expiry rebase
    starts = oracle.init_random(180, k, pop, seed=5)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=8)
    say(f"tabu tables={table} n=180 k={k} T={T}")
    gpu = gpu_run(dlm, g, starts, k, T, 8, table=table, block=128)
    compare(gpu, ref, range(pop), table)


def test_trace_matches(dlm, dev):
    g = gnp(90, 0.5, seed=2)
    k, T = 11, 600
    starts = oracle.init_random(90, k, 3, seed=1)
    say("tabu trace n=90 k=11")
    gpu = gpu_run(dlm, g, starts, k, T, 4, trace_cap=T)
    for i in range(3):
        ref = oracle.tabucol(g, starts[i], k, T, seed=4, ind=i, trace_cap=T)
        it = ref["iters"]
        assert (gpu["trace"][i][:it] == ref["trace"][:it]).all()


def test_edge_cases(dlm, dev):
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
        say(f"tabu edge case {name}")
        gpu = gpu_run(dlm, g, starts, k, T, 6)
        compare(gpu, ref, range(3), name)
    # pop = 0 is a no-op
    G = dlm.Graph.from_csr(gnp(20, 0.3, seed=0))
    r = dlm.tabu_batch(G, torch.zeros((0, 20), dtype=torch.int16, device="cuda"), 3, 10, 1)
    assert r["f_best"].numel() == 0


def test_already_legal_start(dlm, dev):
    g, parts = planted_partite(120, 6, 0.6, seed=9)
    starts = np.stack([parts.astype(np.int16)] * 2)
    say("tabu legal start")
    gpu = gpu_run(dlm, g, starts, 6, 100, 3)
    assert (gpu["iters"] == 0).all() and (gpu["f_best"] == 0).all()
    assert (gpu["colors"] == starts).all()


def test_gnp100_full(dlm, dev):
    """The 64-individual G(100, 0.5), k = 18 workload, int32 gamma, in full."""
    w = workload("gnp100")
    g, k, T = w.graphs[0], w.k[0], w.iters[0]
    starts = oracle.init_random(g.n, k, w.pop, seed=w.init_seed)
    ref = oracle.tabucol_batch(g, starts, np.arange(w.pop), k, T, seed=w.tabu_seed)
    say("tabu gnp100 full, lds32")
    gpu = gpu_run(dlm, g, starts, k, T, w.tabu_seed, table="lds32")
    compare(gpu, ref, range(w.pop), "gnp100")


def test_gnp500_full_size_sampled(dlm, dev):
    """G(500, 0.5), k = 49, 8192 individuals x 100,000 iterations in one launch,
    in the benchmark's launch configuration; individuals i = 128 j are
    replayed by the oracle."""
    from bench import GNP500_BLOCK, GNP500_TABLE
    w = workload("gnp500")
    g, k, T = w.graphs[0], w.k[0], w.iters[0]
    G = dlm.Graph.from_csr(g)
    say("tabu gnp500 full size: init")
    col, _ = dlm.init_population(G, k, w.pop, seed=w.init_seed)
    starts = col.cpu().numpy()
    say("tabu gnp500 full size: 8192 x 100000")
    r = dlm.tabu_batch(G, col, k, T, w.tabu_seed, block=GNP500_BLOCK, table=GNP500_TABLE)
    torch.cuda.synchronize()
    ids = np.arange(0, w.pop, w.extra["sample_stride"])
    ref = oracle.tabucol_batch(g, starts[ids], ids, k, T, seed=w.tabu_seed)
    gpu = {kk: v.cpu().numpy()[ids] for kk, v in r.items() if isinstance(v, torch.Tensor)}
    gpu["hash"] = gpu["hash"].view(np.uint64)
    compare(gpu, ref, ids, "gnp500")
    # properties that hold for every individual
    fb = r["f_best"].cpu().numpy()
    conf, _ = dlm.evaluate(G, r["colors"], k)
    assert (conf.cpu().numpy() == fb).all()
    st = r["stats"].cpu().numpy()
    assert (st[:, 0] + st[:, 1] == r["iters"].cpu().numpy()).all()


def test_gnp500_split_table_sampled(dlm, dev):
    """The split table (gamma in LDS, tabu expiries in device memory) on the
    G(500, 0.5) shape with a reduced population and budget: same results as
    the oracle on every individual."""
    w = workload("gnp500")
    g, k = w.graphs[0], w.k[0]
    pop, T = 24, 20000
    starts = oracle.init_random(g.n, k, pop, seed=w.init_seed)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=w.tabu_seed)
    say("tabu gnp500 split16 pop=24 T=20000")
    gpu = gpu_run(dlm, g, starts, k, T, w.tabu_seed, table="split16", block=256)
    compare(gpu, ref, range(pop), "gnp500 split16")


def test_gnp500_byte_table_sampled(dlm, dev):
    """Byte gamma in LDS on the G(500, 0.5) shape: same results as the oracle."""
    w = workload("gnp500")
    g, k = w.graphs[0], w.k[0]
    pop, T = 24, 20000
    starts = oracle.init_random(g.n, k, pop, seed=w.init_seed)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=w.tabu_seed)
    say("tabu gnp500 split8 pop=24 T=20000")
    gpu = gpu_run(dlm, g, starts, k, T, w.tabu_seed, table="split8", block=256)
    compare(gpu, ref, range(pop), "gnp500 split8")


def _class_sizes_over_run(start, k, trace, iters):
    """Largest class size reached along an oracle trajectory (start included)."""
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


def test_byte_table_reruns_when_a_class_passes_255(dlm, dev):
    """k = 3 on 740 vertices: classes of about 247.  Individuals whose start
    already has a class above 255, and individuals whose class grows past 255
    during the search, are both rerun with 16-bit gamma; every result must
    equal the oracle's."""
    g = gnp(740, 0.012, seed=11)
    k, T, pop = 3, 1500, 12
    starts = oracle.init_random(g.n, k, pop, seed=21)
    ids = np.arange(pop)
    ref = oracle.tabucol_batch(g, starts, ids, k, T, seed=5)
    at_start, mid_run = 0, 0
    for i in range(pop):
        tr = oracle.tabucol(g, starts[i], k, T, seed=5, ind=i, trace_cap=T)
        worst = _class_sizes_over_run(starts[i], k, tr["trace"], tr["iters"])
        at_start += worst[0] > 255
        mid_run += worst[0] <= 255 and max(worst) > 255
    assert at_start > 0 and mid_run > 0, (at_start, mid_run)  # both paths are exercised
    say(f"tabu split8 rerun n=740 k=3 ({at_start} at start, {mid_run} mid-run)")
    gpu = gpu_run(dlm, g, starts, k, T, 5, table="split8", block=256)
    compare(gpu, ref, ids, "split8 rerun")


def test_gnp1000_k85_byte_table_and_auto(dlm, dev):
    """G(1000, 0.5), k = 85 (the memetic shape, whose 16-bit table does not fit
    LDS): the byte table and the automatic choice both equal the oracle."""
    g = gnp(1000, 0.5, seed=0)
    k, T, pop = 85, 4000, 6
    starts = oracle.init_random(g.n, k, pop, seed=3)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=9)
    for table in ("split8", "auto"):
        say(f"tabu gnp1000 k=85 {table}")
        gpu = gpu_run(dlm, g, starts, k, T, 9, table=table, block=256)
        compare(gpu, ref, range(pop), f"gnp1000 {table}")


def test_auto_table_and_block(dlm, dev):
    """Table and block both automatic on G(1000, 0.5), k = 90: the byte table
    fits one individual per CU, so 512 threads are used; results equal the
    oracle's (the choice never changes a trajectory)."""
    g = gnp(1000, 0.5, seed=0)
    k, T, pop = 90, 3000, 5
    starts = oracle.init_random(g.n, k, pop, seed=13)
    ref = oracle.tabucol_batch(g, starts, np.arange(40, 40 + pop), k, T, seed=21)
    say("tabu gnp1000 k=90 auto table, auto block")
    gpu = gpu_run(dlm, g, starts, k, T, 21, ind_base=40)
    compare(gpu, ref, range(pop), "gnp1000 auto/auto")


@pytest.mark.parametrize("block", [64, 128, 1024])
def test_many_rounds_per_lane(dlm, dev, block):
    """A perfect matching on 3000 vertices, all of colour 0, k = 2000: every
    vertex conflicts and every recolouring ties at delta -1 (millions of tied
    moves per iteration).  3000 x 500 colour quads give a 64-thread
    workgroup more rounds per lane (23,438) than 16-bit candidate numbers
    cover, so it takes the count-and-first-two scan; 128 and 1024 threads
    take the key scan with candidate numbers up to 46,876 and 5,860."""
    from workloads.graphs import from_edges
    n, k, T, pop = 3000, 2000, 30, 2
    g = from_edges(n, np.array([(2 * i, 2 * i + 1) for i in range(n // 2)], np.int64), "matching3000")
    starts = np.zeros((pop, n), np.int16)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=5)
    assert (ref["stats"][:, 4] == T).all()  # every iteration had tied moves
    say(f"tabu matching3000 k=2000 block={block} global16")
    gpu = gpu_run(dlm, g, starts, k, T, 5, table="global16", block=block)
    compare(gpu, ref, range(pop), f"matching3000 block={block}")


@pytest.mark.parametrize("num,den", [(7, 3), (5, 1), (32767, 7)])
def test_tenure_slopes(dlm, dev, num, den):
    """Other tenure slopes num/den: the quotient floor(num * f / den) is
    taken through a reciprocal of den in the kernel; trajectories must
    still equal the oracle's."""
    g = gnp(150, 0.5, seed=6)
    k, T, pop = 17, 3000, 6
    starts = oracle.init_random(g.n, k, pop, seed=8)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=12, ten_num=num, ten_den=den)
    say(f"tabu tenure {num}/{den}")
    gpu = gpu_run(dlm, g, starts, k, T, 12, ten_num=num, ten_den=den, table="split8")
    compare(gpu, ref, range(pop), f"tenure {num}/{den}")


def test_workspace_contract(dlm, dev):
    """The size query matches the call: an exact workspace runs (twice, the
    second time on a dirty buffer), a smaller or misaligned one is refused
    before any launch, and the LDS tiers need none."""
    import ctypes as C
    from paper_2109_05948_amd import _abi
    g = gnp(150, 0.5, seed=3)
    k, T, pop = 16, 3000, 9
    G = dlm.Graph.from_csr(g)
    starts = oracle.init_random(g.n, k, pop, seed=2)
    ref = oracle.tabucol_batch(g, starts, np.arange(pop), k, T, seed=5)
    kp = (k + 3) // 4 * 4
    for table, per_ind in [("split8", 2), ("split16", 2), ("global16", 4)]:
        need = dlm.tabu_workspace_bytes(G, pop, k, T, table=table, block=128)
        assert need >= pop * (g.n + 1) * kp * per_ind, table
        big = torch.full((need + 256,), 0xA5, dtype=torch.uint8, device="cuda")
        ws = big[:need]
        for rep in range(2):
            say(f"tabu workspace table={table} bytes={need} rep={rep}")
            col = torch.from_numpy(starts.copy()).cuda()
            r = dlm.tabu_batch(G, col, k, T, 5, table=table, block=128, workspace=ws)
            torch.cuda.synchronize()
            gpu = {kk: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for kk, v in r.items()}
            gpu["hash"] = gpu["hash"].view(np.uint64)
            compare(gpu, ref, range(pop), f"{table} workspace rep {rep}")
        col = torch.from_numpy(starts.copy()).cuda()
        with pytest.raises(dlm.DlmError) as e:
            dlm.tabu_batch(G, col, k, T, 5, table=table, block=128, workspace=ws[: need - 1])
        assert e.value.code == -1 and "workspace" in str(e.value)
        with pytest.raises(dlm.DlmError) as e:  # 256-byte alignment
            dlm.tabu_batch(G, col, k, T, 5, table=table, block=128, workspace=big[16:16 + need])
        assert e.value.code == -1
        # a NULL workspace with a nonzero need is refused too
        prm = _abi._tabu_params(k, T, 5, 0, 6, 10, 10, 128, table, 0)
        f = torch.empty(pop, dtype=torch.int32, device="cuda")
        rc = _abi.lib().dlm_tabu_batch(G.handle, C.byref(prm), pop, _abi._ptr(col), _abi._ptr(f), _abi._ptr(f),
                                       None, None, None, None, 0, None)
        assert rc == -1
    assert dlm.tabu_workspace_bytes(G, pop, k, T, table="lds16") == 0
    assert dlm.tabu_workspace_bytes(G, pop, k, T, table="lds32") == 0
    assert dlm.tabu_workspace_bytes(G, 0, k, T, table="split8") == 0
