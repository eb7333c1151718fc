"""GPU parity of the diversity steps (Sections 2.4 to 2.6) against the
oracle: the approximate partition distance element by element (block and
triangle forms, ragged n and k from 1 to 256, relabelled and close pairs,
invalid colours, writes into a strided pool block, and sampled pairs of the
8192-colouring G(500, 0.5) shape), the spacing update and the nearest
neighbours bit for bit, and the two gathers."""
import sys

import numpy as np
import pytest
import torch

from oracle import diversity as dv

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    return dlm


def colourings(rng, rows, n, k, close_to=None, moved=0):
    """Uniform random colourings, or relabelled copies of close_to's rows with
    `moved` vertices recoloured at random."""
    if close_to is None:
        return rng.integers(0, k, size=(rows, n)).astype(np.int16)
    out = np.empty((rows, n), np.int16)
    for r in range(rows):
        src = close_to[r % close_to.shape[0]]
        out[r] = rng.permutation(k)[src]
        idx = rng.choice(n, size=moved, replace=False)
        out[r, idx] = rng.integers(0, k, size=moved)
    return out


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("k,n,na,nb", [(1, 7, 3, 5), (3, 50, 17, 9), (49, 500, 24, 21), (64, 200, 10, 33),
                                       (65, 130, 12, 11), (130, 300, 6, 7), (256, 600, 3, 4)])
def test_distance_block(dlm, dev, k, n, na, nb):
    rng = np.random.default_rng(k * 1000 + n)
    a = colourings(rng, na, n, k)
    b = np.concatenate([colourings(rng, nb // 2, n, k), colourings(rng, nb - nb // 2, n, k, close_to=a, moved=n // 20)])
    say(f"distance block k={k} n={n} {na}x{nb}")
    got = dlm.partition_distance(cuda(a), k, cuda(b)).cpu().numpy()
    torch.cuda.synchronize()
    ref = dv.distance_matrix(a, b, k)
    assert (got == ref).all(), np.argwhere(got != ref)[:5]


@pytest.mark.parametrize("k,n,m", [(2, 9, 2), (7, 100, 31), (49, 500, 20), (100, 257, 9)])
def test_distance_triangle(dlm, dev, k, n, m):
    rng = np.random.default_rng(7 * k + m)
    half = colourings(rng, m // 2 + 1, n, k)
    rows = np.concatenate([half, colourings(rng, m - half.shape[0], n, k, close_to=half, moved=3)])
    say(f"distance triangle k={k} n={n} m={m}")
    got = dlm.partition_distance(cuda(rows), k).cpu().numpy()
    ref = dv.distance_matrix(rows, rows, k)
    assert (np.diag(got) == 0).all()
    assert (got == ref).all(), np.argwhere(got != ref)[:5]


@pytest.mark.parametrize("m", [2, 33, 70])
def test_distance_upper_triangle_only(dlm, dev, m):
    rng = np.random.default_rng(40 + m)
    rows = colourings(rng, m, 90, 9)
    out = torch.full((m, m), -7, dtype=torch.int32, device="cuda")
    say(f"distance upper triangle m={m}")
    dlm.partition_distance(cuda(rows), 9, out=out, upper_only=True)
    got = out.cpu().numpy()
    ref = dv.distance_matrix(rows, rows, 9)
    iu = np.triu_indices(m, 1)
    assert (got[iu] == ref[iu]).all() and (np.diag(got) == 0).all()
    assert (got[np.tril_indices(m, -1)] == -7).all()


def test_relabelled_copies_are_zero(dlm, dev):
    rng = np.random.default_rng(11)
    a = colourings(rng, 16, 333, 40)
    b = colourings(rng, 16, 333, 40, close_to=a, moved=0)
    say("distance relabelled")
    got = dlm.partition_distance(cuda(a), 40, cuda(b)).cpu().numpy()
    assert (np.diag(got) == 0).all()


def test_invalid_colour_gives_minus_one(dlm, dev):
    rng = np.random.default_rng(12)
    a = colourings(rng, 4, 60, 5)
    b = colourings(rng, 3, 60, 5)
    a[2, 17] = 5
    b[1, 0] = -1
    say("distance invalid colours")
    got = dlm.partition_distance(cuda(a), 5, cuda(b)).cpu().numpy()
    ref = dv.distance_matrix(np.clip(a, 0, 4), np.clip(b, 0, 4), 5)
    for i in range(4):
        for j in range(3):
            assert got[i, j] == (-1 if i == 2 or j == 1 else ref[i, j])


def test_pool_blocks_in_place(dlm, dev):
    """old x new and new x new written into the blocks of one pool matrix
    through its row stride; nothing else is touched."""
    rng = np.random.default_rng(13)
    p, n, k = 9, 80, 6
    old = colourings(rng, p, n, k)
    new = colourings(rng, p, n, k, close_to=old, moved=8)
    pool = torch.full((2 * p, 2 * p), -7, dtype=torch.int32, device="cuda")
    say("distance pool blocks")
    dlm.partition_distance(cuda(old), k, cuda(new), out=pool[:p, p:])
    dlm.partition_distance(cuda(new), k, out=pool[p:, p:], upper_only=True)
    got = pool.cpu().numpy()
    assert (got[:p, p:] == dv.distance_matrix(old, new, k)).all()
    iu = np.triu_indices(p)
    assert (got[p:, p:][iu] == dv.distance_matrix(new, new, k)[iu]).all()
    assert (got[p:, p:][np.tril_indices(p, -1)] == -7).all()
    assert (got[:, :p] == -7).all()


def test_full_shape_sampled(dlm, dev):
    """8192 x 8192 pairs of G(500, 0.5)-sized colourings, k = 49 (one
    generation's old x new block at the benchmark's population): 200 pairs
    checked against the oracle."""
    rng = np.random.default_rng(14)
    p, n, k = 8192, 500, 49
    old = colourings(rng, p, n, k)
    new = colourings(rng, p, n, k, close_to=old[:64], moved=40)
    say("distance 8192 x 8192 k=49 n=500")
    got = dlm.partition_distance(cuda(old), k, cuda(new))
    torch.cuda.synchronize()
    ii = rng.integers(0, p, size=200)
    jj = rng.integers(0, p, size=200)
    ii[:20] = np.arange(20)  # pairs of close colourings
    jj[:20] = np.arange(20)
    sample = got[torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda()].cpu().numpy()
    ref = np.array([dv.approx_distance(old[i], new[j], k) for i, j in zip(ii, jj)])
    assert (sample == ref).all()
    assert sample[:20].max() <= 2 * 40  # close pairs are close


@pytest.mark.parametrize("spacing", [-1, 10, 45, 1000])
def test_spacing_update(dlm, dev, spacing):
    rng = np.random.default_rng(15 + spacing)
    na, nb, n, k = 64, 57, 100, 10
    rows = np.concatenate([colourings(rng, 40, n, k), colourings(rng, na + nb - 40, n, k,
                                                                  close_to=colourings(rng, 10, n, k), moved=5)])
    dist = dv.distance_matrix(rows, rows, k)
    f = rng.integers(0, 12, size=na + nb).astype(np.int32)
    keep = 64
    ref_pick, ref_sp = dv.spacing_update(f, dist, keep, spacing)
    say(f"spacing update spacing={spacing}")
    d = cuda(dist.astype(np.int32))
    pick, nsp = dlm.spacing_update(cuda(f[:na]), cuda(f[na:]), d, keep, spacing)
    assert pick.cpu().numpy().tolist() == ref_pick
    assert int(nsp.item()) == ref_sp


def test_spacing_update_reads_upper_triangle_only(dlm, dev):
    rng = np.random.default_rng(16)
    total, keep = 50, 20
    dist = rng.integers(0, 30, size=(total, total))
    dist = np.triu(dist, 1) + np.triu(dist, 1).T
    f = rng.integers(0, 5, size=total).astype(np.int32)
    ref = dv.spacing_update(f, dist, keep, 12)
    garbage = dist.copy()
    garbage[np.tril_indices(total)] = -5  # below and on the diagonal: never read
    say("spacing update upper triangle")
    pick, nsp = dlm.spacing_update(cuda(f[:30]), cuda(f[30:]), cuda(garbage.astype(np.int32)), keep, 12)
    assert (pick.cpu().numpy().tolist(), int(nsp.item())) == ref


@pytest.mark.parametrize("total,rate", [(1500, 0.0005), (1100, 0.004), (2048, 0.0)])
def test_spacing_update_chunks(dlm, dev, total, rate):
    """A pool of several 512-member chunks with sparse close pairs: the walk
    stops inside a chunk, needs the fill, takes nothing or takes all; the
    lower triangle holds garbage."""
    rng = np.random.default_rng(19 + total)
    close = rng.random((total, total)) < rate
    dist = np.where(close, rng.integers(0, 11, size=(total, total)), rng.integers(11, 80, size=(total, total)))
    dist = np.triu(dist, 1)
    dist = dist + dist.T
    f = rng.integers(0, 60, size=total).astype(np.int32)
    garbage = dist.astype(np.int32)
    garbage[np.tril_indices(total)] = -7
    na = total // 2 + 3
    g = cuda(garbage)
    rows = dist.tolist()
    for keep in (0, 1, 700, total - 1, total):
        ref = dv.spacing_update(f, rows, keep, 10)
        say(f"spacing update chunks total={total} keep={keep}")
        pick, nsp = dlm.spacing_update(cuda(f[:na]), cuda(f[na:]), g, keep, 10)
        assert (pick.cpu().numpy().tolist(), int(nsp.item())) == ref, keep


def test_spacing_update_empty_pool(dlm, dev):
    say("spacing update empty pool")
    e = torch.empty(0, dtype=torch.int32, device=dev)
    pick, nsp = dlm.spacing_update(e, e, torch.zeros((1, 1), dtype=torch.int32, device=dev), 0, 10)
    assert pick.numel() == 0 and int(nsp.item()) == 0


def test_nearest(dlm, dev):
    rng = np.random.default_rng(17)
    p = 150
    dist = rng.integers(0, 12, size=(p, p))  # many ties
    dist = np.triu(dist, 1) + np.triu(dist, 1).T
    say("nearest p=150")
    for K in (1, 16, p - 1):
        got = dlm.nearest(cuda(dist.astype(np.int32)), K).cpu().numpy()
        assert (got == dv.nearest(dist, K)).all(), K


def test_gathers(dlm, dev):
    rng = np.random.default_rng(18)
    total, n = 40, 33
    dist = rng.integers(0, 99, size=(total, total)).astype(np.int32)
    idx = rng.permutation(total)[:25].astype(np.int32)
    say("gather distances and pool")
    got = dlm.gather_distances(cuda(dist), cuda(idx)).cpu().numpy()
    for a in range(25):
        for b in range(25):
            lo, hi = sorted((idx[a], idx[b]))
            assert got[a, b] == (0 if a == b else dist[lo, hi])
    ra, rb = rng.integers(0, 9, size=(22, n)).astype(np.int16), rng.integers(0, 9, size=(18, n)).astype(np.int16)
    fa, fb = rng.integers(0, 50, size=22).astype(np.int32), rng.integers(0, 50, size=18).astype(np.int32)
    pick = np.array([0, 21, 22, 39, 5, 40, -1], np.int32)
    rows, fs = dlm.gather_pool(cuda(ra), cuda(fa), cuda(rb), cuda(fb), cuda(pick))
    rows, fs = rows.cpu().numpy(), fs.cpu().numpy()
    allr, allf = np.concatenate([ra, rb]), np.concatenate([fa, fb])
    for r, s in enumerate(pick):
        if 0 <= s < 40:
            assert (rows[r] == allr[s]).all() and fs[r] == allf[s]
        else:
            assert (rows[r] == -1).all() and fs[r] == -1
