"""GPU checks of the network's BF16 MFMA product dlm_gemm_bf16 (the layer
products of Section 2.3) against its definition C = A B computed on the host.

Two bars.  Small-integer operands (|a|, |b| <= 4, so every partial sum is an
integer below 2^24 and exact in FP32) must give the exact product bit for bit,
in every layout, tile and operand piece width: any misplaced index shows.
Gaussian operands must lie within the FP32 summation bound of the exact
(float64) product of the BF16 values: |C - C_exact| <= K 2^-24 sum_k |a b|
(every product of two BF16 values is exact in FP32; only the additions round).
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    return dlm


def operands(m, n, k, ak, bk, sa, sb, seed, ints, off=0):
    """Host and device operands in the requested layouts.  Returns the BF16
    device buffers (with `off` leading elements), the logical A [m][k] and
    B [k][n] as float64 (the BF16 values), and the pitches."""
    g = torch.Generator().manual_seed(seed)
    sa = sa or (k if ak else m)
    sb = sb or (k if bk else n)
    ra, rb = (m, k) if ak else (k, m), (n, k) if bk else (k, n)
    def make(rows, cols, pitch):
        if ints:
            t = torch.randint(-4, 5, (rows, pitch), generator=g).to(torch.bfloat16)
        else:
            t = torch.randn(rows, pitch, generator=g).to(torch.bfloat16)
        return t
    ta, tb = make(ra[0], ra[1], sa), make(rb[0], rb[1], sb)
    A = ta[:, :ra[1]].double().numpy()
    B = tb[:, :rb[1]].double().numpy()
    A = A if ak else A.T
    B = B.T if bk else B
    def dev(t):
        flat = torch.cat([torch.zeros(off, dtype=torch.bfloat16), t.reshape(-1)])
        return flat.cuda()
    return dev(ta), dev(tb), A, B, sa, sb


def run(dlm, da, db, m, n, k, ak, bk, sa, sb, off=0, tile=0, ldc=None, fill=None, splits=0):
    ldc = ldc or n
    out = torch.full((m, ldc), float("nan") if fill is None else fill, dtype=torch.float32, device="cuda")
    dlm.gemm_bf16(da[off:], db[off:], m, n, k, ak, bk, sa=sa, sb=sb, out=out, ldc=ldc, tile=tile, splits=splits)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def bound(A, B):
    return A.shape[1] * 2.0 ** -24 * (np.abs(A) @ np.abs(B)) + 1e-30


LAYOUTS = [(True, False), (False, False), (True, True), (False, True)]
# piece width -> M, N, K ragged against every tile and the K step of 64
SHAPES = {4: (300, 292, 100), 2: (302, 294, 102), 1: (301, 293, 101)}


@pytest.mark.parametrize("ak,bk", LAYOUTS)
@pytest.mark.parametrize("vec", [4, 2, 1])
@pytest.mark.parametrize("tile", [64, 128, 256])
def test_exact_small_integers(dlm, dev, ak, bk, vec, tile):
    """Edge tiles of the windowed kernels (their reads shifted inside the
    operand), the ragged last K step, and the clamped kernel (single-value
    pieces)."""
    m, n, k = SHAPES[vec]
    say(f"gemm exact ints ak={ak} bk={bk} shape {m}x{n}x{k} tile {tile}")
    da, db, A, B, sa, sb = operands(m, n, k, ak, bk, 0, 0, 100 + vec + 7 * tile, True)
    got = run(dlm, da, db, m, n, k, ak, bk, sa, sb, tile=tile)
    assert np.array_equal(got, A @ B)


@pytest.mark.parametrize("ak,bk", LAYOUTS)
@pytest.mark.parametrize("shape", [(40, 36, 20), (300, 292, 40), (64, 64, 64), (256, 256, 128), (257, 64, 65),
                                   (1, 300, 100), (300, 1, 100), (70, 80, 1)])
def test_exact_small_and_exact_fit(dlm, dev, ak, bk, shape):
    """Shapes below one tile or one K step (the clamped kernel), and shapes
    that fit a tile or a step exactly."""
    m, n, k = shape
    say(f"gemm exact ints small/fit ak={ak} bk={bk} shape {m}x{n}x{k}")
    da, db, A, B, sa, sb = operands(m, n, k, ak, bk, 0, 0, 300 + m + n + k, True)
    for tile in (0, 64, 128, 256):
        got = run(dlm, da, db, m, n, k, ak, bk, sa, sb, tile=tile)
        assert np.array_equal(got, A @ B), tile


@pytest.mark.parametrize("shape", [(300, 292, 104), (256, 256, 64), (520, 264, 200), (130, 300, 72), (64, 70, 1000)])
def test_exact_direct_to_lds(dlm, dev, shape):
    """Both operands K-contiguous with pitches of 8 values: the kernel that
    reads global memory straight into swizzled LDS, with windowed edge tiles,
    a window that overlaps summed k (K not a multiple of 64), and splits."""
    m, n, k = shape
    say(f"gemm exact ints direct {m}x{n}x{k}")
    da, db, A, B, sa, sb = operands(m, n, k, True, True, 0, 0, 700 + m + k, True)
    for tile in (64, 128, 256):
        for splits in (0, 1, 3):
            got = run(dlm, da, db, m, n, k, True, True, sa, sb, tile=tile, splits=splits)
            assert np.array_equal(got, A @ B), (tile, splits)


@pytest.mark.parametrize("ak,bk", LAYOUTS)
@pytest.mark.parametrize("splits", [2, 3, 5])
def test_exact_split_k(dlm, dev, ak, bk, splits):
    """K cut into chunks (the last one ragged, some shorter than a step),
    partials summed in chunk order: exact on integers, in every tile."""
    m, n, k = 300, 292, 1000
    say(f"gemm exact ints split {splits} ak={ak} bk={bk}")
    da, db, A, B, sa, sb = operands(m, n, k, ak, bk, 0, 0, 500 + splits, True)
    for tile in (64, 128, 256):
        got = run(dlm, da, db, m, n, k, ak, bk, sa, sb, tile=tile, splits=splits)
        assert np.array_equal(got, A @ B), tile


@pytest.mark.parametrize("ak,bk", LAYOUTS)
def test_gaussian_within_fp32_bound(dlm, dev, ak, bk):
    m, n, k = 333, 290, 1000
    say(f"gemm gaussian ak={ak} bk={bk} {m}x{n}x{k}")
    da, db, A, B, sa, sb = operands(m, n, k, ak, bk, 0, 0, 5, False)
    want = A @ B
    for tile in (0, 64, 128, 256):
        for splits in (0, 1, 4):
            got = run(dlm, da, db, m, n, k, ak, bk, sa, sb, tile=tile, splits=splits)
            assert np.all(np.abs(got - want) <= bound(A, B)), (tile, splits)


@pytest.mark.parametrize("off,pad", [(1, 3), (2, 6), (4, 4)])
def test_pitch_and_alignment(dlm, dev, off, pad):
    """Pitches wider than the extent and pointers offset by 1, 2 or 4 values
    (piece widths 1, 2 and 4); C written with a wider pitch leaves the
    columns past N alone."""
    m, n, k = 200, 136, 96
    for ak, bk in LAYOUTS:
        say(f"gemm pitch/alignment off={off} pad={pad} ak={ak} bk={bk}")
        sa = (k if ak else m) + pad
        sb = (k if bk else n) + pad
        da, db, A, B, sa, sb = operands(m, n, k, ak, bk, sa, sb, 9 + off, True, off=off)
        got = run(dlm, da, db, m, n, k, ak, bk, sa, sb, off=off, ldc=n + 5, fill=7.0)
        assert np.array_equal(got[:, :n], A @ B)
        assert np.all(got[:, n:] == 7.0)


def test_empty_and_repeat(dlm, dev):
    m, n, k = 70, 50, 40
    da, db, A, B, sa, sb = operands(m, n, k, True, False, 0, 0, 3, False)
    say("gemm K = 0, M = 0, repeat")
    z = run(dlm, da, db, m, n, 0, True, False, 1, n)
    assert np.all(z == 0.0)
    out = torch.full((1, n), 5.0, device="cuda")
    dlm.gemm_bf16(da, db, 0, n, k, True, False, sa=sa, sb=sb, out=out)
    assert torch.all(out == 5.0)
    a1 = run(dlm, da, db, m, n, k, True, False, sa, sb)
    a2 = run(dlm, da, db, m, n, k, True, False, sa, sb)
    assert np.array_equal(a1, a2)
    s1 = run(dlm, da, db, m, n, k, True, False, sa, sb, splits=3)
    s2 = run(dlm, da, db, m, n, k, True, False, sa, sb, splits=3)
    assert np.array_equal(s1, s2)
    with pytest.raises(dlm.DlmError):
        dlm.gemm_bf16(da, db, m, n, k, True, False, tile=96)


@pytest.mark.parametrize("form", ["rows", "rows-t", "at", "at-split", "wt"])
def test_network_shapes_sampled(dlm, dev, form):
    """The largest products of the paper-depth network for G(500, 0.5), k = 49:
    scoring chunks of 2048 colourings (100,352 class rows, 500 -> 5000) and
    training batches of 100 (4,900 rows, 5000 -> 2500); sampled rows checked
    against the float64 product within the FP32 bound."""
    g = torch.Generator().manual_seed(77)
    if form == "rows":  # Z = X Lambda: X [100352][500], Lambda [500][5000]
        M, K, N = 100352, 500, 5000
        X = torch.randn(M, K, generator=g).to(torch.bfloat16)
        W = torch.randn(K, N, generator=g).to(torch.bfloat16)
        say("gemm network rows 100352 x 5000 x 500")
        out = dlm.gemm_bf16(X.cuda(), W.cuda(), M, N, K, True, False)
        rows = np.random.default_rng(1).choice(M, 48, replace=False)
        A, B = X[rows].double().numpy(), W.double().numpy()
        got = out[torch.from_numpy(rows).cuda()].cpu().double().numpy()
    elif form == "rows-t":  # Z = X Lambda from Lambda^T at the 5000 -> 2500 layer (direct to LDS)
        M, K, N = 4900, 5000, 2500
        X = torch.randn(M, K, generator=g).to(torch.bfloat16)
        WT = torch.randn(N, K, generator=g).to(torch.bfloat16)
        say("gemm network rows from the transposed weight 4900 x 2500 x 5000")
        out = dlm.gemm_bf16(X.cuda(), WT.cuda(), M, N, K, True, True)
        rows = np.random.default_rng(5).choice(M, 48, replace=False)
        A, B = X[rows].double().numpy(), WT.double().numpy().T
        got = out[torch.from_numpy(rows).cuda()].cpu().double().numpy()
    elif form == "at":  # dLambda = X^T dZ: X [4900][5000], dZ [4900][2500]
        R, M, N = 4900, 5000, 2500
        X = torch.randn(R, M, generator=g).to(torch.bfloat16)
        D = torch.randn(R, N, generator=g).to(torch.bfloat16)
        say("gemm network at 5000 x 2500 x 4900")
        ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
        out = dlm.gemm_bf16(X.cuda(), D.cuda(), M, N, R, False, False, workspace=ws)
        rows = np.random.default_rng(2).choice(M, 48, replace=False)
        A, B = X[:, rows].double().numpy().T, D.double().numpy()
        got = out[torch.from_numpy(rows).cuda()].cpu().double().numpy()
    elif form == "at-split":  # dLambda = X^T dZ at the 1000-wide layers: split K
        R, M, N = 4900, 1000, 1000
        X = torch.randn(R, M, generator=g).to(torch.bfloat16)
        D = torch.randn(R, N, generator=g).to(torch.bfloat16)
        say("gemm network at 1000 x 1000 x 4900, split K")
        ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
        out = dlm.gemm_bf16(X.cuda(), D.cuda(), M, N, R, False, False, workspace=ws)
        rows = np.random.default_rng(4).choice(M, 48, replace=False)
        A, B = X[:, rows].double().numpy().T, D.double().numpy()
        got = out[torch.from_numpy(rows).cuda()].cpu().double().numpy()
    else:  # dX = dZ Lambda^T: dZ [4900][2500], Lambda [5000][2500]
        M, N, K = 4900, 5000, 2500
        D = torch.randn(M, K, generator=g).to(torch.bfloat16)
        W = torch.randn(N, K, generator=g).to(torch.bfloat16)
        say("gemm network wt 4900 x 5000 x 2500")
        out = dlm.gemm_bf16(D.cuda(), W.cuda(), M, N, K, True, True)
        rows = np.random.default_rng(3).choice(M, 48, replace=False)
        A, B = D[rows].double().numpy(), W.double().numpy().T
        got = out[torch.from_numpy(rows).cuda()].cpu().double().numpy()
    torch.cuda.synchronize()
    assert np.all(np.abs(got - A @ B) <= bound(A, B))
