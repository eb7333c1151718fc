"""GPU parity of the colour-invariant network (Section 2.3) against the FP64
oracle: evaluation forward, the batch-MSE gradient of every trainable, the
running estimates and a short Adam trajectory, on small ragged shapes; label
invariance, chunked evaluation and sampled outputs at the paper's k-COL depth
for a 500-vertex graph.

Tolerance: the kernels round the two operands of every matrix product to
BF16 (relative error at most 2^-9) and do the rest in FP32.  How much that
moves a result depends on the result: the backward pass of the
normalisation subtracts the batch mean of dY and its projection on zhat,
which cancels most of dY, so some gradients move by several per cent.  The
tolerance is therefore measured on the oracle itself: it is rerun with every
product operand rounded to BF16 and, twice, with every operand multiplied by
an independent random factor in [1 - 2^-9, 1 + 2^-9]; dev is the largest
deviation of those runs from the exact result.  The GPU result must lie
within 3 dev of the exact one norm-wise and 6 dev element-wise (plus an FP32
floor of 1e-5 of the result)."""
import sys

import numpy as np
import pytest
import torch

from oracle import invnet as ref
from tolerance import close, deviation

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    return dlm


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def params(n, widths, seed):
    """Oracle initialisation with non-trivial normalisation scale, shift and
    running estimates, so that evaluation exercises every term."""
    P = ref.init_params(n, widths, seed)
    rng = np.random.default_rng(seed + 1)
    for j in range(len(widths) - 1):
        P[f"g{j}"] = rng.uniform(0.5, 1.5, widths[j])
        P[f"m{j}"] = rng.normal(0, 0.1, widths[j])
        P[f"rm{j}"] = rng.normal(0, 0.2, widths[j])
        P[f"rv{j}"] = rng.uniform(0.3, 2.0, widths[j])
    return P


def calibrated(P, colors, k, seed):
    """Running estimates near the statistics of a batch (as after training),
    so that evaluation keeps every layer near unit scale."""
    _, cache = ref.forward(P, colors, k, train=True)
    rng = np.random.default_rng(seed)
    Q = dict(P)
    for j, (m, v) in enumerate(zip(cache["mean"], cache["var"])):
        Q[f"rm{j}"] = m + 0.05 * np.sqrt(v) * rng.normal(size=m.shape)
        Q[f"rv{j}"] = v * rng.uniform(0.8, 1.25, size=v.shape)
    return Q


def f32(P):
    """The FP32 copy the network is created from (the oracle then runs on
    exactly these values in FP64)."""
    return {k: (np.asarray(v, np.float32).astype(np.float64) if isinstance(v, np.ndarray) else v)
            for k, v in P.items()}


SMALL = [(40, 5, [48, 33, 1], 9), (130, 7, [200, 70, 70, 1], 24), (65, 3, [5, 1], 2)]


# k >= 32: evaluation takes the fused product (bias, normalisation, LReLU and
# the BF16 store applied to the accumulators); widths 136 / 264 take the
# direct-to-LDS kernel (pitches of 8 values), 70 the register one
FUSED = [(72, 33, [136, 70, 1], 12), (96, 40, [264, 136, 1], 9), (50, 35, [70, 1], 5)]


@pytest.mark.parametrize("n,k,widths,b", SMALL + FUSED)
def test_forward_eval(dlm, dev, n, k, widths, b):
    rng = np.random.default_rng(1)
    colors = rng.integers(0, k, size=(b, n)).astype(np.int16)
    P = f32(calibrated(params(n, widths, n + k), colors, k, 11))
    say(f"invnet forward n={n} k={k} widths={widths} b={b}")
    net = dlm.InvNet(n, k, widths, P, max_batch=b)
    got = net.forward(cuda(colors)).cpu().numpy()
    want, _ = ref.forward(P, colors, k, train=False)
    dv = deviation(lambda q: {"f": ref.forward(P, colors, k, train=False, q=q)[0]}, {"f": want})
    close(got, want, dv["f"], "forward")


@pytest.mark.parametrize("n,k,widths,b", SMALL)
def test_grad(dlm, dev, n, k, widths, b):
    P = f32(params(n, widths, 3 * n + k))
    rng = np.random.default_rng(2)
    colors = rng.integers(0, k, size=(b, n)).astype(np.int16)
    targets = rng.normal(0, 1, size=b).astype(np.float32)
    say(f"invnet grad n={n} k={k} widths={widths} b={b}")
    net = dlm.InvNet(n, k, widths, P, max_batch=b)
    g, loss = net.grad(cuda(colors), cuda(targets))
    g = net.unpack(g.cpu().numpy(), net.train_names)

    def run(q):
        f, cache = ref.forward(P, colors, k, train=True, q=q)
        out = ref.backward(P, cache, 2.0 * (f - targets) / b, k, q=q)
        out["loss"] = np.mean((f - targets) ** 2)
        return out

    want = run(None)
    dv = deviation(run, want)
    close(loss.cpu().numpy(), want["loss"], dv["loss"], "loss")
    scale = max(np.abs(want[nm]).max() for nm in net.train_names)
    for nm in net.train_names:
        if nm.startswith("b") and int(nm[1:]) < len(widths) - 1:
            # the true gradient is zero (the normalisation removes constant
            # shifts); what remains is the FP32 round-off of a sum over the
            # b k rows, whose worst case ((b k + 8) 2^-24 times the sum of
            # the terms' magnitudes) stays below 4e-5 of the largest gradient
            # on these shapes
            assert np.abs(g[nm]).max() <= 1e-4 * scale, nm
        else:
            # G0's true gradient is zero too (the class mean of the one-hot
            # input is 1/k everywhere); its deviation measures the noise
            close(g[nm], want[nm], dv[nm], nm)
    # neither the trainables nor the running estimates moved
    after = net.params()
    for nm in net.train_names + net.run_names:
        assert np.array_equal(after[nm], np.asarray(P[nm], np.float32)), nm


def test_train_trajectory(dlm, dev):
    """Three epochs of two batches (the second ragged): the per-step losses,
    the running variances and the direction of every weight update follow
    the oracle.  (Parameters with a zero true gradient take +-lr Adam steps
    driven by round-off on both sides; they shift the running means but
    nothing else, so those are checked after a single step instead.)"""
    n, k, widths = 60, 6, [72, 40, 1]
    P = f32(params(n, widths, 77))
    rng = np.random.default_rng(3)
    colors = rng.integers(0, k, size=(30, n)).astype(np.int16)
    targets = rng.normal(0, 1, size=30).astype(np.float32)
    say("invnet train trajectory")
    net = dlm.InvNet(n, k, widths, P, max_batch=16)
    losses = net.train(cuda(colors), cuda(targets), batch=16, epochs=3, lr=1e-3).cpu().numpy()
    got = net.params()

    def run(q):
        Q = {kk: (v.copy() if isinstance(v, np.ndarray) else v) for kk, v in P.items()}
        Q["losses"] = np.array(ref.train(Q, colors, targets.astype(np.float64), k, batch=16, epochs=3,
                                         lr=1e-3, q=q)[0])
        return Q

    Q = run(None)
    dv = deviation(run, {nm: Q[nm] for nm in ("losses", "rv0", "rv1")})
    assert losses.shape == (6,)
    close(losses, Q["losses"], dv["losses"], "losses")
    for nm in ("rv0", "rv1"):
        close(got[nm], Q[nm], dv[nm], nm)
    for nm in ("L0", "L1", "G1", "L2", "G2", "b2", "g0", "m0", "g1", "m1"):
        d_got = got[nm].astype(np.float64) - P[nm]
        d_want = Q[nm] - P[nm]
        cos = (d_got * d_want).sum() / (np.linalg.norm(d_got) * np.linalg.norm(d_want))
        assert cos > 0.9, (nm, cos)


def test_one_step_running_estimates(dlm, dev):
    """One training step moves the running mean and variance by momentum 0.1
    towards the batch statistics (the variance unbiased over b k rows)."""
    n, k, widths = 70, 8, [90, 50, 1]
    P = f32(params(n, widths, 12))
    rng = np.random.default_rng(13)
    colors = rng.integers(0, k, size=(20, n)).astype(np.int16)
    targets = rng.normal(0, 1, size=20).astype(np.float32)
    say("invnet one step running estimates")
    net = dlm.InvNet(n, k, widths, P, max_batch=20)
    net.train(cuda(colors), cuda(targets), batch=20, epochs=1)
    got = net.params()

    def run(q):
        Q = {kk: (v.copy() if isinstance(v, np.ndarray) else v) for kk, v in P.items()}
        ref.train(Q, colors, targets.astype(np.float64), k, batch=20, epochs=1, q=q)
        return Q

    Q = run(None)
    dv = deviation(run, {nm: Q[nm] for nm in net.run_names})
    for nm in net.run_names:
        close(got[nm], Q[nm], dv[nm], nm)


def test_train_learns(dlm, dev):
    """A label-invariant target (the size of the largest class) is learned:
    the loss of the last epoch is far below the first."""
    n, k, widths = 50, 5, [100, 50, 25, 1]
    P = f32(params(n, widths, 5))
    rng = np.random.default_rng(4)
    colors = rng.integers(0, k, size=(400, n)).astype(np.int16)
    for r in range(0, 400, 3):  # skewed classes, so the target varies
        colors[r, rng.random(n) < 0.4] = 0
    t = np.array([np.bincount(c, minlength=k).max() for c in colors], np.float32)
    t = (t - t.mean()) / t.std()
    say("invnet train learns")
    net = dlm.InvNet(n, k, widths, P, max_batch=100)
    losses = net.train(cuda(colors), cuda(t), batch=100, epochs=30, lr=1e-3).cpu().numpy()
    assert np.isfinite(losses).all()
    assert losses[-4:].mean() < 0.3 * losses[:4].mean(), losses


def test_chunked_forward_and_relabelling(dlm, dev):
    """Evaluation in chunks of max_batch equals one pass per chunk, and a
    relabelling of the colours leaves every output unchanged up to FP32
    summation order."""
    n, k, widths = 90, 9, [120, 60, 1]
    rng = np.random.default_rng(5)
    colors = rng.integers(0, k, size=(37, n)).astype(np.int16)
    P = f32(calibrated(params(n, widths, 8), colors, k, 14))
    perm = np.stack([rng.permutation(k)[c] for c in colors]).astype(np.int16)
    say("invnet chunked forward")
    net = dlm.InvNet(n, k, widths, P, max_batch=8)
    a = net.forward(cuda(colors)).cpu().numpy()
    b = net.forward(cuda(perm)).cpu().numpy()
    one = np.concatenate([net.forward(cuda(colors[i:i + 8])).cpu().numpy() for i in range(0, 37, 8)])
    assert np.array_equal(a, one)
    assert np.abs(a - b).max() <= 1e-4 * (np.abs(a).max() + 1)
    want, _ = ref.forward(P, colors, k, train=False)
    dv = deviation(lambda q: {"f": ref.forward(P, colors, k, train=False, q=q)[0]}, {"f": want})
    close(a, want, dv["f"], "chunked forward")


def test_colour_outside_range_gives_no_class(dlm, dev):
    """A vertex whose colour is outside [0, k) belongs to no class: the
    output equals the oracle's on the graph without that vertex."""
    n, k, widths = 40, 4, [30, 1]
    rng = np.random.default_rng(6)
    colors = rng.integers(0, k, size=(3, n)).astype(np.int16)
    P = f32(calibrated(params(n, widths, 9), rng.integers(0, k, size=(8, n)), k, 15))
    colors[1, 7] = -1
    colors[2, 0] = k
    say("invnet colour outside range")
    net = dlm.InvNet(n, k, widths, P, max_batch=4)
    got = net.forward(cuda(colors)).cpu().numpy()
    for r, v in ((1, 7), (2, 0)):
        Q = dict(P)
        Q["L0"] = np.delete(P["L0"], v, axis=0)
        Q["G0"] = np.delete(P["G0"], v, axis=0)
        c = np.delete(colors[r:r + 1], v, axis=1)
        want, _ = ref.forward(Q, c, k, train=False)
        dv = deviation(lambda q: {"f": ref.forward(Q, c, k, train=False, q=q)[0]}, {"f": want})
        close(got[r:r + 1], want, dv["f"], f"row {r}")


def test_paper_depth_sampled(dlm, dev):
    """The k-COL network of the paper for n = 500 (hidden widths 10n, 5n,
    2n x 5, n, n // 2), k = 49: 200 colourings evaluated in chunks of 100,
    four of them checked against the oracle one by one; one training batch of
    100 gives a finite loss and leaves the running estimates finite; and
    2100 colourings evaluated in the benchmark's chunks of 2048, five
    checked against the oracle."""
    n, k = 500, 49
    widths = [10 * n, 5 * n] + [2 * n] * 5 + [n, n // 2, 1]
    rng = np.random.default_rng(7)
    colors = rng.integers(0, k, size=(200, n)).astype(np.int16)
    P = f32(calibrated(params(n, widths, 10), colors[:8], k, 16))
    say("invnet paper depth n=500 k=49")
    net = dlm.InvNet(n, k, widths, P, max_batch=100)
    got = net.forward(cuda(colors)).cpu().numpy()
    idx = [0, 99, 100, 199]
    want, _ = ref.forward(P, colors[idx], k, train=False)
    dv = deviation(lambda q: {"f": ref.forward(P, colors[idx], k, train=False, q=q)[0]}, {"f": want})
    close(got[idx], want, dv["f"], "paper depth")
    t = rng.normal(0, 1, size=100).astype(np.float32)
    losses = net.train(cuda(colors[:100]), cuda(t), batch=100, epochs=1).cpu().numpy()
    assert np.isfinite(losses).all()
    after = net.params()
    assert all(np.isfinite(after[nm]).all() for nm in net.run_names)
    del net
    # the benchmark's evaluation pass: chunks of 2048 colourings (100,352 class
    # rows per product), 2100 colourings so the second chunk is ragged
    big = rng.integers(0, k, size=(2100, n)).astype(np.int16)
    big[:200] = colors
    say("invnet paper depth, chunks of 2048")
    net = dlm.InvNet(n, k, widths, P, max_batch=2048)
    got = net.forward(cuda(big)).cpu().numpy()
    idx = [0, 99, 2047, 2048, 2099]
    want, _ = ref.forward(P, big[idx], k, train=False)
    dv = deviation(lambda q: {"f": ref.forward(P, big[idx], k, train=False, q=q)[0]}, {"f": want})
    close(got[idx], want, dv["f"], "paper depth, chunks of 2048")


def test_odd_widths_repeatable(dlm, dev):
    """Odd widths (every product takes single-value operand pieces) follow the
    oracle, and a second evaluation and gradient repeat the first bit for bit
    (the products accumulate in a fixed order)."""
    n, k, widths, b = 131, 7, [201, 71, 69, 1], 24
    rng = np.random.default_rng(21)
    colors = rng.integers(0, k, size=(b, n)).astype(np.int16)
    targets = rng.normal(0, 1, size=b).astype(np.float32)
    P = f32(calibrated(params(n, widths, 22), colors, k, 23))
    say("invnet odd widths, repeated calls")
    net = dlm.InvNet(n, k, widths, P, max_batch=b)
    got = net.forward(cuda(colors)).cpu().numpy()
    assert np.array_equal(got, net.forward(cuda(colors)).cpu().numpy())
    want, _ = ref.forward(P, colors, k, train=False)
    dv = deviation(lambda q: {"f": ref.forward(P, colors, k, train=False, q=q)[0]}, {"f": want})
    close(got, want, dv["f"], "odd-width forward")
    g, _ = net.grad(cuda(colors), cuda(targets))
    g2, _ = net.grad(cuda(colors), cuda(targets))
    assert torch.equal(g, g2)
    g = net.unpack(g.cpu().numpy(), net.train_names)

    def run(q):
        f, cache = ref.forward(P, colors, k, train=True, q=q)
        return ref.backward(P, cache, 2.0 * (f - targets) / b, k, q=q)

    wg = run(None)
    dg = deviation(run, wg)
    for nm in ("L0", "G0", "L1", "G1", "L2", "G2", "L3", "G3", "g0", "m0", "g1", "m1"):
        close(g[nm], wg[nm], dg[nm], nm)


def test_edge_cases(dlm, dev):
    """Empty evaluation, zero epochs, a gradient batch of one colouring (the
    normalisation then runs over its k class rows only), and training data
    shorter than one batch."""
    n, k, widths = 50, 6, [40, 24, 1]
    P = f32(params(n, widths, 31))
    rng = np.random.default_rng(32)
    colors = rng.integers(0, k, size=(5, n)).astype(np.int16)
    targets = rng.normal(0, 1, size=5).astype(np.float32)
    say("invnet edge cases")
    net = dlm.InvNet(n, k, widths, P, max_batch=8)
    out = net.forward(cuda(colors[:0]))
    assert out.shape == (0,)
    before = net.params()
    assert net.train(cuda(colors), cuda(targets), batch=8, epochs=0).shape == (0,)
    after = net.params()
    assert all(np.array_equal(before[nm], after[nm]) for nm in before)
    # one colouring per batch
    g, loss = net.grad(cuda(colors[:1]), cuda(targets[:1]))
    g = net.unpack(g.cpu().numpy(), net.train_names)

    def run(q):
        f, cache = ref.forward(P, colors[:1], k, train=True, q=q)
        out = ref.backward(P, cache, 2.0 * (f - targets[:1]), k, q=q)
        out["loss"] = np.mean((f - targets[:1]) ** 2)
        return out

    want = run(None)
    dv = deviation(run, want)
    close(loss.cpu().numpy(), want["loss"], dv["loss"], "loss")
    for nm in ("L0", "L1", "L2", "G2", "g0", "m0", "g1", "m1"):
        close(g[nm], want[nm], dv[nm], nm)
    # with one colouring every row of a hidden layer's batch shares the class
    # mean, so the normalisation removes that path too: the hidden layers'
    # Gamma gradients are zero up to FP32 round-off (as their biases are)
    scale = max(np.abs(want[nm]).max() for nm in net.train_names)
    for nm in ("G0", "G1", "b0", "b1"):
        assert np.abs(want[nm]).max() <= 1e-12 * scale and np.abs(g[nm]).max() <= 1e-4 * scale, nm
    # five pairs with a batch of eight: one step over all five
    losses = net.train(cuda(colors), cuda(targets), batch=8, epochs=2).cpu().numpy()
    assert losses.shape == (2,) and np.isfinite(losses).all()

    def first_loss(q):  # the first step's loss: a training-mode pass over the five
        f, _ = ref.forward(P, colors, k, train=True, q=q)
        return {"loss": np.mean((f - targets) ** 2)}

    want1 = first_loss(None)
    close(losses[:1], np.array([want1["loss"]]), deviation(first_loss, want1)["loss"], "first loss")


def test_paper_depth_gradient(dlm, dev):
    """Every gradient of the paper's k-COL network for n = 500 (hidden widths
    10n, 5n, 2n x 5, n, n // 2; the layer shapes and vector widths of the
    benchmark) on a batch of four colourings at k = 49, against the oracle.
    At this depth BF16 operands move some gradients by about 10 %, which the
    measured deviation reflects."""
    n, k, b = 500, 49, 4
    widths = [10 * n, 5 * n] + [2 * n] * 5 + [n, n // 2, 1]
    P = f32(params(n, widths, 40))
    rng = np.random.default_rng(41)
    colors = rng.integers(0, k, size=(b, n)).astype(np.int16)
    targets = rng.normal(0, 1, size=b).astype(np.float32)
    say("invnet paper depth gradient n=500 k=49 b=4")
    net = dlm.InvNet(n, k, widths, P, max_batch=b)
    g, loss = net.grad(cuda(colors), cuda(targets))
    g = net.unpack(g.cpu().numpy(), net.train_names)

    def run(q):
        f, cache = ref.forward(P, colors, k, train=True, q=q)
        out = ref.backward(P, cache, 2.0 * (f - targets) / b, k, q=q)
        out["loss"] = np.mean((f - targets) ** 2)
        return out

    want = run(None)
    dv = deviation(run, want)
    close(loss.cpu().numpy(), want["loss"], dv["loss"], "loss")
    scale = max(np.abs(want[nm]).max() for nm in net.train_names)
    for nm in net.train_names:
        if nm.startswith("b") and int(nm[1:]) < len(widths) - 1:
            assert np.abs(g[nm]).max() <= 1e-4 * scale, nm  # zero up to FP32 round-off
        else:
            close(g[nm], want[nm], dv[nm], nm)
