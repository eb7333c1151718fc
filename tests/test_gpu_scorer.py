"""GPU parity of the offspring scorer (Section 2.3): BF16-MFMA inference
within 1e-2 relative of the FP64 oracle; every gradient element, and the
losses and weights of a multi-step Adam training run, against the FP64
oracle within a tolerance measured on the oracle with BF16-rounded and
jittered product operands (tests/tolerance.py); the Adam step against the
FP64 rule; determinism, permutation invariance, and a loss that falls when
trained."""
import sys

import numpy as np
import pytest
import torch

from oracle import scorer as ref
from tolerance import close, deviation
from workloads.scorer_init import scorer_weights

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dlm():
    import paper_2109_05948_amd as dlm
    return dlm


def rel_ok(got, want, tol=1e-2):
    return np.abs(got - want) <= tol * np.maximum(np.abs(want), 1.0)


def colorings(rng, count, n, k, empty=0):
    c = rng.integers(0, k - empty, (count, n)).astype(np.int16)
    return c


@pytest.mark.parametrize("n,k,count", [(1000, 85, 48), (300, 40, 33), (77, 5, 9), (500, 33, 20)])
def test_forward_parity(dlm, dev, n, k, count):
    W = scorer_weights(n, seed=n)
    rng = np.random.default_rng(k)
    cols = colorings(rng, count, n, k, empty=2)   # two empty classes exercise the b1 path
    sc = dlm.Scorer(n, k, W, max_batch=64)
    say(f"scorer forward n={n} k={k} count={count}")
    y = sc.score(torch.from_numpy(cols).cuda()).cpu().numpy()
    P = {kk: v.astype(np.float64) for kk, v in W.items()}
    yr = ref.forward(P, cols, k)
    assert rel_ok(y, yr).all(), np.max(np.abs(y - yr) / np.maximum(np.abs(yr), 1))
    # deterministic, and invariant to a relabelling of the classes
    y2 = sc.score(torch.from_numpy(cols).cuda()).cpu().numpy()
    assert (y == y2).all()
    perm = rng.permutation(k).astype(np.int16)
    y3 = sc.score(torch.from_numpy(perm[cols]).cuda()).cpu().numpy()
    assert np.allclose(y3, y, rtol=1e-5, atol=1e-6)


def test_forward_full_size_sampled(dlm, dev):
    """memetic1000 shapes: 32,768 children of n = 1000, k = 85 in one call."""
    n, k, count = 1000, 85, 32768
    W = scorer_weights(n, seed=0)
    rng = np.random.default_rng(5)
    cols = colorings(rng, count, n, k)
    sc = dlm.Scorer(n, k, W, max_batch=16)
    say("scorer forward 32768 x n=1000 k=85")
    y = sc.score(torch.from_numpy(cols).cuda()).cpu().numpy()
    idx = np.arange(0, count, 1024)
    yr = ref.forward({kk: v.astype(np.float64) for kk, v in W.items()}, cols[idx], k)
    assert rel_ok(y[idx], yr).all()
    assert np.isfinite(y).all()


@pytest.mark.parametrize("n,k,B", [(300, 40, 64), (1000, 85, 32), (77, 5, 9)])
def test_gradient_parity(dlm, dev, n, k, B):
    """Every element of every gradient, and the loss: the oracle at FP32
    copies of the weights, tolerance measured with the BF16 operand hook."""
    W = scorer_weights(n, seed=1)
    rng = np.random.default_rng(2)
    cols = colorings(rng, B, n, k)
    tgt = rng.normal(size=B).astype(np.float32)
    sc = dlm.Scorer(n, k, W, max_batch=B)
    say(f"scorer grad n={n} k={k} B={B}")
    g, loss = sc.grad(torch.from_numpy(cols).cuda(), torch.from_numpy(tgt).cuda())
    G = sc.unpack(g.cpu().numpy())
    P = {kk: v.astype(np.float64) for kk, v in W.items()}

    def run(q):
        y, cache = ref.forward(P, cols, k, keep=True, q=q)
        lr_, dy = ref.mse(y, tgt.astype(np.float64))
        out = ref.backward(P, cache, dy, q=q)
        out["loss"] = lr_
        return out

    want = run(None)
    dv = deviation(run, want)
    close(loss.cpu().numpy(), want["loss"], dv["loss"], "loss")
    for nm in ref.NAMES:
        close(G[nm], want[nm], dv[nm], nm)


def test_train_trajectory(dlm, dev):
    """Four Adam steps (two epochs of two batches, the second ragged): every
    step's loss and the final weights against the oracle's train(), with the
    tolerance measured on the oracle's own trajectory under the operand
    variants."""
    n, k, B, N = 120, 9, 24, 40
    W = scorer_weights(n, seed=5)
    rng = np.random.default_rng(6)
    cols = colorings(rng, N, n, k)
    # a learnable target, so that the steps move the weights coherently
    tgt = (((cols == 0) | (cols == 1)).sum(axis=1) / n * 10 - 1).astype(np.float32)
    sc = dlm.Scorer(n, k, W, max_batch=B)
    say("scorer train trajectory")
    losses = sc.train(torch.from_numpy(cols).cuda(), torch.from_numpy(tgt).cuda(), batch=B, epochs=2,
                      lr=1e-3).cpu().numpy()
    got = sc.params()
    P0 = {kk: v.astype(np.float64) for kk, v in W.items()}

    def run(q):
        Q, _, ls = ref.train(P0, cols, tgt.astype(np.float64), k, batch=B, epochs=2, lr=1e-3, q=q)
        out = {nm: Q[nm] - P0[nm] for nm in ref.NAMES}  # the updates
        out["losses"] = np.array(ls)
        return out

    want = run(None)
    assert losses.shape == (4,) and want["losses"].shape == (4,)
    dv = deviation(run, want)
    close(losses, want["losses"], dv["losses"], "losses")
    for nm in ref.NAMES:
        d = got[nm].astype(np.float64) - P0[nm]
        close(d, want[nm], dv[nm], "update of " + nm)
        # Adam's first steps follow the gradient's sign, so single elements
        # with a noise-sized gradient may flip; the update as a whole must not
        cos = (d * want[nm]).sum() / (np.linalg.norm(d) * np.linalg.norm(want[nm]))
        assert cos > 0.98, (nm, cos)


def test_adam_step_and_training(dlm, dev):
    n, k, B = 200, 20, 64
    W = scorer_weights(n, seed=3)
    rng = np.random.default_rng(4)
    cols = colorings(rng, 4 * B, n, k)
    # a learnable target: the number of vertices in classes 0 and 1
    tgt = (((cols == 0) | (cols == 1)).sum(axis=1) / n * 10 - 1).astype(np.float32)
    sc = dlm.Scorer(n, k, W, max_batch=B)
    c0 = torch.from_numpy(cols[:B]).cuda()
    t0 = torch.from_numpy(tgt[:B]).cuda()
    say("scorer adam step")
    g, _ = sc.grad(c0, t0)
    g = g.cpu().numpy().astype(np.float64)
    sc.train(c0, t0, batch=B, epochs=1, lr=1e-3)
    P1 = sc.params()
    # the Adam rule (Kingma and Ba) applied in FP64 to the same gradient
    flat0 = np.concatenate([W[nm].reshape(-1).astype(np.float64) for nm in ref.NAMES])
    m = 0.1 * g
    v = 0.001 * g * g
    want = flat0 - 1e-3 * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    got = np.concatenate([P1[nm].reshape(-1) for nm in ref.NAMES]).astype(np.float64)
    assert np.allclose(got, want, rtol=1e-5, atol=1e-7)
    say("scorer training")
    losses = sc.train(torch.from_numpy(cols).cuda(), torch.from_numpy(tgt).cuda(), batch=B,
                      epochs=30, lr=1e-3).cpu().numpy()
    assert np.isfinite(losses).all()
    assert losses[-4:].mean() < 0.5 * losses[:4].mean()
