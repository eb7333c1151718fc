"""Pins for the FP64 scorer reference (Section 2.3): colour-permutation
invariance, closed forms, finite-difference gradients, and agreement with
torch's CPU autograd and torch.optim.Adam (library cross-checks)."""
import numpy as np
import pytest
import torch

from oracle import scorer
from workloads.scorer_init import scorer_weights


def _params(n, seed=0, h=(16, 8, 4)):
    return {k: v.astype(np.float64) for k, v in scorer_weights(n, *h, seed=seed).items()}


def test_permutation_invariance():
    rng = np.random.default_rng(0)
    n, k = 30, 6
    P = _params(n)
    cols = rng.integers(0, k, (5, n))
    perm = rng.permutation(k)
    y1 = scorer.forward(P, cols, k)
    y2 = scorer.forward(P, perm[cols], k)
    assert np.allclose(y1, y2, rtol=0, atol=1e-12)


def test_single_class_closed_form():
    n, k = 12, 4
    P = _params(n, seed=3)
    cols = np.zeros((1, n), int)
    lr = scorer.lrelu
    full = lr(lr(P["b1"] + P["W1"].sum(axis=0)) @ P["W2"] + P["b2"])
    empty = lr(lr(P["b1"]) @ P["W2"] + P["b2"])
    z = full + (k - 1) * empty
    y = lr(z @ P["W3"] + P["b3"]) @ P["w4"] + P["b4"][0]
    assert np.isclose(scorer.forward(P, cols, k)[0], y, rtol=1e-13)


def _torch_forward(P, cols, k):
    T = {kk: torch.tensor(v, dtype=torch.float64, requires_grad=True) for kk, v in P.items()}
    X = torch.nn.functional.one_hot(torch.tensor(cols, dtype=torch.int64), k)
    X = X.permute(0, 2, 1).to(torch.float64)
    f = torch.nn.functional.leaky_relu
    h1 = f(X @ T["W1"] + T["b1"], 0.2)
    h2 = f(h1 @ T["W2"] + T["b2"], 0.2)
    h3 = f(h2.sum(1) @ T["W3"] + T["b3"], 0.2)
    return h3 @ T["w4"] + T["b4"][0], T


def test_forward_backward_vs_torch():
    rng = np.random.default_rng(1)
    n, k, B = 20, 5, 7
    P = _params(n, seed=1)
    cols = rng.integers(0, k, (B, n))
    tgt = rng.normal(size=B)
    y, cache = scorer.forward(P, cols, k, keep=True)
    loss, dy = scorer.mse(y, tgt)
    G = scorer.backward(P, cache, dy)
    ty, T = _torch_forward(P, cols, k)
    tl = ((ty - torch.tensor(tgt)) ** 2).mean()
    tl.backward()
    assert np.allclose(y, ty.detach().numpy(), rtol=1e-12)
    assert np.isclose(loss, tl.item(), rtol=1e-12)
    for kk in scorer.NAMES:
        assert np.allclose(G[kk], T[kk].grad.numpy(), rtol=1e-10, atol=1e-14), kk


def test_finite_difference_gradients():
    rng = np.random.default_rng(2)
    n, k, B = 9, 3, 4
    P = _params(n, seed=2, h=(6, 5, 3))
    cols = rng.integers(0, k, (B, n))
    tgt = rng.normal(size=B)
    y, cache = scorer.forward(P, cols, k, keep=True)
    _, dy = scorer.mse(y, tgt)
    G = scorer.backward(P, cache, dy)
    eps = 1e-6
    for kk in scorer.NAMES:
        flat = P[kk].reshape(-1)
        for j in rng.choice(flat.size, size=min(flat.size, 6), replace=False):
            old = flat[j]
            flat[j] = old + eps
            lp = scorer.mse(scorer.forward(P, cols, k), tgt)[0]
            flat[j] = old - eps
            lm = scorer.mse(scorer.forward(P, cols, k), tgt)[0]
            flat[j] = old
            num = (lp - lm) / (2 * eps)
            assert abs(num - G[kk].reshape(-1)[j]) <= 1e-6 * max(1.0, abs(num)), (kk, j)


def test_adam_vs_torch():
    rng = np.random.default_rng(4)
    n, k, B = 15, 4, 10
    P = _params(n, seed=4)
    cols = rng.integers(0, k, (3 * B, n))
    tgt = rng.normal(size=3 * B)
    Pn, _, losses = scorer.train(P, cols, tgt, k, batch=B, epochs=2, lr=1e-3)
    T = {kk: torch.tensor(v, dtype=torch.float64, requires_grad=True) for kk, v in P.items()}
    opt = torch.optim.Adam([T[kk] for kk in scorer.NAMES], lr=1e-3, betas=(0.9, 0.999),
                           eps=1e-8)
    X = torch.nn.functional.one_hot(torch.tensor(cols), k).permute(0, 2, 1).double()
    f = torch.nn.functional.leaky_relu
    tl = []
    for _ in range(2):
        for s in range(0, 3 * B, B):
            opt.zero_grad()
            h1 = f(X[s:s + B] @ T["W1"] + T["b1"], 0.2)
            h2 = f(h1 @ T["W2"] + T["b2"], 0.2)
            y = f(h2.sum(1) @ T["W3"] + T["b3"], 0.2) @ T["w4"] + T["b4"][0]
            loss = ((y - torch.tensor(tgt[s:s + B])) ** 2).mean()
            loss.backward()
            opt.step()
            tl.append(loss.item())
    assert np.allclose(losses, tl, rtol=1e-10)
    for kk in scorer.NAMES:
        assert np.allclose(Pn[kk], T[kk].detach().numpy(), rtol=1e-9, atol=1e-12), kk


@pytest.mark.parametrize("n", [50, 1000])
def test_init_shapes(n):
    W = scorer_weights(n, 256, 128, 64, seed=0)
    total = sum(v.size for v in W.values())
    assert total == n * 256 + 256 + 256 * 128 + 128 + 128 * 64 + 64 + 64 + 1
    assert all(v.dtype == np.float32 for v in W.values())


def test_operand_hook_reaches_the_layer2_products():
    """The operand hook (used to measure the GPU parity tolerance) scales
    both operands of each layer-2 product: with q = multiplication by c, the
    layer-2 pre-activation moves to b2 + c^2 (a2 - b2); given the same
    cached activations, the W2, h1 and so W1 / b1 gradients scale by c^2,
    the b2 gradient by c, and the head's gradients do not change."""
    n, k, B, c = 12, 4, 3, 1.5
    P = _params(n, seed=2)
    rng = np.random.default_rng(6)
    cols = rng.integers(0, k, (B, n))
    q = lambda a: c * np.asarray(a)  # noqa: E731
    _, c0 = scorer.forward(P, cols, k, keep=True)
    _, c1 = scorer.forward(P, cols, k, keep=True, q=q)
    assert np.allclose(c1["a2"] - P["b2"], c * c * (c0["a2"] - P["b2"]), rtol=1e-12, atol=1e-14)
    assert np.allclose(c1["a1"], c0["a1"])  # layer 1 is a gather, not hooked
    dy = rng.normal(size=B)
    g = scorer.backward(P, c0, dy)
    gq = scorer.backward(P, c0, dy, q=q)
    for nm in ("W2", "W1", "b1"):
        assert np.allclose(gq[nm], c * c * g[nm], rtol=1e-12, atol=1e-14), nm
    assert np.allclose(gq["b2"], c * g["b2"], rtol=1e-12)
    for nm in ("W3", "b3", "w4", "b4"):
        assert np.array_equal(gq[nm], g[nm]), nm
    assert np.abs(g["W2"]).max() > 1e-6 and np.abs(g["W1"]).max() > 1e-6
