"""Pins of the colour-invariant network reference (Section 2.3) against an
independent build of the same network from torch's FP64 autograd, its
batch normalisation and its Adam: forward values in both BN modes, running
statistics, every gradient, and one training step; and the defining
property, invariance under any relabelling of the colours."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import invnet as inv


def torch_net(P, colors, k, train, running=None):
    x = torch.from_numpy(inv.one_hot(colors, k))
    b = x.shape[0]
    params = {nm: torch.tensor(P[nm], requires_grad=True) for nm in inv.trainable(P)}
    nl = len(P["widths"])
    rs = running if running is not None else {}
    for j in range(nl):
        rho = x.mean(dim=1, keepdim=True)
        z = x @ params[f"L{j}"] + rho @ params[f"G{j}"] + params[f"b{j}"]
        if j == nl - 1:
            return z[:, :, 0].mean(dim=1), params
        flat = z.reshape(b * k, -1)
        rm = rs.setdefault(f"rm{j}", torch.tensor(P[f"rm{j}"]))
        rv = rs.setdefault(f"rv{j}", torch.tensor(P[f"rv{j}"]))
        y = F.batch_norm(flat, rm, rv, params[f"g{j}"], params[f"m{j}"], training=train, momentum=0.1, eps=1e-5)
        x = F.leaky_relu(y, 0.2).reshape(b, k, -1)


@pytest.fixture
def setup():
    n, k, b = 11, 4, 7
    P = inv.init_params(n, [9, 6, 5, 1], seed=3)
    rng = np.random.default_rng(4)
    for j in range(3):  # non-trivial BN parameters and running estimates
        P[f"g{j}"] = rng.uniform(0.5, 1.5, P[f"g{j}"].shape)
        P[f"m{j}"] = rng.normal(0, 0.3, P[f"m{j}"].shape)
        P[f"rm{j}"] = rng.normal(0, 0.2, P[f"rm{j}"].shape)
        P[f"rv{j}"] = rng.uniform(0.5, 2.0, P[f"rv{j}"].shape)
    colors = rng.integers(0, k, size=(b, n))
    return P, colors, k


@pytest.mark.parametrize("train", [False, True])
def test_forward_matches_torch(setup, train):
    P, colors, k = setup
    f, _ = inv.forward(P, colors, k, train=train)
    ft, _ = torch_net(P, colors, k, train)
    assert np.allclose(f, ft.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_running_statistics_match_torch(setup):
    P, colors, k = setup
    f, cache = inv.forward(P, colors, k, train=True)
    running = {}
    torch_net(P, colors, k, True, running)
    inv.update_running(P, cache, colors.shape[0], k)
    for j in range(3):
        assert np.allclose(P[f"rm{j}"], running[f"rm{j}"].numpy(), rtol=1e-12, atol=1e-14)
        assert np.allclose(P[f"rv{j}"], running[f"rv{j}"].numpy(), rtol=1e-12, atol=1e-14)


def test_gradients_match_torch(setup):
    P, colors, k = setup
    f, cache = inv.forward(P, colors, k, train=True)
    df = np.linspace(-1.0, 2.0, f.shape[0])
    g = inv.backward(P, cache, df, k)
    ft, params = torch_net(P, colors, k, True)
    (ft * torch.from_numpy(df)).sum().backward()
    for nm in inv.trainable(P):
        assert np.allclose(g[nm], params[nm].grad.numpy(), rtol=1e-10, atol=1e-12), nm


def test_adam_step_matches_torch(setup):
    P, colors, k = setup
    targets = np.linspace(0.0, 3.0, colors.shape[0])
    Q = {kk: (v.copy() if isinstance(v, np.ndarray) else v) for kk, v in P.items()}
    inv.train(Q, colors, targets, k, batch=colors.shape[0], epochs=3, lr=1e-2)
    running = {}
    params = None
    opt = None
    tp = {nm: torch.tensor(P[nm], requires_grad=True) for nm in inv.trainable(P)}
    opt = torch.optim.Adam(tp.values(), lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(3):
        R = dict(P)
        R.update({nm: tp[nm].detach().numpy() for nm in tp})
        ft, params = torch_net(R, colors, k, True, running)
        loss = ((ft - torch.from_numpy(targets)) ** 2).mean()
        opt.zero_grad()
        loss.backward()
        for nm in tp:
            tp[nm].grad = params[nm].grad
        opt.step()
    for nm in tp:
        # G0 (its term is the same on every row) and the hidden biases shift a
        # feature by a constant that the batch normalisation removes: their
        # true gradient is 0 and rounding noise moves them by ~lr * 1e-15 / eps
        zero_grad = nm == "G0" or (nm.startswith("b") and int(nm[1:]) < len(P["widths"]) - 1)
        if zero_grad:
            assert np.abs(Q[nm] - P[nm]).max() < 1e-6 and np.abs(tp[nm].detach().numpy() - P[nm]).max() < 1e-6, nm
        else:
            assert np.allclose(Q[nm], tp[nm].detach().numpy(), rtol=1e-9, atol=1e-12), nm


@pytest.mark.parametrize("train", [False, True])
def test_invariant_under_relabelling(setup, train):
    P, colors, k = setup
    f, _ = inv.forward(P, colors, k, train=train)
    rng = np.random.default_rng(9)
    for _ in range(5):
        perm = rng.permutation(k)
        g, _ = inv.forward(P, perm[colors], k, train=train)
        assert np.allclose(f, g, rtol=1e-12, atol=1e-12)


def test_shifts_removed_by_the_normalisation(setup):
    """BN cancels any per-feature constant, so the gradients of G0 and of
    the hidden biases vanish (to rounding)."""
    P, colors, k = setup
    f, cache = inv.forward(P, colors, k, train=True)
    g = inv.backward(P, cache, np.linspace(-1.0, 2.0, f.shape[0]), k)
    assert np.abs(g["G0"]).max() < 1e-12
    for j in range(len(P["widths"]) - 1):
        assert np.abs(g[f"b{j}"]).max() < 1e-12
    assert np.abs(g["L0"]).max() > 1e-3 and np.abs(g["b3"]).max() > 1e-3


def test_first_layer_mixing_is_constant(setup):
    """Every vertex lies in exactly one class, so rho of the one-hot input
    is 1/k everywhere and the first layer's mixing term is the same for
    every colouring."""
    P, colors, k = setup
    x = inv.one_hot(colors, k)
    assert np.allclose(x.mean(axis=1), 1.0 / k)


def test_operand_hook_reaches_both_operands_of_every_product():
    """The operand hook (used to measure the parity tolerance) scales both
    operands of each product: with q = multiplication by c, a one-layer
    network's output moves to beta + c^2 (f - beta), its Lambda and Gamma
    gradients scale by c^2; in a deeper network in evaluation mode the
    first layer's products scale by c^2 as well."""
    n, k, b, c = 9, 3, 5, 1.5
    rng = np.random.default_rng(8)
    colors = rng.integers(0, k, size=(b, n))
    P = inv.init_params(n, [1], seed=9)
    q = lambda a: c * np.asarray(a)  # noqa: E731
    f, cache = inv.forward(P, colors, k, train=True)
    fq, cacheq = inv.forward(P, colors, k, train=True, q=q)
    beta = P["b0"][0]
    assert np.allclose(fq - beta, c * c * (f - beta), rtol=1e-12, atol=1e-14)
    df = rng.normal(size=b)
    g = inv.backward(P, cache, df, k)
    gq = inv.backward(P, cacheq, df, k, q=q)
    for nm in ("L0", "G0"):
        assert np.allclose(gq[nm], c * c * g[nm], rtol=1e-12, atol=1e-14), nm
    assert np.allclose(gq["b0"], g["b0"], rtol=1e-12)  # the bias is no product
    # deeper network, evaluation: the first layer's pre-normalisation values
    P2 = inv.init_params(n, [4, 1], seed=10)
    _, c0 = inv.forward(P2, colors, k, train=False)
    _, c1 = inv.forward(P2, colors, k, train=False, q=q)
    # zhat = (z + b - rm) / std with rm = 0 and rv = 1 at initialisation, so
    # zhat * std - b is the sum of the two products
    std = np.sqrt(1.0 + inv.BN_EPS)
    prod0 = c0["zhat"][0] * std - P2["b0"]
    prod1 = c1["zhat"][0] * std - P2["b0"]
    assert np.abs(prod0).max() > 1e-3
    assert np.allclose(prod1, c * c * prod0, rtol=1e-12, atol=1e-14)
