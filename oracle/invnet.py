"""FP64 reference of the paper's colour-invariant network and its training
step (Section 2.3).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may import this module; the product path never
does.  It shares no code with the HIP kernels.

A colouring S = (V_1 .. V_k) enters as k one-hot class vectors over the n
vertices.  Layer j maps the k x l_j class features X to k x l_{j+1}:

    Z_i = X_i Lambda + rho(X) Gamma + beta,   rho(X) = (1/k) sum_i X_i
    hidden layers:  X'_i = LReLU_0.2(BN(Z)_i)
    output layer (width 1):  f(S) = (1/k) sum_i Z_i

BN is the invariant batch normalisation: per feature, the mean and the
(biased) variance over the mini-batch and all k classes, eps = 1e-5, a
learnable scale gamma and shift mu per feature (the paper writes them as
scalars; per-feature vectors are taken here, as in the batch normalisation
it adapts), running estimates with momentum 0.1 (unbiased variance) used in
evaluation.  Training minimises the mean squared error with Adam (beta1 0.9,
beta2 0.999, eps 1e-8, learning rate 1e-3 in the paper).

Every matrix product takes its two operands through q (the identity unless
given): a test can pass a perturbation of the size of a rounding to measure
how sensitive each result is to the precision of the products' operands.
"""
from __future__ import annotations

import numpy as np

SLOPE = 0.2
BN_EPS = 1e-5
MOMENTUM = 0.1


def one_hot(colors: np.ndarray, k: int) -> np.ndarray:
    """(b, n) colours -> (b, k, n) class indicator vectors."""
    b, n = colors.shape
    x = np.zeros((b, k, n))
    for c in range(b):
        x[c, colors[c], np.arange(n)] = 1.0
    return x


def init_params(n: int, widths: list[int], seed: int) -> dict:
    """Uniform(-1/sqrt(l_in), 1/sqrt(l_in)) weights and biases, BN scale 1,
    shift 0, running mean 0 and variance 1 (layer widths: hidden..., 1)."""
    rng = np.random.default_rng(seed)
    P = {"widths": list(widths), "n": n}
    l_in = n
    for j, l_out in enumerate(widths):
        a = 1.0 / np.sqrt(l_in)
        P[f"L{j}"] = rng.uniform(-a, a, size=(l_in, l_out))
        P[f"G{j}"] = rng.uniform(-a, a, size=(l_in, l_out))
        P[f"b{j}"] = rng.uniform(-a, a, size=l_out)
        if j < len(widths) - 1:
            P[f"g{j}"] = np.ones(l_out)
            P[f"m{j}"] = np.zeros(l_out)
            P[f"rm{j}"] = np.zeros(l_out)
            P[f"rv{j}"] = np.ones(l_out)
        l_in = l_out
    return P


def trainable(P: dict) -> list[str]:
    names = []
    for j in range(len(P["widths"])):
        names += [f"L{j}", f"G{j}", f"b{j}"]
        if j < len(P["widths"]) - 1:
            names += [f"g{j}", f"m{j}"]
    return names


def _identity(a):
    return a


def forward(P: dict, colors: np.ndarray, k: int, train: bool, q=None):
    """Returns (f of shape (b,), cache).  In training mode BN uses the batch
    statistics and the cache holds what the backward pass needs; the running
    estimates are not touched here (see update_running)."""
    q = q or _identity
    x = one_hot(np.asarray(colors), k)
    b = x.shape[0]
    cache = {"x": [], "zhat": [], "std": [], "y": [], "mean": [], "var": []}
    nl = len(P["widths"])
    for j in range(nl):
        rho = x.mean(axis=1, keepdims=True)
        z = q(x) @ q(P[f"L{j}"]) + q(rho) @ q(P[f"G{j}"]) + P[f"b{j}"]
        cache["x"].append(x)
        if j == nl - 1:
            return z[:, :, 0].mean(axis=1), cache
        flat = z.reshape(b * k, -1)
        if train:
            mean = flat.mean(axis=0)
            var = flat.var(axis=0)
        else:
            mean, var = P[f"rm{j}"], P[f"rv{j}"]
        std = np.sqrt(var + BN_EPS)
        zhat = (z - mean) / std
        y = zhat * P[f"g{j}"] + P[f"m{j}"]
        cache["zhat"].append(zhat)
        cache["std"].append(std)
        cache["y"].append(y)
        cache["mean"].append(mean)
        cache["var"].append(var)
        x = np.maximum(SLOPE * y, y)
    raise AssertionError("no output layer")


def backward(P: dict, cache: dict, df: np.ndarray, k: int, q=None) -> dict:
    """Gradients of sum_c df[c] * f[c] with respect to every trainable."""
    q = q or _identity
    nl = len(P["widths"])
    grads = {}
    b = df.shape[0]
    dz = np.repeat((df / k)[:, None, None], k, axis=1)  # f = mean over classes of the last z
    for j in range(nl - 1, -1, -1):
        x = cache["x"][j]
        rho = x.mean(axis=1, keepdims=True)
        du = dz.sum(axis=1, keepdims=True)  # the rho term reaches every class row
        grads[f"L{j}"] = np.einsum("cil,cim->lm", q(x), q(dz))
        grads[f"G{j}"] = np.einsum("cil,cim->lm", q(rho), q(du))
        grads[f"b{j}"] = dz.sum(axis=(0, 1))
        if j == 0:
            break
        dx = q(dz) @ q(P[f"L{j}"]).T + (q(du) @ q(P[f"G{j}"]).T) / k
        # through LReLU and the invariant BN of layer j - 1
        y = cache["y"][j - 1]
        dy = dx * np.where(y > 0, 1.0, SLOPE)
        zhat = cache["zhat"][j - 1]
        grads[f"g{j - 1}"] = (dy * zhat).sum(axis=(0, 1))
        grads[f"m{j - 1}"] = dy.sum(axis=(0, 1))
        dzhat = dy * P[f"g{j - 1}"]
        N = b * k
        s1 = dzhat.sum(axis=(0, 1))
        s2 = (dzhat * zhat).sum(axis=(0, 1))
        dz = (N * dzhat - s1 - zhat * s2) / (N * cache["std"][j - 1])
    return grads


def update_running(P: dict, cache: dict, b: int, k: int) -> None:
    """Running estimates after a training-mode forward (momentum 0.1, the
    variance unbiased over the b k rows)."""
    N = b * k
    for j in range(len(P["widths"]) - 1):
        P[f"rm{j}"] = (1 - MOMENTUM) * P[f"rm{j}"] + MOMENTUM * cache["mean"][j]
        P[f"rv{j}"] = (1 - MOMENTUM) * P[f"rv{j}"] + MOMENTUM * cache["var"][j] * N / (N - 1)


def train(P: dict, colors: np.ndarray, targets: np.ndarray, k: int, batch: int, epochs: int,
          lr: float = 1e-3, state: dict | None = None, q=None) -> tuple[list, dict]:
    """Consecutive mini-batches, MSE loss, Adam; returns (losses, Adam state)."""
    b1, b2, eps = 0.9, 0.999, 1e-8
    st = state or {"t": 0, **{f"M_{nm}": np.zeros_like(P[nm]) for nm in trainable(P)},
                   **{f"V_{nm}": np.zeros_like(P[nm]) for nm in trainable(P)}}
    losses = []
    n_rows = colors.shape[0]
    for _ in range(epochs):
        for s in range(0, n_rows, batch):
            c = colors[s:s + batch]
            t = np.asarray(targets[s:s + batch], dtype=np.float64)
            f, cache = forward(P, c, k, train=True, q=q)
            losses.append(float(((f - t) ** 2).mean()))
            g = backward(P, cache, 2.0 * (f - t) / c.shape[0], k, q=q)
            update_running(P, cache, c.shape[0], k)
            st["t"] += 1
            for nm in trainable(P):
                st[f"M_{nm}"] = b1 * st[f"M_{nm}"] + (1 - b1) * g[nm]
                st[f"V_{nm}"] = b2 * st[f"V_{nm}"] + (1 - b2) * g[nm] ** 2
                mh = st[f"M_{nm}"] / (1 - b1 ** st["t"])
                vh = st[f"V_{nm}"] / (1 - b2 ** st["t"])
                P[nm] = P[nm] - lr * mh / (np.sqrt(vh) + eps)
    return losses, st
