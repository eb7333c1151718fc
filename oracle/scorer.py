"""FP64 reference of the offspring scorer and its training step.

TEST INFRASTRUCTURE ONLY.

The network is the colour-permutation-invariant deep-set regressor of
Section 2.3 in the form used here: every colour class i of a colouring is
the binary vector V_i over the vertices (Section 2.3, input encoding); a
shared per-class MLP maps it to a feature vector, the class features are
summed (the invariant pooling), and a small head maps the pooled vector to
the predicted post-search score.

    a1_i = b1 + V_i W1            h1_i = LReLU(a1_i)      (n -> H1)
    a2_i = b2 + h1_i W2           h2_i = LReLU(a2_i)      (H1 -> H2)
    z    = sum_i h2_i                                    (sum pool over k)
    a3   = b3 + z W3              h3   = LReLU(a3)        (H2 -> H3)
    y    = h3 . w4 + b4

LReLU(x) = max(0.2 x, x) (Section 2.3).  Training minimises the mean
squared error with Adam (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8)
at learning rate 1e-3 (Section 2.3), one pass of consecutive mini-batches
per epoch.

The optional operand hook q (identity by default) is applied to both
operands of the layer-2 products (forward h1 W2; backward da2 W2^T and
h1^T da2) and to the da2 values summed into the b2 gradient.  It does not
change the arithmetic when absent; tests pass a rounding or jitter function
to measure how far low-precision operands move a result.
"""
from __future__ import annotations

import numpy as np

SLOPE = 0.2
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4")


def lrelu(x):
    return np.maximum(SLOPE * x, x)


def lrelu_grad(x):
    return np.where(x > 0, 1.0, SLOPE)


def one_hot(colors: np.ndarray, k: int) -> np.ndarray:
    """X[b, i, v] = 1 when vertex v has colour i in colouring b (the V_i)."""
    colors = np.asarray(colors)
    B, n = colors.shape
    X = np.zeros((B, k, n), dtype=np.float64)
    b_idx = np.repeat(np.arange(B), n)
    v_idx = np.tile(np.arange(n), B)
    X[b_idx, colors.reshape(-1).astype(np.int64), v_idx] = 1.0
    return X


def _identity(a):
    return a


def forward(P: dict, colors: np.ndarray, k: int, keep: bool = False, q=None):
    q = q or _identity
    X = one_hot(colors, k)
    a1 = X @ P["W1"] + P["b1"]
    h1 = lrelu(a1)
    a2 = q(h1) @ q(P["W2"]) + P["b2"]
    h2 = lrelu(a2)
    z = h2.sum(axis=1)
    a3 = z @ P["W3"] + P["b3"]
    h3 = lrelu(a3)
    y = h3 @ P["w4"] + P["b4"][0]
    if keep:
        return y, dict(X=X, a1=a1, h1=h1, a2=a2, h2=h2, z=z, a3=a3, h3=h3)
    return y


def backward(P: dict, cache: dict, dy: np.ndarray, q=None) -> dict:
    """Gradients of sum_b dy[b] * y[b] with respect to every parameter."""
    q = q or _identity
    g = {}
    g["b4"] = np.array([dy.sum()])
    g["w4"] = cache["h3"].T @ dy
    da3 = np.outer(dy, P["w4"]) * lrelu_grad(cache["a3"])
    g["W3"] = cache["z"].T @ da3
    g["b3"] = da3.sum(axis=0)
    dz = da3 @ P["W3"].T
    da2 = dz[:, None, :] * lrelu_grad(cache["a2"])
    g["W2"] = np.einsum("bkh,bko->ho", q(cache["h1"]), q(da2))
    g["b2"] = q(da2).sum(axis=(0, 1))
    dh1 = q(da2) @ q(P["W2"]).T
    da1 = dh1 * lrelu_grad(cache["a1"])
    g["W1"] = np.einsum("bkn,bkh->nh", cache["X"], da1)
    g["b1"] = da1.sum(axis=(0, 1))
    return g


def mse(y: np.ndarray, target: np.ndarray):
    """Mean squared error and its gradient with respect to y."""
    r = y - target
    return float(np.mean(r * r)), 2.0 * r / r.shape[0]


class Adam:
    """Adam with bias correction, as stated by Kingma and Ba (Algorithm 1)."""

    def __init__(self, P: dict, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(v) for k, v in P.items()}
        self.v = {k: np.zeros_like(v) for k, v in P.items()}
        self.t = 0

    def step(self, P: dict, G: dict):
        self.t += 1
        for k in P:
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * G[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * G[k] * G[k]
            mhat = self.m[k] / (1 - self.b1 ** self.t)
            vhat = self.v[k] / (1 - self.b2 ** self.t)
            P[k] = P[k] - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def train(P: dict, colors: np.ndarray, targets: np.ndarray, k: int, batch: int, epochs: int,
          lr: float = 1e-3, opt: Adam | None = None, q=None):
    """Epochs of consecutive mini-batches; returns (params, optimiser, losses)."""
    P = {kk: np.array(v, dtype=np.float64) for kk, v in P.items()}
    opt = opt or Adam(P, lr=lr)
    losses = []
    N = colors.shape[0]
    for _ in range(epochs):
        for s in range(0, N, batch):
            y, cache = forward(P, colors[s:s + batch], k, keep=True, q=q)
            loss, dy = mse(y, targets[s:s + batch])
            G = backward(P, cache, dy, q=q)
            opt.step(P, G)
            losses.append(loss)
    return P, opt, losses


NO_LEGAL = 0x7FFFFFFF  # a WVCP search that met no legal colouring


def wvcp_targets(f: np.ndarray):
    """Training scores of one WVCP generation (Section 2.3 trains the scorer
    on the post-search score f(S'); a search that met no legal colouring has
    none, and takes the worst legal score of its generation).  Returns None
    when no search of the generation met a legal colouring (no training)."""
    f = np.asarray(f, dtype=np.int64)
    legal = [v for v in f if v != NO_LEGAL]
    if not legal:
        return None
    worst = max(legal)
    return np.array([v if v != NO_LEGAL else worst for v in f], dtype=np.int64)
