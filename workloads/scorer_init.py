"""Seeded initial weights for the offspring scorer (an input, like a graph).

Each weight matrix and bias is uniform on [-1/sqrt(fan_in), 1/sqrt(fan_in)]
(the usual fully connected layer initialisation), drawn from numpy's PCG64
generator.  Layout: W1 [n, H1], b1 [H1], W2 [H1, H2], b2 [H2], W3 [H2, H3],
b3 [H3], w4 [H3], b4 [1]; all float32, row-major.
"""
from __future__ import annotations

import numpy as np


def scorer_weights(n: int, h1: int = 256, h2: int = 128, h3: int = 64,
                   seed: int = 0) -> dict:
    rng = np.random.default_rng(seed)

    def u(shape, fan_in):
        b = 1.0 / np.sqrt(fan_in)
        return rng.uniform(-b, b, size=shape).astype(np.float32)

    return {
        "W1": u((n, h1), n), "b1": u((h1,), n),
        "W2": u((h1, h2), h1), "b2": u((h2,), h1),
        "W3": u((h2, h3), h2), "b3": u((h3,), h2),
        "w4": u((h3,), h3), "b4": u((1,), h3),
    }
