"""Plain reference of the step between two k-COL problems of the
decreasing-k driver.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark may import this module; the product path never
does.  It shares no code with the HIP kernels.

Section 2.7 solves COL as a series of k-COL problems: once a legal
k-colouring is found, k drops by one and the search goes on.  The paper does
not say how the population moves to k - 1 colours; the reading taken here
keeps each individual's partition as far as it can: the individual's
smallest colour class (ties by smaller colour) is dissolved, each of its
vertices v takes the colour floor(w0 (k - 1) / 2^32) of the new labelling,
w0 = word 0 of Philox(seed; r, step, v, D_REDUCE) for row r, and the classes
above the dissolved one move down by one.  A row with a colour outside
[0, k) becomes all -1.
"""
from __future__ import annotations

import numpy as np

from . import philox, uniform

D_REDUCE = 0x8000000B


def reduce_colours(colors: np.ndarray, k: int, seed: int, step: int) -> np.ndarray:
    colors = np.asarray(colors)
    out = np.empty_like(colors, dtype=np.int16)
    pop, n = colors.shape
    for r in range(pop):
        row = [int(c) for c in colors[r]]
        if any(c < 0 or c >= k for c in row):
            out[r] = -1
            continue
        sizes = [0] * k
        for c in row:
            sizes[c] += 1
        gone = min(range(k), key=lambda c: (sizes[c], c))
        for v, c in enumerate(row):
            if c == gone:
                out[r, v] = uniform(philox(r, step, v, D_REDUCE, seed)[0], k - 1)
            else:
                out[r, v] = c - 1 if c > gone else c
    return out
