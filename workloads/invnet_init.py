"""Seeded initial state of the colour-invariant network (an input, like a
graph), in the packed naming of the library's binding.

Per layer j: Lambda L{j} and Gamma G{j} [l_in, l_out] and the bias b{j}
[l_out] uniform on [-1/sqrt(l_in), 1/sqrt(l_in)] (the usual fully connected
layer initialisation); for hidden layers the normalisation scale g{j} = 1,
shift m{j} = 0, running mean rm{j} = 0 and running variance rv{j} = 1.
Drawn from numpy's PCG64 generator; all float32, row-major.
"""
from __future__ import annotations

import numpy as np


def col_widths(n: int) -> list[int]:
    """Layer widths of the paper's k-COL network: hidden 10n, 5n, 2n (five
    times), n, n // 2, then the output of width 1 (Section 3.2)."""
    return [10 * n, 5 * n] + [2 * n] * 5 + [n, n // 2, 1]


def wvcp_widths(n: int) -> list[int]:
    """Layer widths of the paper's WVCP network: hidden 5n, 2n, n, n // 2,
    then the output of width 1 (Section 3.2)."""
    return [5 * n, 2 * n, n, n // 2, 1]


def invnet_weights(n: int, widths, seed: int = 0) -> dict:
    rng = np.random.default_rng(seed)
    out, l_in = {}, n
    for j, l_out in enumerate(widths):
        a = 1.0 / np.sqrt(l_in)
        out[f"L{j}"] = rng.uniform(-a, a, size=(l_in, l_out)).astype(np.float32)
        out[f"G{j}"] = rng.uniform(-a, a, size=(l_in, l_out)).astype(np.float32)
        out[f"b{j}"] = rng.uniform(-a, a, size=l_out).astype(np.float32)
        if j < len(widths) - 1:
            out[f"g{j}"] = np.ones(l_out, np.float32)
            out[f"m{j}"] = np.zeros(l_out, np.float32)
            out[f"rm{j}"] = np.zeros(l_out, np.float32)
            out[f"rv{j}"] = np.ones(l_out, np.float32)
        l_in = l_out
    return out
