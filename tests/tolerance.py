"""Parity tolerance measured on the oracle itself, for kernels that round the
operands of their matrix products to BF16 (relative error at most 2^-9) and
do the rest in FP32.

How far that moves a result depends on the result, so the oracle is rerun
with its operand hook set to each of three variants: every product operand
rounded to BF16, and twice every operand multiplied by an independent random
factor in [1 - 2^-9, 1 + 2^-9].  dev is the largest deviation of those runs
from the exact result; a GPU result must lie within 3 dev of the exact one
norm-wise and 6 dev element-wise, plus an FP32 floor of 1e-5 of the
result."""
import numpy as np


def to_bf16(a):
    """Round to the nearest BF16 value, ties to even (the operands' format)."""
    x = np.ascontiguousarray(a, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def jitter(seed):
    rng = np.random.default_rng(seed)
    return lambda a: np.asarray(a) * (1.0 + 2.0 ** -9 * rng.uniform(-1.0, 1.0, size=np.shape(a)))


def operand_variants():
    return [to_bf16, jitter(101), jitter(102)]


def deviation(run, exact):
    """Largest deviation from `exact` (a dict of arrays) of run(q) over the
    operand variants, per entry: (norm-wise, element-wise)."""
    dev = {nm: [0.0, 0.0] for nm in exact}
    for q in operand_variants():
        alt = run(q)
        for nm in exact:
            d = np.asarray(alt[nm], np.float64) - np.asarray(exact[nm], np.float64)
            dev[nm][0] = max(dev[nm][0], float(np.linalg.norm(d)))
            dev[nm][1] = max(dev[nm][1], float(np.abs(d).max()))
    return dev


def close(got, want, dev, what):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    d = got - want
    floor_n, floor_e = 1e-5 * np.linalg.norm(want), 1e-5 * np.abs(want).max()
    assert np.linalg.norm(d) <= 3 * dev[0] + floor_n, (what, np.linalg.norm(d), dev, np.linalg.norm(want))
    assert np.abs(d).max() <= 6 * dev[1] + floor_e, (what, np.abs(d).max(), dev, np.abs(want).max())
