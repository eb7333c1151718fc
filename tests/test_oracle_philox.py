"""Pin the oracle's Philox4x32-10 to the published known-answer vectors
(Random123 distribution, Salmon et al. SC'11) and the Lemire mapping."""
import os

import numpy as np

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox_kat.txt")


def _kat():
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        yield w[:4], w[4] | (w[5] << 32), tuple(w[6:10])


def test_known_answers():
    rows = list(_kat())
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle.philox(*ctr, key) == out


def test_uniform_mapping():
    assert oracle.uniform(0, 10) == 0
    assert oracle.uniform(0xffffffff, 10) == 9
    assert oracle.uniform(0x80000000, 10) == 5
    assert oracle.uniform(123456789, 1) == 0
    xs = [oracle.philox(i, 0, 0, 0, 7)[0] for i in range(2000)]
    us = np.array([oracle.uniform(x, 10) for x in xs])
    assert us.min() == 0 and us.max() == 9
    assert np.all(np.bincount(us, minlength=10) > 130)
