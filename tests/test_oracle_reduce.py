"""Pins of the colour-count reduction between successive k-COL problems
(Section 2.7): which class is dissolved, that every other class survives
whole under the relabelling, the closed form at k = 2, the uniformity of
the redrawn colours, and the invalid-row rule."""
import numpy as np

import oracle
from oracle import reduce as rd


def test_smallest_class_dissolved_others_kept():
    rng = np.random.default_rng(0)
    for _ in range(40):
        k = int(rng.integers(2, 12))
        row = rng.integers(0, k, size=int(rng.integers(1, 80)))
        out = rd.reduce_colours(row[None, :], k, seed=3, step=7)[0]
        sizes = np.bincount(row, minlength=k)
        gone = int(np.argmin(sizes))  # argmin takes the first minimum: smaller colour on ties
        assert out.min() >= 0 and out.max() < k - 1
        keep = row != gone
        assert (out[keep] == row[keep] - (row[keep] > gone)).all()
        for c in range(k):  # every other class is still a class of its own
            if c != gone and sizes[c]:
                assert len(set(out[row == c])) == 1


def test_two_colours_closed_form():
    row = np.array([1, 0, 1, 1, 0, 1], np.int16)  # class 0 (2 vertices) goes, one colour left
    assert rd.reduce_colours(row[None, :], 2, seed=1, step=0).tolist() == [[0, 0, 0, 0, 0, 0]]
    tie = np.array([0, 1, 1, 0], np.int16)  # equal sizes: class 0 goes, class 1 becomes 0
    assert rd.reduce_colours(tie[None, :], 2, seed=1, step=0).tolist() == [[0, 0, 0, 0]]


def test_empty_class_is_the_one_dissolved():
    row = np.array([0, 2, 2, 3, 0, 3], np.int16)  # class 1 is empty
    assert rd.reduce_colours(row[None, :], 4, seed=5, step=2).tolist() == [[0, 1, 1, 2, 0, 2]]


def test_redrawn_colours_uniform():
    k, n = 6, 6000
    row = np.concatenate([np.zeros(n, np.int16), np.repeat(np.arange(1, k), n + 1).astype(np.int16)])
    out = rd.reduce_colours(row[None, :], k, seed=11, step=4)[0]
    drawn = out[:n]  # the vertices of class 0, the smallest
    counts = np.bincount(drawn, minlength=k - 1)
    assert counts.min() > 0.9 * n / (k - 1) and counts.max() < 1.1 * n / (k - 1)
    # the draw is word 0 of the published Philox4x32-10 scaled to [0, k - 1)
    w0 = oracle.philox(0, 4, 17, rd.D_REDUCE, 11)[0]
    assert drawn[17] == (w0 * (k - 1)) >> 32


def test_invalid_row():
    rows = np.array([[0, 1, 2], [0, 3, 1]], np.int16)
    out = rd.reduce_colours(rows, 3, seed=0, step=0)
    assert (out[1] == -1).all() and out[0].max() < 2
