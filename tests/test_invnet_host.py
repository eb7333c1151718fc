"""Host-side pieces of the colour-invariant network: the binding's packed
order of the parameters matches the oracle's list of trainables, and the
seeded initial state has the oracle's shapes at the paper's widths
(Section 3.2)."""
import numpy as np

from oracle import invnet as ref
from paper_2109_05948_amd._abi import invnet_names
from workloads.invnet_init import col_widths, invnet_weights, wvcp_widths


def test_paper_widths():
    assert col_widths(500) == [5000, 2500, 1000, 1000, 1000, 1000, 1000, 500, 250, 1]
    assert wvcp_widths(300) == [1500, 600, 300, 150, 1]
    assert len(col_widths(7)) == 10 and col_widths(7)[-2:] == [3, 1]


def test_packed_order_matches_the_oracle():
    widths = [9, 5, 1]
    train, run = invnet_names(widths)
    P = ref.init_params(6, widths, seed=0)
    assert train == ref.trainable(P)
    assert run == ["rm0", "rv0", "rm1", "rv1"]


def test_initial_state_shapes_and_ranges():
    n, widths = 40, col_widths(40)
    W = invnet_weights(n, widths, seed=3)
    P = ref.init_params(n, widths, seed=3)
    train, run = invnet_names(widths)
    for nm in train + run:
        assert W[nm].shape == P[nm].shape, nm
        assert W[nm].dtype == np.float32
    l_in = n
    for j, l_out in enumerate(widths):
        a = 1.0 / np.sqrt(l_in)
        for nm in (f"L{j}", f"G{j}", f"b{j}"):
            assert np.abs(W[nm]).max() <= a
        if j < len(widths) - 1:
            assert (W[f"g{j}"] == 1).all() and (W[f"m{j}"] == 0).all()
            assert (W[f"rm{j}"] == 0).all() and (W[f"rv{j}"] == 1).all()
        l_in = l_out
    total = sum(W[nm].size for nm in train)
    assert total == sum(2 * a * b + b + (2 * b if j < len(widths) - 1 else 0)
                        for j, (a, b) in enumerate(zip([n] + widths[:-1], widths)))
