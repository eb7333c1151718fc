"""Host-side logic of the learned loop, checked on hand-made cases: the
measures of the network's prediction quality (the paper's analysis of its
network, Section 4.2: Pearson correlation and median relative error) and
the WVCP training scores of searches without a legal colouring."""
import math

import torch

from paper_2109_05948_amd.memetic import prediction_quality


def test_exact_predictions():
    actual = torch.tensor([10, 20, 30, 40], dtype=torch.int32)
    mean, sd = 25.0, math.sqrt(125.0)
    pred = (actual.double() - mean) / sd  # standardised exactly
    r, rel = prediction_quality(pred.float(), actual, mean, sd)
    assert abs(r - 1.0) < 1e-6 and rel < 1e-4


def test_relative_error_and_anticorrelation():
    actual = torch.tensor([100, 200, 300], dtype=torch.int32)
    # predictions in score units 110, 180, 300 -> errors 10 %, 10 %, 0 %: median 10 %
    mean, sd = 200.0, 100.0
    pred = torch.tensor([-0.9, -0.2, 1.0])
    r, rel = prediction_quality(pred, actual, mean, sd)
    assert abs(rel - 10.0) < 1e-4 and r > 0.9
    r2, _ = prediction_quality(-pred, actual, mean, sd)
    assert abs(r2 + r) < 1e-9


def test_individuals_without_a_score_are_left_out():
    actual = torch.tensor([10, 0x7FFFFFFF, 30, 20], dtype=torch.int32)
    pred = torch.tensor([-1.0, 50.0, 1.0, 0.0])
    r, rel = prediction_quality(pred, actual, 20.0, 10.0)
    assert abs(r - 1.0) < 1e-9 and rel < 1e-9


def test_degenerate_cases_give_nan():
    actual = torch.tensor([5, 5, 5], dtype=torch.int32)
    assert all(math.isnan(x) for x in prediction_quality(torch.tensor([0.1, 0.2, 0.3]), actual, 5.0, 1.0))
    actual = torch.tensor([1, 2, 3], dtype=torch.int32)
    assert all(math.isnan(x) for x in prediction_quality(torch.zeros(3), actual, 2.0, 1.0))
    assert all(math.isnan(x) for x in prediction_quality(torch.zeros(1), actual[:1], 2.0, 1.0))


def test_wvcp_targets_oracle():
    """The oracle's training-target rule for WVCP generations, on hand cases:
    the worst legal score replaces the searches without a legal colouring."""
    from oracle.scorer import wvcp_targets
    assert wvcp_targets([120, 0x7FFFFFFF, 90, 0x7FFFFFFF]).tolist() == [120, 120, 90, 120]
    assert wvcp_targets([7, 5]).tolist() == [7, 5]
    assert wvcp_targets([0x7FFFFFFF] * 3) is None
    assert wvcp_targets([0x7FFFFFFE, 0x7FFFFFFF]).tolist() == [0x7FFFFFFE, 0x7FFFFFFE]
