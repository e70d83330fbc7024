"""Host logic of the order trainer: margin calibration and the held-out choice report."""
import pytest

torch = pytest.importorskip("torch")

from paper_1801_04070_amd import learned  # noqa: E402


def test_calibrated_margins_remove_every_miss():
    g = torch.Generator().manual_seed(0)
    # per row, errors fall by 1.5 decades per candidate from a random level: every column
    # has rows on both sides of the tolerance
    base = -12 + 10 * torch.rand(5000, 1, generator=g)
    true = base - 1.5 * torch.arange(6.0)
    noise = torch.randn(5000, 6, generator=g) * torch.tensor([0.5, 0.1, 0.1, 0.1, 0.1, 0.1])
    pred = true + noise
    m = learned.calibrate(pred, true, tols=(-10.0,))
    margins = m[-10.0]
    # the noisier first candidate needs the wider margin
    assert margins[0] > max(margins[1:])
    rep = learned.choice_report(pred, true, m)["-10.0"]
    assert rep["miss_rate"] == 0.0 and rep["worst_log10_err"] <= -10.0
    assert rep["mean_order"] >= rep["mean_best_order"]


def test_choice_report_by_hand():
    # two rows, candidates 4..16; row 0 meets -10 from order 8, row 1 from order 4
    true = torch.tensor([[-6.0, -9.0, -11.0, -12.0, -13.0, -14.0],
                         [-11.0, -12.0, -13.0, -13.0, -13.0, -13.0]])
    pred = true.clone()
    rep = learned.choice_report(pred, true, {-10.0: [0.0] * 6})["-10.0"]
    assert rep["mean_order"] == 6.0 and rep["mean_best_order"] == 6.0
    assert rep["uniform_order"] == 8 and rep["miss_rate"] == 0.0
    # a margin of 1.5 on every order pushes row 0 to 10 and row 1 to 6
    rep = learned.choice_report(pred, true, {-10.0: [1.5] * 6})["-10.0"]
    assert rep["mean_order"] == 8.0


def test_margin_lookup():
    model = learned.OrderModel([0.0], margins={-8.0: [1, 1, 1, 1, 1, 1],
                                               -12.0: [3, 2, 2, 2, 2, 2]})
    assert model.margin(-8.0) == [1, 1, 1, 1, 1, 1]
    assert model.margin(-10.0) == [3, 2, 2, 2, 2, 2]   # nearest calibrated one below
    assert model.margin(-6.0) == [1, 1, 1, 1, 1, 1]
    assert model.margin(-14.0) == [3, 2, 2, 2, 2, 2]   # none below: the tightest
