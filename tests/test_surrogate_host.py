"""Host-side pieces of the surrogate pipeline (no GPU): the error metric,
target encoding/decoding, the confidence gate and the out-of-range queries."""

import numpy as np

from paper_1309_6726_amd import inputs
from paper_1309_6726_amd import surrogate as S


def test_front_error_definition():
    true = np.array([[0.0, 5.0, 10.0], [0.0, 0.2, 0.5]])
    pred = true + np.array([[0.1, -0.1, 0.1], [0.2, 0.2, 0.2]])
    e = S.front_error(pred, true)
    assert np.allclose(e, [0.1 / 10.0, 0.2 / 1.0])   # travel floor of 1 lu


def test_targets_roundtrip_and_washburn_scale():
    rows = inputs.sweep_params(4, 16)
    x = inputs.surrogate_inputs(rows)
    T = 10000
    S_ = S.washburn_scale(x, T)
    assert (S_ >= 1.0).all() and (S_ <= x[:, 1] + 1.0).all()
    rng = np.random.default_rng(0)
    fronts = rng.uniform(0, 1, (16, 64)) * (x[:, 1:2] - 1)
    closure = np.where(rng.uniform(size=16) < 0.3, rng.integers(100, T, 16), -1)
    y = S.make_targets(x, fronts, closure, T)
    f, c = S.decode(x, y.astype(np.float64), T)
    assert np.allclose(f, fronts, rtol=1e-6, atol=1e-4)
    assert np.array_equal(c, closure)
    # larger width and smaller angle -> faster Washburn front, longer L -> slower
    xa = np.array([[20.0, 500, 1e-3, 30, 1], [40.0, 500, 1e-3, 30, 1], [20.0, 1000, 1e-3, 30, 1]])
    v = S.washburn_scale(xa, 100)
    assert v[1] > v[0] > v[2]


def test_gate_picks_smallest_travel_meeting_target():
    class Fixed:
        def __init__(self, y):
            self.y = y

        def predict(self, x):
            return self.y
    T = 10000
    x = np.tile([[30.0, 800.0, 1e-3, 30.0, 1.0]], (40, 1))
    Sx = S.washburn_scale(x, T)[0]
    true = np.tile(np.linspace(0, 1, 64), (40, 1)) * np.linspace(0.5, 40, 40)[:, None]
    pred = true.copy()
    pred[:10] += 0.5                     # small-travel runs carry an absolute error
    y = np.concatenate([pred / Sx, np.ones((40, 1))], axis=1)
    g = S.choose_gate(Fixed(y), x, true, T, target=0.01)
    sel = true[:, -1] >= g
    assert sel.sum() >= 10 and S.front_error(pred, true)[sel].mean() <= 0.01
    assert g > true[9, -1] * 0.5


def test_spread_gate_keeps_the_agreeing_runs():
    """Runs sorted by ensemble spread: the gate is the largest spread whose
    runs at or below it average <= target error, with a minimum coverage."""
    spread = np.array([0.01, 0.02, 0.03, 0.04, 0.5, 0.6, 0.7, 0.8])
    err = np.array([0.001, 0.002, 0.003, 0.004, 0.05, 0.06, 0.07, 0.08])
    g = S.choose_spread_gate(spread, err, target=0.005, min_frac=0.25)
    assert g == 0.04
    assert S.choose_spread_gate(spread, err, target=0.0005, min_frac=0.25) == -1.0
    # the mean error over the selected runs is what counts, not each run's
    err2 = np.array([0.009, 0.001, 0.001, 0.001, 0.05, 0.06, 0.07, 0.08])
    assert S.choose_spread_gate(spread, err2, target=0.005, min_frac=0.25) == 0.04


def test_out_of_range_rows_are_outside_the_box():
    lo, hi = inputs.surrogate_box()
    rows = S.out_of_range_rows(3, 32)
    x = inputs.surrogate_inputs(rows)
    assert not S.in_box(x, lo, hi).any()
    inside = inputs.surrogate_inputs(inputs.sweep_params(9, 100))
    assert S.in_box(inside, lo, hi).all()
