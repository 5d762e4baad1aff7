"""Host-side pieces of the surrogate pipeline (no GPU): the error metric,
target encoding/decoding, the confidence gates and the out-of-range queries."""

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


def test_joint_gates_bound_mean_and_95th_percentile():
    """Twenty runs: errors grow with the spread, and the five runs of smallest
    travel carry a large error whatever their spread.  Worked by hand: with
    travel gate 6 lu the runs left are 5..19 (spread 0.05..0.19, error
    0.001..0.015 except run 17 at 0.05); the largest prefix by spread whose
    mean is <= 1% and whose 95th percentile is <= 2% is runs 5..16 (mean
    0.0065, 95th percentile 0.0114), so the gates are (6, 0.16)."""
    n = 20
    travel = np.arange(n, dtype=float) + 1.0          # 1..20 lu
    spread = np.arange(n, dtype=float) / 100.0        # 0.00..0.19
    err = np.full(n, 0.3)                              # small travel: large error
    err[5:] = (np.arange(5, n) - 4) / 1000.0           # 0.001..0.015
    err[17] = 0.05                                     # one outlier among the agreeing runs
    g_t, g_s = S.joint_gates(travel, spread, err, target=0.01, p95=0.02, min_frac=0.25)
    assert (g_t, g_s) == (6.0, 0.16)
    sel = (travel >= g_t) & (spread <= g_s)
    assert sel.sum() == 12 and err[sel].mean() <= 0.01 and np.quantile(err[sel], 0.95) <= 0.02
    # with the mean bound relaxed, the 95th percentile alone keeps the outlier out
    g_t2, g_s2 = S.joint_gates(travel, spread, err, target=1.0, p95=0.02, min_frac=0.25)
    sel2 = (travel >= g_t2) & (spread <= g_s2)
    assert (g_t2, g_s2) == (6.0, 0.16) and np.quantile(err[sel2], 0.95) <= 0.02
    # nothing qualifies: every query goes to the lattice Boltzmann model
    assert S.joint_gates(travel, spread, err, target=1e-4) == (float("inf"), -1.0)
    # equal spreads are admitted together or not at all
    sp = np.zeros(n)
    g = S.joint_gates(travel, sp, err, target=0.01, p95=0.02, min_frac=0.25)
    assert g == (float("inf"), -1.0) or ((travel >= g[0]) & (sp <= g[1])).sum() == (travel >= g[0]).sum()


def test_out_of_range_rows_are_outside_the_box():
    lo, hi = inputs.surrogate_box()
    rows = S.out_of_range_rows(3, 32)
    x = inputs.surrogate_inputs(rows)
    assert not S.in_box(x, lo, hi).any()
    inside = inputs.surrogate_inputs(inputs.sweep_params(9, 100))
    assert S.in_box(inside, lo, hi).all()
