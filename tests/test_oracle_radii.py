"""Pins of the capillary radii of Fig. 4 (section "Results and discussion"):
r_min, r_ave = A / L and the hydraulic radius r_h = A / P, P the length of the
lower wall's profile, on hand-built solid masks whose values follow by
counting; and the effective radius from Eq. (1) on synthetic fronts."""

import math

import numpy as np
import pytest

from paper_1309_6726_amd import inputs, radii


def _obs(oracle_mod, solid, cap, **kw):
    ny, nx = solid.shape
    p = inputs.Params(nx=nx, ny=ny, x_in=cap.x_in, x_out=cap.x_out, y0=cap.y0, W=cap.W, **kw)
    r = np.where(solid, 0.0, 1.0)
    return oracle_mod.Oracle(p, solid, r, np.where(solid, 0.0, 0.05)).observe()


def test_straight_slit_all_radii_equal_width(oracle_mod):
    cap = inputs.capillary(96, 24, 14)
    o = _obs(oracle_mod, cap.solid, cap)
    assert o["r_min"] == o["r_ave"] == o["r_h"] == 14.0


def test_lower_bump_counts_area_and_two_steps(oracle_mod):
    """A block of height b over c columns on the lower wall removes b c nodes
    from the area and adds two vertical steps of b to the lower profile."""
    cap = inputs.capillary(96, 24, 14)
    s = cap.solid.copy()
    b, c0, c1 = 3, cap.x_in + 10, cap.x_in + 17
    s[cap.y0:cap.y0 + b, c0:c1] = 1
    L = cap.x_out - cap.x_in
    A = 14 * L - b * (c1 - c0)
    o = _obs(oracle_mod, s, cap)
    assert o["r_min"] == 14 - b
    assert o["r_ave"] == pytest.approx(A / L, rel=1e-15)
    assert o["r_h"] == pytest.approx(A / (L + 2 * b), rel=1e-15)


def test_upper_growth_does_not_lengthen_lower_profile(oracle_mod):
    cap = inputs.capillary(96, 24, 14)
    s = cap.solid.copy()
    s[cap.y0 + 14 - 4:cap.y0 + 14, cap.x_in + 5:cap.x_in + 9] = 1
    L = cap.x_out - cap.x_in
    o = _obs(oracle_mod, s, cap)
    assert o["r_min"] == 10
    assert o["r_h"] == pytest.approx((14 * L - 16) / L, rel=1e-15)


def test_staircase_and_closed_column(oracle_mod):
    """Lower wall grown 1, 2, 3 nodes over three consecutive columns, then one
    fully closed column: steps 1 + 1 + 1 + 3 up to the closed column (height
    W = 14, w = 0) and 14 back down."""
    cap = inputs.capillary(96, 24, 14)
    s = cap.solid.copy()
    x = cap.x_in + 20
    for k in range(3):
        s[cap.y0:cap.y0 + k + 1, x + k] = 1
    s[cap.y0:cap.y0 + 14, x + 3] = 1
    L = cap.x_out - cap.x_in
    A = 14 * L - (1 + 2 + 3) - 14
    P = L + 1 + 1 + 1 + (14 - 3) + 14
    o = _obs(oracle_mod, s, cap)
    assert o["r_min"] == 0
    assert o["r_ave"] == pytest.approx(A / L, rel=1e-15)
    assert o["r_h"] == pytest.approx(A / P, rel=1e-15)


def test_no_capillary_gives_nan(oracle_mod):
    solid = np.zeros((16, 16), np.uint8)
    p = inputs.Params(nx=16, ny=16)
    o = oracle_mod.Oracle(p, solid, np.ones((16, 16)), np.zeros((16, 16))).observe()
    assert math.isnan(o["r_min"]) and math.isnan(o["r_h"])


def test_effective_radius_from_least_squares_velocity():
    """Eq. (1) at long times: z = v (t - t_d), v = gamma H cos(theta) / (6 mu L).
    The no-reaction run fixes cos(theta); a run with velocity v' then has
    r_eff = H v' / v, the same H when v' = v, whatever gamma, mu and L."""
    t = np.arange(0, 10001, 500, dtype=float)
    H, L, gamma, mu, cos_t = 20.0, 500.0, 0.076, 0.177, math.cos(math.radians(30))
    v0 = gamma * H * cos_t / (6 * mu * L)
    z0 = v0 * (t - 300.0)
    assert radii.velocity(t, z0) == pytest.approx(v0, rel=1e-12)
    ct = radii.cos_theta(radii.velocity(t, z0), H, L, gamma, mu)
    assert ct == pytest.approx(cos_t, rel=1e-12)
    z1 = 0.6 * v0 * t + 3.0
    assert radii.r_eff(t, z1, L, gamma, mu, ct) == pytest.approx(0.6 * H, rel=1e-12)
    assert radii.r_eff(t, z0, L, gamma, mu, ct) == pytest.approx(H, rel=1e-12)
    # noise-free fronts on a window only
    assert radii.velocity(t, z1, t_min=2000) == pytest.approx(0.6 * v0, rel=1e-12)
