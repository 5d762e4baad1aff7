"""Pins of the reaction and solute-lattice variants of the oracle (section
"LB models": precipitation at the surface on an advection-diffusion BGK
lattice):
  * D2Q4 solute lattice: exact variance of a point source at rest;
  * saturation concentration c_eq: closed form of an isolated reacting node;
  * held source: fixed point and the interior of the held region."""

import math

import numpy as np
import pytest

from paper_1309_6726_amd import inputs


def _params(nx, ny, **kw):
    base = dict(G=0.0, G_ads1=0.0, G_ads2=0.0)
    base.update(kw)
    return inputs.Params(nx=nx, ny=ny, **base)


@pytest.mark.parametrize("tau_g", [0.65, 1.0, 1.7])
def test_d2q4_variance_exact(oracle_mod, tau_g):
    """Point source at rest, equilibrium start, D2Q4 (weights 1/4, sound
    speed^2 1/2).  Per axis with lambda = 1 - 1/tau_g the second moment a and
    the flux moment b obey a(n+1) = a(n) + 2 lambda b(n) + M/2,
    b(n+1) = lambda b(n) + M/2, whence
    var(n) = (2 tau_g - 1) n / 2 - tau_g (tau_g - 1)(1 - lambda^n)
    (D = (tau_g - 1/2)/2); no rest population ever appears."""
    nx = ny = 96
    p = _params(nx, ny, tau_g=tau_g, solute_q=4)
    c = np.zeros((ny, nx))
    x0, y0 = 47, 40
    c[y0, x0] = 1.0
    o = oracle_mod.Oracle(p, np.zeros((ny, nx), np.uint8), np.ones((ny, nx)), np.zeros((ny, nx)), c)
    lam = 1 - 1 / tau_g
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    for n in (1, 2, 5, 17, 40):
        o.step(n - o.steps)
        C = o.fields()["conc"]
        M = C.sum()
        expect = (2 * tau_g - 1) * n / 2 - tau_g * (tau_g - 1) * (1 - lam ** n)
        assert math.isclose(M, 1.0, rel_tol=1e-13)
        assert math.isclose((C * (x - x0) ** 2).sum() / M, expect, rel_tol=1e-12)
        assert math.isclose((C * (y - y0) ** 2).sum() / M, expect, rel_tol=1e-12)
    assert np.all(o.state()[1][0] == 0.0)


def test_d2q4_differs_from_d2q5(oracle_mod):
    """Same relaxation time, different lattice: the D2Q4 spreads faster
    (sound speed^2 1/2 against 1/3)."""
    nx = ny = 48
    c = np.zeros((ny, nx))
    c[24, 24] = 1.0
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    var = {}
    for q in (5, 4):
        p = _params(nx, ny, tau_g=0.8, solute_q=q)
        o = oracle_mod.Oracle(p, np.zeros((ny, nx), np.uint8), np.ones((ny, nx)), np.zeros((ny, nx)), c)
        o.step(10)
        C = o.fields()["conc"]
        var[q] = (C * (x - 24) ** 2).sum()
    assert var[4] / var[5] == pytest.approx(1.5, rel=1e-12)


@pytest.mark.parametrize("c0,c_eq", [(2.0, 0.5), (0.3, 0.5)])
def test_saturation_isolated_node_closed_form(oracle_mod, c0, c_eq):
    """One fluid node inside solid, phi = 1, n_s = 4, r = 4 k_r: above
    saturation C(n) - c_eq = (C0 - c_eq)(1 - r)^n and m(n) = C0 - C(n); below
    saturation nothing precipitates."""
    nx = ny = 8
    solid = np.ones((ny, nx), np.uint8)
    solid[3, 4] = 0
    k = 0.01
    p = _params(nx, ny, tau_g=0.65, k_r=k, threshold=10.0, c_eq=c_eq)
    o = oracle_mod.Oracle(p, solid, np.where(solid, 0.0, 1.0), np.zeros((ny, nx)),
                          np.where(solid, 0.0, c0))
    for n in range(1, 30):
        o.step(1)
        fl = o.fields()
        if c0 > c_eq:
            expect = c_eq + (c0 - c_eq) * (1 - 4 * k) ** n
        else:
            expect = c0
        assert math.isclose(fl["conc"][3, 4], expect, rel_tol=1e-14)
        assert math.isclose(fl["m"][3, 4], c0 - expect, rel_tol=1e-12, abs_tol=1e-15)


def test_held_source_interior_and_fixed_point(oracle_mod):
    """Held region x < 6 at c_hold = 0.8, no flow, empty elsewhere: nodes two
    or more columns inside the region read exactly c_hold after every step;
    the total solute grows monotonically; a field uniform at c_hold is a fixed
    point (D2Q5 and D2Q4)."""
    for q in (5, 4):
        nx, ny = 40, 6
        p = _params(nx, ny, tau_g=0.9, hold_x=6, c_hold=0.8, solute_q=q)
        one, zero = np.ones((ny, nx)), np.zeros((ny, nx))
        o = oracle_mod.Oracle(p, np.zeros((ny, nx), np.uint8), one, zero, zero)
        tot = 0.0
        for n in range(1, 40):
            o.step(1)
            C = o.fields()["conc"]
            assert np.all(C[:, 1:5] == pytest.approx(0.8, rel=1e-15)), (q, n)
            assert C.sum() > tot
            tot = C.sum()
        o2 = oracle_mod.Oracle(p, np.zeros((ny, nx), np.uint8), one, zero, 0.8 * one)
        o2.step(25)
        assert np.allclose(o2.fields()["conc"], 0.8, rtol=1e-14, atol=0)


def test_variant_parameters_are_checked(oracle_mod):
    ok = _params(8, 8, tau_g=0.7)
    assert oracle_mod.params_valid(ok)
    assert not oracle_mod.params_valid(ok.replace(c_eq=-1.0))
    assert not oracle_mod.params_valid(ok.replace(hold_x=9))
    assert not oracle_mod.params_valid(ok.replace(solute_q=3))
    assert not oracle_mod.params_valid(_params(8, 8, hold_x=2, c_hold=1.0))
